"""MI355X-native device-wide sum reduction (arXiv 2004.05371, Section VII).

Importing the package loads nothing native; ``paper_2004_05371_amd.redsum``
loads the HIP library (and raises if it is missing).
"""
__all__ = ["inputs", "model", "redsum", "autotune"]
