"""CPU oracle for the device-wide sum reduction and the iterative stencil --
test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the product path never does.
"""
from .oracle import (  # noqa: F401
    ExactSum, build, exact_abs_sum, exact_sum, jacobi_1d_f32, jacobi_1d_f64, kernel_total_latency,
    launch_overhead_eq6, neumaier, per_op_latency_eq7, rel_err,
    segmented_sums, segmented_sums_i32, sigma_eq8, sum_float, sum_i32,
)
