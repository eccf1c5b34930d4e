"""Seeded synthetic inputs for the reduction workloads.

This module only draws random numbers; it holds none of the reduction's
arithmetic.  Both the GPU path's tests/benchmark and the CPU oracle's callers
use it, so the two sides always see bit-identical arrays.

The paper (Section VII) sums synthetic arrays of unspecified size and type.
The workloads here are:

* ``small``     -- fp32 U[-1,1] and int32 U[-1000,1000] (both ends
                   inclusive), 2^20 elements each.
* ``int``       -- int32 U[-1000,1000], 2^26 elements.
* ``f32``       -- fp32, 2^28 elements, either N(0,1) ("normal") or
                   magnitude 10^U(-8,8) with a random sign ("mixed").
* ``half``      -- 2^29 elements N(0,1) drawn in fp32 and rounded to
                   bf16 / fp16 (round to nearest even).
* ``segments``  -- 10,000 segments with lengths floor(exp(U(0, ln 2^20)))
                   clamped to [1, 2^20], int64 CSR offsets, fp32 N(0,1).

Every generator takes the element count (so tests can draw smaller arrays
with the same distribution) and a ``stream`` index that selects an
independent child of ``numpy.random.SeedSequence(SEED)``.
"""
from __future__ import annotations

import numpy as np

SEED = 200405371

# Child-stream indices, one per workload family.
STREAM_SMALL, STREAM_INT, STREAM_F32, STREAM_HALF, STREAM_SEGMENTS = range(5)


def rng(stream: int, sub: int = 0) -> np.random.Generator:
    """PCG64 generator for child ``stream`` of SEED, sub-stream ``sub``."""
    ss = np.random.SeedSequence(SEED).spawn(max(5, stream + 1))[stream]
    if sub:
        ss = ss.spawn(sub + 1)[sub]
    return np.random.Generator(np.random.PCG64(ss))


def uniform_f32(n: int, lo: float = -1.0, hi: float = 1.0, stream: int = STREAM_SMALL, sub: int = 0) -> np.ndarray:
    """U[lo, hi) drawn in float64, rounded to nearest float32."""
    return rng(stream, sub).uniform(lo, hi, n).astype(np.float32)


def uniform_i32(n: int, lo: int = -1000, hi: int = 1000, stream: int = STREAM_INT, sub: int = 0) -> np.ndarray:
    """Integers uniform on [lo, hi], both ends inclusive."""
    return rng(stream, sub).integers(lo, hi, n, endpoint=True, dtype=np.int32)


def normal_f32(n: int, stream: int = STREAM_F32, sub: int = 0) -> np.ndarray:
    """N(0,1) drawn directly in float32."""
    return rng(stream, sub).standard_normal(n, dtype=np.float32)


def mixed_f32(n: int, stream: int = STREAM_F32, sub: int = 1) -> np.ndarray:
    """Magnitude 10^U(-8,8) (drawn in float64) with a random sign, rounded
    to float32."""
    g = rng(stream, sub)
    mag = np.power(10.0, g.uniform(-8.0, 8.0, n))
    sign = np.where(g.integers(0, 2, n, dtype=np.int8) == 0, -1.0, 1.0)
    return (mag * sign).astype(np.float32)


def normal_half_bits(n: int, kind: str, stream: int = STREAM_HALF, sub: int = 0) -> np.ndarray:
    """N(0,1) drawn in float32 and rounded to nearest-even bf16 or fp16.

    Returns the raw 16-bit patterns as uint16 (numpy has no bfloat16)."""
    import torch  # conversion only: torch's CPU casts round to nearest even

    x = torch.from_numpy(normal_f32(n, stream=stream, sub=sub))
    if kind == "bf16":
        y = x.to(torch.bfloat16)
    elif kind == "f16":
        y = x.to(torch.float16)
    else:
        raise ValueError(kind)
    return y.view(torch.int16).numpy().view(np.uint16)


def segment_lengths(nseg: int, max_len: int = 1 << 20, stream: int = STREAM_SEGMENTS,
                    total: int | None = None) -> np.ndarray:
    """Log-uniform lengths floor(exp(U(0, ln max_len))) clamped to
    [1, max_len].  With ``total`` the same draws are scaled by
    total / sum(lengths) (floor, minimum 1)."""
    g = rng(stream, 0)
    lens = np.floor(np.exp(g.uniform(0.0, np.log(max_len), nseg))).astype(np.int64)
    lens = np.clip(lens, 1, max_len)
    if total is not None:
        lens = np.maximum(1, np.floor(lens * (total / lens.sum()))).astype(np.int64)
    return lens


def offsets_from_lengths(lens: np.ndarray) -> np.ndarray:
    """CSR offsets (int64, nseg + 1 entries, offsets[0] == 0)."""
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def segments(nseg: int = 10000, max_len: int = 1 << 20, total: int | None = None,
             stream: int = STREAM_SEGMENTS):
    """(values fp32 N(0,1), offsets int64) for a segmented batch."""
    lens = segment_lengths(nseg, max_len, stream=stream, total=total)
    off = offsets_from_lengths(lens)
    vals = normal_f32(int(off[-1]), stream=stream, sub=1)
    return vals, off
