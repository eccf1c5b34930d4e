"""Oracle for the device-wide sum reduction -- TEST INFRASTRUCTURE ONLY.

Plain, slow and obviously correct CPU implementation of what the reduction
hot path computes, following the reduction case study (Section VII, "Case
Study: Reduction Operator") and the measurement formulas of Sections IV and
IX of Zhang, Wahib, Zhang, Matsuoka, "A Study of Single and Multi-device
Synchronization Methods in Nvidia GPUs" (arXiv 2004.05371).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this module.  It shares no code with the HIP
library and never imports the product package.

Contents
--------
* ``sum_i32``            -- integer sum in int64 (exact by definition).
* ``exact_sum``          -- exact real-number sum of fp32 / bf16 / fp16
                            inputs via per-exponent integer bins (C code in
                            ``oracle_sum.c``), combined here with Python
                            integers and rounded once to binary64.
* ``segmented_sums``     -- the same per CSR segment.
* ``rel_err``            -- exact relative error of a double against an
                            exact sum (rational arithmetic).
* ``neumaier``           -- FP64 compensated sum, a secondary cross-check.
* ``kernel_total_latency``, ``launch_overhead_eq6``, ``per_op_latency_eq7``,
  ``sigma_eq8``          -- the probe formulas of Sections IV and IX.
* ``jacobi_1d_f32``      -- the iterative stencil whose time loop the paper
                            proposes to move inside one persistent kernel
                            (Section VII-B): explicit 1D Jacobi / heat steps
                            in binary32 with one fixed operation order.
* ``jacobi_1d_f64``      -- the same steps in binary64 (for the closed-form
                            pins).

Every function cites the passage it follows.  Pins (tests that fix this code
to something other than itself) live in ``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_sum.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile ``oracle_sum.c`` with gcc into ``liboracle.so`` (plain C, -O2,
    strict IEEE: no fast-math).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_sum_i32.restype = ctypes.c_int64
        lib.oracle_sum_i32.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        for name in ("oracle_bins_f32", "oracle_bins_bf16", "oracle_bins_f16"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, i64p, i64p]
        lib.oracle_neumaier_f64.restype = ctypes.c_double
        lib.oracle_neumaier_f64.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        _lib = lib
    return _lib


# --------------------------------------------------------------------------
# Integer sums (Section VII: "summing the elements of an array")
# --------------------------------------------------------------------------
def sum_i32(x: np.ndarray) -> int:
    """Sum of an int32 array, accumulated in int64 (exact for n <= 2^32)."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    return int(_load().oracle_sum_i32(x.ctypes.data, x.size))


# --------------------------------------------------------------------------
# Exact floating-point sums
# --------------------------------------------------------------------------
# Scale of the lowest bin: value = N * 2^-SHIFT for an integer N.
_F32_SHIFT = 149   # fp32/bf16: significand * 2^(max(E,1)-150), min exponent -149
_F16_SHIFT = 24    # fp16: significand * 2^(max(E,1)-25), min exponent -24


@dataclass(frozen=True)
class ExactSum:
    """Exact sum S* = num * 2^-shift, plus NaN/inf counts."""
    num: int
    shift: int
    n_nan: int = 0
    n_pinf: int = 0
    n_ninf: int = 0

    @property
    def fraction(self) -> Fraction:
        if not self.finite:
            raise ValueError("sum is not finite")
        return Fraction(self.num, 1 << self.shift)

    @property
    def finite(self) -> bool:
        return self.n_nan == 0 and self.n_pinf == 0 and self.n_ninf == 0

    @property
    def value(self) -> float:
        """S* rounded once to binary64 (round-to-nearest-even).

        CPython's int / int true division is correctly rounded, so this is
        the correctly rounded value of the exact rational sum."""
        if self.n_nan or (self.n_pinf and self.n_ninf):
            return math.nan
        if self.n_pinf:
            return math.inf
        if self.n_ninf:
            return -math.inf
        return self.num / (1 << self.shift)


def _as_bits(x: np.ndarray, kind: str) -> np.ndarray:
    if kind == "f32":
        if x.dtype == np.float32:
            return np.ascontiguousarray(x).view(np.uint32)
        if x.dtype in (np.uint32, np.int32):
            return np.ascontiguousarray(x).view(np.uint32)
    elif kind == "f16":
        if x.dtype == np.float16:
            return np.ascontiguousarray(x).view(np.uint16)
        if x.dtype in (np.uint16, np.int16):
            return np.ascontiguousarray(x).view(np.uint16)
    elif kind == "bf16":
        # numpy has no bfloat16: bf16 arrays are passed as raw uint16/int16 bits
        if x.dtype in (np.uint16, np.int16):
            return np.ascontiguousarray(x).view(np.uint16)
    raise TypeError("unsupported array dtype %s for kind %s" % (x.dtype, kind))


def _bins(bits: np.ndarray, kind: str):
    lib = _load()
    nb = 32 if kind == "f16" else 256
    bins = (ctypes.c_int64 * 256)()
    special = (ctypes.c_int64 * 3)()
    fn = {"f32": lib.oracle_bins_f32, "bf16": lib.oracle_bins_bf16,
          "f16": lib.oracle_bins_f16}[kind]
    fn(bits.ctypes.data if bits.size else None, bits.size, bins, special)
    return [bins[e] for e in range(nb)], (special[0], special[1], special[2])


def _combine(bins: Sequence[int], special, kind: str) -> ExactSum:
    # bin E holds integer significands of weight 2^(max(E,1) - bias_shift);
    # relative to the lowest weight 2^-SHIFT that is a left shift of max(E,1)-1.
    shift = _F16_SHIFT if kind == "f16" else _F32_SHIFT
    num = 0
    for e, b in enumerate(bins):
        if b:
            num += b << (max(e, 1) - 1)
    return ExactSum(num, shift, *special)


def exact_sum(x: np.ndarray, kind: str) -> ExactSum:
    """Exact real sum of the values of an fp32 / bf16 / fp16 array.

    ``kind`` is "f32", "bf16" or "f16"; bf16 data is given as raw 16-bit
    patterns (uint16/int16), fp16 as float16 or raw bits."""
    bits = _as_bits(x, kind)
    bins, special = _bins(bits, kind)
    return _combine(bins, special, kind)


def exact_abs_sum(x: np.ndarray, kind: str) -> ExactSum:
    """Exact sum of |x_i| (sign bits cleared), used to scale errors when the
    exact sum itself is zero."""
    bits = _as_bits(x, kind).copy()
    if kind == "f32":
        bits &= np.uint32(0x7FFFFFFF)
    else:
        bits &= np.uint16(0x7FFF)
    return exact_sum(bits, kind)


def sum_float(x: np.ndarray, kind: str) -> float:
    """Correctly rounded binary64 value of the exact sum."""
    return exact_sum(x, kind).value


def rel_err(result: float, exact: ExactSum) -> float:
    """|result - S*| / |S*| evaluated exactly in rationals, rounded to a float.

    Returns the absolute error when S* == 0 (the caller then compares it to
    a bound scaled by sum |x_i|)."""
    s = exact.fraction
    d = abs(Fraction(result) - s)
    return float(d / abs(s)) if s != 0 else float(d)


# --------------------------------------------------------------------------
# Segmented sums (CSR offsets: segment k is x[offsets[k]:offsets[k+1]])
# --------------------------------------------------------------------------
def segmented_sums(x: np.ndarray, offsets: np.ndarray, kind: str = "f32") -> List[ExactSum]:
    """Exact sum of every CSR segment; an empty segment sums to zero."""
    offsets = np.asarray(offsets, dtype=np.int64)
    if offsets.ndim != 1 or offsets.size < 1 or offsets[0] != 0:
        raise ValueError("offsets must be 1-D with offsets[0] == 0")
    if np.any(np.diff(offsets) < 0) or offsets[-1] > x.size:
        raise ValueError("offsets must be non-decreasing and within the array")
    out = []
    for k in range(offsets.size - 1):
        out.append(exact_sum(x[offsets[k]:offsets[k + 1]], kind))
    return out


def segmented_sums_i32(x: np.ndarray, offsets: np.ndarray) -> List[int]:
    offsets = np.asarray(offsets, dtype=np.int64)
    return [sum_i32(x[offsets[k]:offsets[k + 1]]) for k in range(offsets.size - 1)]


# --------------------------------------------------------------------------
# FP64 Neumaier (secondary cross-check only)
# --------------------------------------------------------------------------
def neumaier(x: np.ndarray) -> float:
    """Neumaier-compensated FP64 sum of the values of ``x`` (upcast exactly)."""
    d = np.ascontiguousarray(x, dtype=np.float64)
    return float(_load().oracle_neumaier_f64(d.ctypes.data, d.size))


# --------------------------------------------------------------------------
# Probe formulas (Sections IV and IX)
# --------------------------------------------------------------------------
def kernel_total_latency(t1: float, t2: float, t3: float, n_many: int = 5, n_one: int = 1) -> float:
    """Per-kernel total latency from three host timestamps (Section IV):
    one launch between t1 and t2, ``n_many`` launches between t2 and t3, so
    T = ((t3 - t2) - (t2 - t1)) / (n_many - n_one)."""
    return ((t3 - t2) - (t2 - t1)) / (n_many - n_one)


def launch_overhead_eq6(lat_ij: float, lat_ji: float, i: int, j: int) -> float:
    """Launch overhead by kernel fusion (Eq. 6): ``lat_ij`` is the latency of
    i launches of a kernel with j wait units, ``lat_ji`` of j launches with i
    wait units; both do i*j units of work, so O = (L_ij - L_ji) / (i - j)."""
    return (lat_ij - lat_ji) / (i - j)


def per_op_latency_eq7(lat_k1: float, lat_k2: float, r1: int, r2: int) -> float:
    """Host-clock differential latency (Eq. 7): two kernels that differ only
    in the repeat count r of the operation under test,
    T = (L_k1 - L_k2) / (r1 - r2)."""
    return (lat_k1 - lat_k2) / (r1 - r2)


def sigma_eq8(samples_k1: Sequence[float], samples_k2: Sequence[float], r1: int, r2: int) -> float:
    """Uncertainty of the Eq. 7 estimate (Eq. 8, last form): with
    independent measurements of the two kernels,
    sigma = sqrt(sigma_k1^2 + sigma_k2^2) / (r1 - r2), where sigma_k is the
    sample standard deviation (N - 1 denominator) of kernel k's latency."""
    def sd(v):
        v = [float(a) for a in v]
        m = sum(v) / len(v)
        return math.sqrt(sum((a - m) ** 2 for a in v) / (len(v) - 1))
    return math.sqrt(sd(samples_k1) ** 2 + sd(samples_k2) ** 2) / abs(r1 - r2)


# ---------------------------------------------------------------------------
# Iterative stencil.  Section VII-B names iterative stencil methods as the
# case where a persistent kernel holding the time loop can keep data in
# on-chip memory across grid barriers, instead of one kernel launch per
# step.  The method is the explicit step of the 1D heat equation with fixed
# end values:
#     u'[i] = u[i] + r * ((u[i-1] + u[i+1]) - 2 u[i])   for 1 <= i <= n-2,
#     u'[0] = u[0],  u'[n-1] = u[n-1],
# evaluated in exactly this order.  In ``jacobi_1d_f32`` every operation is
# one binary32 operation rounded to nearest even (numpy float32 arithmetic,
# no fused multiply-add), so a GPU that performs the same operations in the
# same order must reproduce it bit for bit.  Arrays of fewer than 3 values
# have no interior and do not change.
# ---------------------------------------------------------------------------
def jacobi_1d_f32(u0: np.ndarray, steps: int, r: float) -> np.ndarray:
    u = np.array(u0, dtype=np.float32, copy=True)
    r32 = np.float32(r)
    two = np.float32(2.0)
    if u.size < 3:
        return u
    for _ in range(steps):
        nxt = u.copy()
        neighbours = u[:-2] + u[2:]        # u[i-1] + u[i+1]
        centre = two * u[1:-1]             # 2 u[i], exact
        nxt[1:-1] = u[1:-1] + r32 * (neighbours - centre)
        u = nxt
    return u


def jacobi_1d_f64(u0: np.ndarray, steps: int, r: float) -> np.ndarray:
    """The same steps in binary64."""
    u = np.array(u0, dtype=np.float64, copy=True)
    if u.size < 3:
        return u
    for _ in range(steps):
        nxt = u.copy()
        nxt[1:-1] = u[1:-1] + r * ((u[:-2] + u[2:]) - 2.0 * u[1:-1])
        u = nxt
    return u
