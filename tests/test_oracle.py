"""Pins for the CPU oracle (no GPU).

Each test fixes the oracle to something other than itself: arbitrary
precision brute force (Python int / fractions.Fraction) on small inputs, a
correctly rounded library routine (math.fsum) on larger ones, closed forms,
special values and invariants.  The cases are chosen so that a plausible
mistake in the oracle (a wrong exponent bias, a dropped implicit bit, a
wrong subnormal exponent, a lost sign, a wrong fp16 layout, an off-by-one in
a segment bound) fails at least one of them.
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2004_05371_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def frac_sum(values):
    return sum((Fraction(float(v)) for v in values), Fraction(0))


# ---------------------------------------------------------------- integers
def test_i32_bruteforce_small():
    r = np.random.default_rng(1)
    for n in [0, 1, 2, 3, 63, 64, 65, 1000, 4096]:
        x = r.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
        assert oracle.sum_i32(x) == sum(int(v) for v in x)


def test_i32_closed_forms():
    cf = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))
    for n_log2 in (20, 26):
        n = 1 << n_log2
        x = np.arange(1, n + 1, dtype=np.int64).astype(np.int32)
        assert oracle.sum_i32(x) == cf["int_1_to_n"][str(n_log2)]
    k = 1 << 20
    assert oracle.sum_i32(np.full(k, -2**31, dtype=np.int32)) == -(2**51)
    assert oracle.sum_i32(np.full(k, 2**31 - 1, dtype=np.int32)) == k * (2**31 - 1)


# -------------------------------------------------------------- fp32 exact
def _f32_cases():
    r = np.random.default_rng(7)
    cases = {
        "normal": r.standard_normal(4096).astype(np.float32),
        "wide": (np.power(10.0, r.uniform(-38, 38, 4096)) * r.choice([-1.0, 1.0], 4096)).astype(np.float32),
        "subnormal": (r.integers(1, 1 << 23, 2048).astype(np.uint32)
                      | (r.integers(0, 2, 2048).astype(np.uint32) << 31)).view(np.float32),
        "huge": np.array([3.4028235e38, 3.4028235e38, -3.4028235e38, 1e-45, -1e-45, 1.0], dtype=np.float32),
        "cancel": np.concatenate([np.float32([1e30, 1.0, -1e30, 2**-149]),
                                  np.float32([2**24, 1, -(2**24)])]),
        "tiny_n": np.float32([0.1]),
        "empty": np.zeros(0, dtype=np.float32),
    }
    # random bit patterns over every finite exponent
    bits = r.integers(0, 2**32, 4096, dtype=np.uint64).astype(np.uint32)
    bits = bits[((bits >> 23) & 0xFF) != 0xFF]
    cases["bits"] = bits.view(np.float32)
    return cases


@pytest.mark.parametrize("name", list(_f32_cases().keys()))
def test_f32_exact_vs_fraction(name):
    x = _f32_cases()[name]
    ex = oracle.exact_sum(x, "f32")
    ref = frac_sum(x)
    assert ex.fraction == ref
    assert ex.value == float(ref)  # float(Fraction) is correctly rounded


@pytest.mark.parametrize("gen", ["uniform", "normal", "mixed"])
def test_f32_vs_fsum(gen):
    n = 1 << 20
    x = {"uniform": lambda: inputs.uniform_f32(n),
         "normal": lambda: inputs.normal_f32(n),
         "mixed": lambda: inputs.mixed_f32(n)}[gen]()
    # math.fsum is correctly rounded; fp32 -> fp64 is exact
    assert oracle.sum_float(x, "f32") == math.fsum(x.astype(np.float64).tolist())


def test_f32_closed_forms():
    cf = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))
    x = np.arange(1, (1 << 24) + 1, dtype=np.float32)
    assert oracle.exact_sum(x, "f32").fraction == cf["f32_1_to_2^24"]
    n = 1 << 24
    assert oracle.exact_sum(np.ones(n, np.float32), "f32").fraction == n
    # 0.1f == 13421773 * 2^-27 exactly
    c = np.float32(0.1)
    assert Fraction(float(c)) == Fraction(13421773, 2**27)
    assert oracle.exact_sum(np.full(n, c), "f32").fraction == Fraction(n * 13421773, 2**27)
    alt = np.tile(np.float32([0.3, -0.3]), n // 2)
    assert oracle.exact_sum(alt, "f32").fraction == 0
    # powers of two across the whole exponent range, each once: a geometric
    # series with a closed form sum_{k=-149}^{127} 2^k = 2^128 - 2^-149
    p = np.array([2.0**k for k in range(-149, 128)], dtype=np.float64).astype(np.float32)
    assert oracle.exact_sum(p, "f32").fraction == Fraction(2**128) - Fraction(1, 2**149)


def test_f32_specials():
    nan, inf = np.float32("nan"), np.float32("inf")
    assert math.isnan(oracle.sum_float(np.float32([1, nan, 2]), "f32"))
    assert oracle.sum_float(np.float32([1, inf, 2]), "f32") == math.inf
    assert oracle.sum_float(np.float32([1, -inf]), "f32") == -math.inf
    assert math.isnan(oracle.sum_float(np.float32([inf, -inf]), "f32"))
    assert oracle.exact_sum(np.float32([1, nan]), "f32").n_nan == 1


def test_f32_invariants():
    x = inputs.mixed_f32(1 << 16)
    a = oracle.exact_sum(x, "f32")
    perm = np.random.default_rng(3).permutation(x.size)
    assert oracle.exact_sum(x[perm], "f32").fraction == a.fraction
    assert oracle.exact_sum(-x, "f32").fraction == -a.fraction
    assert oracle.exact_sum(x * np.float32(4.0), "f32").fraction == 4 * a.fraction
    assert oracle.exact_sum(x * np.float32(0.5), "f32").fraction == a.fraction / 2
    # splitting the array: sum of parts equals the whole
    parts = [oracle.exact_sum(p, "f32").fraction for p in np.array_split(x, 7)]
    assert sum(parts) == a.fraction


# ---------------------------------------------------------------- fp16
def test_f16_every_finite_pattern():
    bits = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16)
    exp = (bits >> 10) & 0x1F
    bits = bits[exp != 0x1F]
    x = bits.view(np.float16)
    ex = oracle.exact_sum(x, "f16")
    # positive and negative patterns cancel exactly
    assert ex.fraction == 0
    pos = x[x > 0]
    assert oracle.exact_sum(pos, "f16").fraction == frac_sum(pos)


def test_f16_subnormals_and_random():
    r = np.random.default_rng(11)
    sub = (r.integers(1, 1 << 10, 3000).astype(np.uint16)
           | (r.integers(0, 2, 3000).astype(np.uint16) << 15)).view(np.float16)
    assert oracle.exact_sum(sub, "f16").fraction == frac_sum(sub)
    x = r.standard_normal(4096).astype(np.float16)
    assert oracle.exact_sum(x, "f16").fraction == frac_sum(x)
    assert oracle.exact_sum(x.view(np.uint16), "f16").fraction == frac_sum(x)
    y = inputs.normal_half_bits(1 << 20, "f16")
    assert oracle.sum_float(y, "f16") == math.fsum(y.view(np.float16).astype(np.float64).tolist())


def test_f16_specials():
    assert math.isnan(oracle.sum_float(np.float16([1, np.nan]), "f16"))
    assert oracle.sum_float(np.float16([1, np.inf]), "f16") == math.inf
    assert math.isnan(oracle.sum_float(np.float16([np.inf, -np.inf]), "f16"))


# ---------------------------------------------------------------- bf16
def test_bf16_vs_torch_upcast():
    import torch
    r = np.random.default_rng(5)
    x = torch.from_numpy((r.standard_normal(4096) * 10.0 ** r.uniform(-30, 30, 4096)).astype(np.float32))
    b = x.to(torch.bfloat16)
    bits = b.view(torch.int16).numpy().view(np.uint16)
    vals = b.to(torch.float32).numpy()  # bf16 -> fp32 is exact
    assert oracle.exact_sum(bits, "bf16").fraction == frac_sum(vals)
    y = inputs.normal_half_bits(1 << 20, "bf16")
    yv = torch.from_numpy(y.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    assert oracle.sum_float(y, "bf16") == math.fsum(yv.tolist())


# ------------------------------------------------------------ error metric
def test_rel_err_exact():
    x = np.float32([1.0, 2.0**-30])
    ex = oracle.exact_sum(x, "f32")
    assert oracle.rel_err(1.0 + 2.0**-30, ex) == 0.0
    e = oracle.rel_err(1.0, ex)
    assert e == float(Fraction(2**-30) / (1 + Fraction(2**-30)))
    zero = oracle.exact_sum(np.float32([1.0, -1.0]), "f32")
    assert oracle.rel_err(0.5, zero) == 0.5  # absolute error when S* == 0


def test_abs_sum():
    x = np.float32([1.5, -2.5, 3.0])
    assert oracle.exact_abs_sum(x, "f32").fraction == 7


# ------------------------------------------------------------ Neumaier
def test_neumaier_close_to_exact():
    x = inputs.normal_f32(1 << 18)
    ex = oracle.exact_sum(x, "f32").value
    nm = oracle.neumaier(x)
    assert abs(nm - ex) <= 4 * math.ulp(ex)


# ------------------------------------------------------------ segmented
def test_segmented_matches_slices():
    x = inputs.normal_f32(5000, sub=3)
    off = np.array([0, 0, 1, 1, 10, 4000, 4000, 5000], dtype=np.int64)
    sums = oracle.segmented_sums(x, off)
    assert len(sums) == 7
    for k in range(7):
        assert sums[k].fraction == frac_sum(x[off[k]:off[k + 1]])
    assert sums[0].fraction == 0 and sums[2].fraction == 0 and sums[5].fraction == 0
    assert sum(s.fraction for s in sums) == oracle.exact_sum(x, "f32").fraction
    xi = inputs.uniform_i32(5000)
    si = oracle.segmented_sums_i32(xi, off)
    assert si == [sum(int(v) for v in xi[off[k]:off[k + 1]]) for k in range(7)]


def test_segmented_rejects_bad_offsets():
    x = np.zeros(10, np.float32)
    with pytest.raises(ValueError):
        oracle.segmented_sums(x, np.array([1, 5], np.int64))
    with pytest.raises(ValueError):
        oracle.segmented_sums(x, np.array([0, 5, 3], np.int64))
    with pytest.raises(ValueError):
        oracle.segmented_sums(x, np.array([0, 11], np.int64))


# ------------------------------------------------------------ probe formulas
def test_eq6_recovers_injected_overhead():
    # latency model: i launches of a kernel with j wait units of w ns each,
    # launch overhead O ns per launch, fixed host cost c ns
    O, w, c = 1081.0, 5000.0, 7000.0
    for i, j in [(8, 1), (5, 2), (3, 7)]:
        lij = c + i * O + i * j * w
        lji = c + j * O + i * j * w
        assert oracle.launch_overhead_eq6(lij, lji, i, j) == pytest.approx(O, rel=1e-12)


def test_eq7_recovers_per_op_latency():
    t, base = 4.0, 3210.0
    for r1, r2 in [(1024, 512), (4096, 512), (10, 1)]:
        assert oracle.per_op_latency_eq7(base + r1 * t, base + r2 * t, r1, r2) == pytest.approx(t, rel=1e-12)


def test_kernel_total_latency_section4():
    # t2 - t1 = overhead + 1 kernel; t3 - t2 = overhead + 5 kernels
    k, ovh = 8888.0, 2500.0
    t1 = 0.0
    t2 = t1 + ovh + k
    t3 = t2 + ovh + 5 * k
    assert oracle.kernel_total_latency(t1, t2, t3) == pytest.approx(k)


def test_eq8_sigma():
    import statistics
    a = [10.0, 12.0, 11.0, 13.0, 9.0]
    b = [5.0, 5.5, 4.5, 5.0, 6.0]
    want = math.sqrt(statistics.stdev(a) ** 2 + statistics.stdev(b) ** 2) / 7
    assert oracle.sigma_eq8(a, b, 8, 1) == pytest.approx(want, rel=1e-12)
    assert oracle.sigma_eq8([3.0] * 4, [1.0] * 4, 2, 1) == 0.0


# ------------------------------------------------------------- stencil
# The iterative stencil of Section VII-B (the time loop a persistent kernel
# can hold): u'[i] = u[i] + r ((u[i-1] + u[i+1]) - 2 u[i]), ends fixed.

def test_jacobi_binomial_closed_form():
    """r = 1/4 turns a step into u' = (u[i-1] + 2 u[i] + u[i+1]) / 4, so T
    steps from a unit impulse give C(2T, T+k) / 4^T at distance k.  Every
    value is a multiple of 4^-T below 1, exact in binary32 for T <= 12."""
    for T in (0, 1, 2, 5, 12):
        n = 2 * T + 9
        c = n // 2
        u = np.zeros(n, np.float32)
        u[c] = 1.0
        got = oracle.jacobi_1d_f32(u, T, 0.25)
        want = np.zeros(n)
        for k in range(-T, T + 1):
            want[c + k] = math.comb(2 * T, T + k) / 4.0 ** T
        assert np.array_equal(got.astype(np.float64), want), T


def test_jacobi_constant_and_linear_fields_are_fixed_points():
    """A constant or an integer-valued linear field has zero second
    difference: every step leaves it unchanged, bit for bit."""
    for r in (0.1, 0.25, 0.4999):
        c = np.full(101, 3.75, np.float32)
        assert np.array_equal(oracle.jacobi_1d_f32(c, 50, r), c)
        lin = (7 - 3 * np.arange(101)).astype(np.float32)
        assert np.array_equal(oracle.jacobi_1d_f32(lin, 50, r), lin)


def test_jacobi_mirror_symmetry_and_fixed_ends():
    x = inputs.normal_f32(1001, sub=50)
    a = oracle.jacobi_1d_f32(x, 37, 0.3)
    b = oracle.jacobi_1d_f32(x[::-1], 37, 0.3)
    assert np.array_equal(a, b[::-1])  # (u[i-1] + u[i+1]) is symmetric
    assert a[0] == x[0] and a[-1] == x[-1]
    assert not np.array_equal(a[1:-1], x[1:-1])


def test_jacobi_eigenmode_decay():
    """sin(pi k i / (n-1)) vanishes at both ends and is an eigenvector:
    one step multiplies it by 1 - 4 r sin^2(pi k / (2 (n-1)))."""
    n, k, r, T = 257, 3, 0.3, 200
    i = np.arange(n)
    u0 = np.sin(np.pi * k * i / (n - 1))
    lam = 1 - 4 * r * math.sin(math.pi * k / (2 * (n - 1))) ** 2
    got = oracle.jacobi_1d_f64(u0, T, r)
    assert np.max(np.abs(got - lam ** T * u0)) <= 1e-12
    got32 = oracle.jacobi_1d_f32(u0.astype(np.float32), T, r).astype(np.float64)
    assert np.max(np.abs(got32 - lam ** T * u0)) <= 2e-5


def test_jacobi_brute_force_rationals():
    """Exact rational evaluation of the recurrence on tiny random inputs:
    the binary64 version agrees to rounding, the binary32 version within
    its rounding bound (a few ulps of the largest value per step)."""
    rng = random.Random(7)
    for _ in range(20):
        n = rng.randint(3, 9)
        T = rng.randint(0, 6)
        r = rng.choice([0.125, 0.3, 0.45])
        x = np.array([rng.uniform(-2, 2) for _ in range(n)], np.float32)
        u = [Fraction(float(v)) for v in x]
        fr = Fraction(float(np.float32(r)))
        for _ in range(T):
            u = [u[0]] + [u[j] + fr * ((u[j - 1] + u[j + 1]) - 2 * u[j]) for j in range(1, n - 1)] + [u[-1]]
        exact = np.array([float(v) for v in u])
        g64 = oracle.jacobi_1d_f64(x.astype(np.float64), T, float(np.float32(r)))
        assert np.max(np.abs(g64 - exact)) <= 1e-14
        g32 = oracle.jacobi_1d_f32(x, T, r).astype(np.float64)
        assert np.max(np.abs(g32 - exact)) <= 4 * (T + 1) * 2.0 ** -22


def test_jacobi_short_arrays_and_zero_steps():
    for n in (0, 1, 2):
        x = np.arange(n, dtype=np.float32)
        assert np.array_equal(oracle.jacobi_1d_f32(x, 5, 0.25), x)
    x = inputs.normal_f32(50, sub=51)
    assert np.array_equal(oracle.jacobi_1d_f32(x, 0, 0.25), x)
