"""GPU parity of the device-wide sum (red_sum / red_sum_ex) against the CPU
oracle.  Every call goes through the C ABI of libredsum.

Bars: int32 -> int64 bit-exact; fp32 inputs (compensated) relative error
<= 1e-6 against the exact sum; bf16/fp16 inputs <= 1e-3.  When the exact
sum is 0 the absolute error is compared with 1e-6 * sum |x|.  Plain fp32
accumulation is reported, and held only to a loose bound.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2004_05371_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = [1, 2, 3, 4]  # relaunch, atomic, persistent, single workgroup
BOUND = {"f32": 1e-6, "f16": 1e-3, "bf16": 1e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_tensor(a: np.ndarray, kind: str = None, pad: int = 0):
    """Copy a host array to the GPU; with pad > 0 the returned view starts
    `pad` elements into its allocation (misaligned base pointer)."""
    if kind == "bf16":
        t = torch.from_numpy(a.view(np.int16)).view(torch.bfloat16)
    elif kind == "f16":
        t = torch.from_numpy(a.view(np.int16)).view(torch.float16)
    else:
        t = torch.from_numpy(a)
    if pad:
        buf = torch.zeros(a.size + pad, dtype=t.dtype, device="cuda")
        buf[pad:].copy_(t)
        return buf[pad:]
    return t.to("cuda")


def gpu_sum(lib, t, variant=0, wg=0, ipt=0, grid=0, acc=0, flags=0):
    opts = lib.make_opts(variant=variant, wg=wg, ipt=ipt, grid=grid, acc=acc, flags=flags)
    out = lib.sum(t, opts=opts)
    torch.cuda.synchronize()
    return out.item()


def check_float(r, x, kind, bound):
    ex = oracle.exact_sum(x, kind)
    if ex.fraction == 0:
        absx = float(oracle.exact_abs_sum(x, kind).fraction)
        assert abs(r) <= 1e-6 * absx, (r, absx)
        return 0.0
    e = oracle.rel_err(r, ex)
    assert e <= bound, (kind, r, ex.value, e)
    return e


# ------------------------------------------------------------------ int32
INT_SIZES = [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 4095, 4096, 4097, (1 << 16) - 1, (1 << 16) + 1,
             512 * 4 * 4 - 1, 512 * 4 * 4 + 1, 1000003]


@pytest.mark.parametrize("variant", VARIANTS)
def test_int32_sizes_bit_exact(lib, variant):
    x_all = inputs.uniform_i32(max(INT_SIZES), lo=-2**31, hi=2**31 - 1, sub=5)
    for n in INT_SIZES:
        x = x_all[:n]
        say("int32 n=%d variant=%d" % (n, variant))
        r = gpu_sum(lib, dev_tensor(x) if n else torch.zeros(0, dtype=torch.int32, device="cuda"), variant=variant)
        assert r == oracle.sum_i32(x), n


@pytest.mark.parametrize("pad", [1, 2, 3, 5, 7])
def test_int32_misaligned(lib, pad):
    x = inputs.uniform_i32(100003, sub=6)
    for variant in VARIANTS:
        r = gpu_sum(lib, dev_tensor(x, pad=pad), variant=variant)
        assert r == oracle.sum_i32(x)


@pytest.mark.parametrize("wg,ipt", [(64, 1), (128, 2), (256, 8), (1024, 4), (1024, 8)])
@pytest.mark.parametrize("grid", [1, 7, 256, 2048])
def test_int32_plans(lib, wg, ipt, grid):
    x = inputs.uniform_i32(3 * 1000 * 1000 + 17, sub=7)
    ref = oracle.sum_i32(x)
    t = dev_tensor(x)
    for variant in VARIANTS:
        g = grid
        if variant == 3:
            g = min(grid, lib.red_max_coresident(wg))
        if variant == 4:
            g = 1
        assert gpu_sum(lib, t, variant=variant, wg=wg, ipt=ipt, grid=g) == ref


def test_int32_closed_forms(lib):
    n = 1 << 20
    t = torch.arange(1, n + 1, dtype=torch.int32, device="cuda")
    for variant in VARIANTS:
        assert gpu_sum(lib, t, variant=variant) == n * (n + 1) // 2
    k = 1 << 20
    assert gpu_sum(lib, torch.full((k,), -2**31, dtype=torch.int32, device="cuda")) == -(2**51)
    assert gpu_sum(lib, torch.full((k,), 2**31 - 1, dtype=torch.int32, device="cuda")) == k * (2**31 - 1)


# ------------------------------------------------------------------ fp32
F32_SIZES = [1, 2, 3, 5, 63, 64, 65, 257, 4095, 4097, 65537, 1000003]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("gen", ["uniform", "normal", "mixed"])
def test_f32_compensated_sizes(lib, variant, gen):
    n_max = max(F32_SIZES)
    x_all = {"uniform": inputs.uniform_f32, "normal": inputs.normal_f32, "mixed": inputs.mixed_f32}[gen](n_max)
    for n in F32_SIZES:
        x = x_all[:n]
        r = gpu_sum(lib, dev_tensor(x), variant=variant)
        check_float(r, x, "f32", BOUND["f32"])


@pytest.mark.parametrize("pad", [1, 2, 3])
def test_f32_misaligned(lib, pad):
    x = inputs.mixed_f32(300007, sub=4)
    for variant in VARIANTS:
        check_float(gpu_sum(lib, dev_tensor(x, pad=pad), variant=variant), x, "f32", BOUND["f32"])


def test_f32_plain_loose(lib):
    x = inputs.normal_f32(1 << 22)
    for variant in VARIANTS:
        r = gpu_sum(lib, dev_tensor(x), variant=variant, acc=1)
        check_float(r, x, "f32", 1e-3)


def test_f32_closed_forms(lib):
    n = 1 << 24
    t = torch.arange(1, n + 1, dtype=torch.float32, device="cuda")
    # compensated accumulation is exact here (every partial and error term
    # is an integer well inside fp32 / binary64 range); plain fp32 is not,
    # since thread partials pass 2^24
    for variant in VARIANTS:
        assert gpu_sum(lib, t, variant=variant) == 140737496743936.0
    ones = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    for acc in (0, 1):
        assert gpu_sum(lib, ones, acc=acc) == float(1 << 26)
    c = torch.full((1 << 22,), 0.1, dtype=torch.float32, device="cuda")
    assert gpu_sum(lib, c) == (1 << 22) * 13421773 * 2.0**-27
    alt = torch.tensor([0.3, -0.3], dtype=torch.float32, device="cuda").repeat(1 << 20)
    assert gpu_sum(lib, alt) == 0.0


def test_f32_invariants_bitwise(lib):
    x = inputs.mixed_f32(2000003, sub=8)
    t = dev_tensor(x)
    for variant in VARIANTS:
        a = gpu_sum(lib, t, variant=variant)
        assert gpu_sum(lib, t, variant=variant) == a  # re-run identical
        assert gpu_sum(lib, -t, variant=variant) == -a
        assert gpu_sum(lib, t * 4.0, variant=variant) == 4.0 * a
        assert gpu_sum(lib, t * 0.125, variant=variant) == a * 0.125


def test_f32_specials(lib):
    x = torch.ones(100000, dtype=torch.float32, device="cuda")
    x[5000] = float("nan")
    assert math.isnan(gpu_sum(lib, x))
    x[5000] = float("inf")
    assert gpu_sum(lib, x) == math.inf
    x[7000] = float("-inf")
    assert math.isnan(gpu_sum(lib, x))


def test_f32_subnormals(lib):
    r = np.random.default_rng(2)
    bits = (r.integers(1, 1 << 23, 100003).astype(np.uint32) | (r.integers(0, 2, 100003).astype(np.uint32) << 31))
    x = bits.view(np.float32)
    for variant in VARIANTS:
        check_float(gpu_sum(lib, dev_tensor(x), variant=variant), x, "f32", BOUND["f32"])


# ------------------------------------------------------------------ 16-bit
@pytest.mark.parametrize("kind", ["bf16", "f16"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_half_sizes(lib, kind, variant):
    xa = inputs.normal_half_bits(1000003, kind, sub=2)
    for n in [1, 2, 7, 8, 9, 64, 513, 4097, 65537, 1000003]:
        x = xa[:n]
        for acc in (0, 1):
            r = gpu_sum(lib, dev_tensor(x, kind), variant=variant, acc=acc)
            check_float(r, x, kind, BOUND[kind])


@pytest.mark.parametrize("kind", ["bf16", "f16"])
@pytest.mark.parametrize("pad", [1, 3, 7])
def test_half_misaligned(lib, kind, pad):
    x = inputs.normal_half_bits(200001, kind, sub=3)
    check_float(gpu_sum(lib, dev_tensor(x, kind, pad=pad)), x, kind, BOUND[kind])


def test_f16_subnormal_exact_conversion(lib):
    # every fp16 subnormal pattern once (positive): the sum is small enough
    # that fp32 accumulation of subnormal fp16 values is exact
    bits = np.arange(1, 1 << 10, dtype=np.uint16)
    x = bits
    r = gpu_sum(lib, dev_tensor(x, "f16"))
    assert r == oracle.exact_sum(x, "f16").value


# ------------------------------------------------------------------ full sizes
def test_full_small_config(lib):
    """2^20 fp32 U[-1,1] and int32 U[-1000,1000], two-launch variant."""
    xf = inputs.uniform_f32(1 << 20)
    xi = inputs.uniform_i32(1 << 20)
    say("small config")
    check_float(gpu_sum(lib, dev_tensor(xf), variant=1), xf, "f32", BOUND["f32"])
    assert gpu_sum(lib, dev_tensor(xi), variant=1) == oracle.sum_i32(xi)


def test_full_int_config_three_variants(lib):
    """int32 2^26, bit-exact, relaunch vs atomic vs persistent."""
    x = inputs.uniform_i32(1 << 26)
    ref = oracle.sum_i32(x)
    t = dev_tensor(x)
    for v in VARIANTS:
        say("int 2^26 variant", v)
        assert gpu_sum(lib, t, variant=v) == ref


@pytest.mark.parametrize("gen", ["normal", "mixed"])
def test_full_f32_config(lib, gen):
    """fp32 2^28, plain and compensated, error vs the exact sum."""
    n = 1 << 28
    x = inputs.normal_f32(n) if gen == "normal" else inputs.mixed_f32(n)
    t = dev_tensor(x)
    ex = oracle.exact_sum(x, "f32")
    for v in VARIANTS:
        r = gpu_sum(lib, t, variant=v)
        e = oracle.rel_err(r, ex)
        say("f32 2^28 %s variant %d compensated rel_err %.3e" % (gen, v, e))
        assert e <= BOUND["f32"]
        rp = gpu_sum(lib, t, variant=v, acc=1)
        say("f32 2^28 %s variant %d plain rel_err %.3e" % (gen, v, oracle.rel_err(rp, ex)))
    del t
    torch.cuda.empty_cache()


def test_headline_plan_from_the_cache(lib):
    """The launch configuration the benchmark times: the committed plan for
    fp32 compensated 2^28, repeated calls bit-identical and within bound."""
    from paper_2004_05371_amd import autotune
    assert autotune.load() > 0
    n = 1 << 28
    plan = lib.red_get_plan(lib.RED_F32, lib.RED_ACC_COMPENSATED, n)
    say("headline plan", plan.as_dict())
    import json
    with open(autotune.cache_path()) as fh:
        entries = json.load(fh)["entries"]
    cached = [e["plan"] for e in entries
              if e["kind"] == "sum" and e["dtype"] == "f32" and e["acc"] == "compensated"
              and autotune.bucket(e["n"]) == autotune.bucket(n)]
    assert len(cached) == 1 and plan.as_dict() == cached[0]
    x = inputs.normal_f32(n)
    t = dev_tensor(x)
    ex = oracle.exact_sum(x, "f32")
    o = lib.opts_from_plan(plan)
    outs = [lib.sum(t, opts=o) for _ in range(5)]
    torch.cuda.synchronize()
    vals = [v.item() for v in outs]
    assert len(set(vals)) == 1
    assert oracle.rel_err(vals[0], ex) <= BOUND["f32"]
    del t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_full_half_config(lib, kind):
    """bf16 / fp16 2^29 N(0,1), compensated."""
    n = 1 << 29
    x = inputs.normal_half_bits(n, kind)
    t = dev_tensor(x, kind)
    ex = oracle.exact_sum(x, kind)
    for v in VARIANTS:
        r = gpu_sum(lib, t, variant=v)
        e = oracle.rel_err(r, ex)
        say("%s 2^29 variant %d rel_err %.3e" % (kind, v, e))
        assert e <= BOUND[kind]
    del t
    torch.cuda.empty_cache()


def test_budgeted_tune_sum_installs_the_plan_it_returns(lib):
    """autotune.tune_sum (red_autotune, Section VII-A/B's search over launch
    shapes and variants, timed on the data) with a budget: the plan it
    returns is the one installed for that size, red_sum without options
    then gives the same bits as that plan given explicitly, and the result
    is within the bound of the exact oracle."""
    from paper_2004_05371_amd import autotune
    n = 3_000_017
    before = lib.red_get_plan(lib.RED_F32, lib.RED_ACC_COMPENSATED, n)
    x = inputs.normal_f32(n, sub=61)
    t = torch.from_numpy(x).to("cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    try:
        entry = autotune.tune_sum(t, out, budget=12)
        say("tuned", entry)
        got = lib.red_get_plan(lib.RED_F32, lib.RED_ACC_COMPENSATED, n)
        assert got.as_dict() == entry["plan"]
        assert entry["us"] > 0
        auto = lib.sum(t)
        explicit = lib.sum(t, opts=lib.opts_from_plan(got))
        torch.cuda.synchronize()
        assert auto.item() == explicit.item()
        assert oracle.rel_err(auto.item(), oracle.exact_sum(x, "f32")) <= BOUND["f32"]
    finally:
        lib.red_set_plan(lib.RED_F32, lib.RED_ACC_COMPENSATED, n, before)
