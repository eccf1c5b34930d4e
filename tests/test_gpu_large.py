"""GPU parity beyond 2^31 elements (64-bit indexing): the device-wide sum
and the segmented batch on about 8.6 GB of values, against closed forms.

The values repeat the integers -1000 .. 1000 (period 2001), so every prefix
sum has a closed form and every partial sum is exact in fp32 and int64:
P(m) = sum_{i<m} x_i = r (r - 1) / 2 - 1000 r with r = m mod 2001 (a whole
period sums to zero).  Inputs are built on the device.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

PERIOD = 2001
N = (1 << 31) + (1 << 20) + 3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def prefix(m: int) -> int:
    r = m % PERIOD
    return r * (r - 1) // 2 - 1000 * r


def pattern(n: int, dtype):
    base = torch.arange(PERIOD, dtype=dtype, device="cuda") - 1000
    return base.repeat(n // PERIOD + 1)[:n]


# 16-bit inputs: the integers -128 .. 128 (period 257), exact in bf16 and fp16.
PERIOD16 = 257


def prefix16(m: int) -> int:
    r = m % PERIOD16
    return r * (r - 1) // 2 - 128 * r


def pattern16(n: int, dtype):
    base = (torch.arange(PERIOD16, dtype=torch.float32, device="cuda") - 128).to(dtype)
    return base.repeat(n // PERIOD16 + 1)[:n]


def test_closed_form():
    x = np.arange(5 * PERIOD + 77) % PERIOD - 1000
    for m in (0, 1, 1000, PERIOD, 3 * PERIOD + 5, x.size):
        assert prefix(m) == int(x[:m].sum())
    y = np.arange(5 * PERIOD16 + 77) % PERIOD16 - 128
    for m in (0, 1, 128, PERIOD16, 3 * PERIOD16 + 5, y.size):
        assert prefix16(m) == int(y[:m].sum())


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_half_sum_beyond_2p31(lib, kind):
    say(kind, "sum, n =", N)
    dtype = torch.bfloat16 if kind == "bf16" else torch.float16
    code = lib.RED_BF16 if kind == "bf16" else lib.RED_F16
    x = pattern16(N, dtype)
    out = torch.empty((), dtype=torch.float64, device="cuda")
    lib.red_sum_ex(code, x.data_ptr(), N, out.data_ptr(), lib.current_stream(), lib.make_opts())
    torch.cuda.synchronize()
    assert out.item() == float(prefix16(N))
    del x
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [1, 2, 3])
def test_int32_sum_beyond_2p31(lib, variant):
    say("int32 sum, n =", N, "variant", variant)
    x = pattern(N, torch.int32)
    out = torch.empty((), dtype=torch.int64, device="cuda")
    lib.red_sum_ex(lib.RED_I32, x.data_ptr(), N, out.data_ptr(), lib.current_stream(),
                   lib.make_opts(variant=variant))
    torch.cuda.synchronize()
    assert out.item() == prefix(N)
    del x
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [1, 2, 3])
def test_f32_sum_beyond_2p31(lib, variant):
    say("f32 sum, n =", N, "variant", variant)
    x = pattern(N, torch.float32)
    out = torch.empty((), dtype=torch.float64, device="cuda")
    lib.red_sum_ex(lib.RED_F32, x.data_ptr(), N, out.data_ptr(), lib.current_stream(),
                   lib.make_opts(variant=variant))
    torch.cuda.synchronize()
    assert out.item() == float(prefix(N))  # every partial is an exact integer
    del x
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("form", [0, 32, 64, 128])
def test_segmented_beyond_2p31(lib, form):
    """A first segment of 2^31 + 5 values, then short and mid-length
    segments and empties that all lie past position 2^31."""
    r = np.random.default_rng(77)
    tail = N - ((1 << 31) + 5)
    lens = []
    while sum(lens) < tail:
        lens.append(int(r.choice([0, 3, 17, 64, 300, 5000, 70000])))
    lens[-1] -= sum(lens) - tail
    lens = [(1 << 31) + 5] + lens
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    assert off[-1] == N
    nseg = off.size - 1
    say("segmented, values", N, "segments", nseg, "form", form)
    x = pattern(N, torch.float32)
    ot = torch.from_numpy(off).to("cuda")
    out = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
    lib.red_sum_segmented_ex(x.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), lib.current_stream(),
                             lib.make_opts(flags=form))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    exp = np.array([prefix(int(off[k + 1])) - prefix(int(off[k])) for k in range(nseg)], dtype=np.float64)
    bad = np.nonzero(got != exp)[0]
    assert bad.size == 0, (int(bad[0]), got[bad[0]], exp[bad[0]], bad.size)
    del x, ot, out
    torch.cuda.empty_cache()
