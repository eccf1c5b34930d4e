"""red_sum_noalloc (the entry point that allocates nothing: its partials and
barrier words live in the library's static device scratch) against
red_sum_ex, the entry point it varies, through the C ABI: the same plan
gives the same bits, on two calls in a row, the second with a smaller
input, for every synchronization variant, and within the oracle's bound.
Its grid limit is refused with RED_EINVAL."""
import ctypes
import sys

import pytest

import oracle
from paper_2004_05371_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# relaunch, atomic ticket, persistent (cooperative), persistent through an
# ordinary occupancy-capped launch, one workgroup, and the default plan
PLANS = [dict(variant=1, wg=256, ipt=4, grid=512), dict(variant=2, wg=256, ipt=2, grid=300),
         dict(variant=3, wg=256, ipt=4, grid=256), dict(variant=3, wg=512, ipt=2, grid=128, flags=4),
         dict(variant=4, wg=1024, ipt=2, grid=1), dict()]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("plan", range(len(PLANS)))
@pytest.mark.parametrize("kind", ["f32", "i32", "bf16"])
def test_noalloc_matches_red_sum_ex_twice(lib, plan, kind):
    p = PLANS[plan]
    opts = lib.make_opts(**p) if p else None
    code = {"f32": lib.RED_F32, "i32": lib.RED_I32, "bf16": lib.RED_BF16}[kind]
    s = torch.cuda.current_stream().cuda_stream
    for call, n in enumerate((3_000_017, 200_003)):  # the second call smaller
        say("noalloc plan", p, kind, "call", call, "n", n)
        if kind == "i32":
            h = inputs.uniform_i32(n, sub=70 + call)
            x = torch.from_numpy(h).to("cuda")
            out_t, ref_t = (torch.full((), -1, dtype=torch.int64, device="cuda") for _ in range(2))
        else:
            h = inputs.normal_f32(n, sub=70 + call)
            x = torch.from_numpy(h).to("cuda")
            if kind == "bf16":
                x = x.to(torch.bfloat16)
            out_t, ref_t = (torch.full((), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2))
        lib.red_sum_noalloc(code, x.data_ptr(), n, out_t.data_ptr(), s, opts)
        lib.red_sum_ex(code, x.data_ptr(), n, ref_t.data_ptr(), s, opts)
        torch.cuda.synchronize()
        got, ref = out_t.item(), ref_t.item()
        assert got == ref, (p, kind, call, got, ref)
        if kind == "i32":
            assert got == oracle.sum_i32(h)
        else:
            hx = h if kind == "f32" else x.view(torch.int16).cpu().numpy().view("uint16")
            ex = oracle.exact_sum(hx, "f32" if kind == "f32" else "bf16")
            assert oracle.rel_err(got, ex) <= (1e-6 if kind == "f32" else 1e-3)


def test_noalloc_empty_and_tiny(lib):
    s = torch.cuda.current_stream().cuda_stream
    out = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    x = torch.ones(5, dtype=torch.float32, device="cuda")
    lib.red_sum_noalloc(lib.RED_F32, x.data_ptr(), 0, out.data_ptr(), s)
    torch.cuda.synchronize()
    assert out.item() == 0.0
    lib.red_sum_noalloc(lib.RED_F32, x.data_ptr(), 5, out.data_ptr(), s)
    torch.cuda.synchronize()
    assert out.item() == 5.0


def test_noalloc_refuses_a_grid_beyond_its_scratch(lib):
    x = torch.ones(1 << 20, dtype=torch.float32, device="cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    big = lib.make_opts(variant=1, wg=256, ipt=1, grid=lib.RED_NOALLOC_MAX_GRID + 1)
    rc = lib.load().red_sum_noalloc(lib.RED_F32, ctypes.c_void_p(x.data_ptr()), x.numel(),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s), ctypes.byref(big))
    assert rc == lib.RED_EINVAL
    assert "scratch" in lib.last_error()
    ok = lib.make_opts(variant=1, wg=256, ipt=1, grid=lib.RED_NOALLOC_MAX_GRID)
    lib.red_sum_noalloc(lib.RED_F32, x.data_ptr(), x.numel(), out.data_ptr(), s, ok)
    torch.cuda.synchronize()
    assert out.item() == float(1 << 20)
