"""GPU parity of the iterative stencil (stencil_jacobi_1d) with the oracle,
bit for bit: every form performs the same binary32 operations in the same
order, so one launch per step, the persistent kernel with any number of
steps per grid barrier, any grid and any barrier shape must all equal
the step-by-step definition exactly."""
import sys

import numpy as np
import pytest

import oracle
from paper_2004_05371_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RELAUNCH, PERSISTENT, AUTO = 1, 3, 0


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(lib, x, steps, r, variant=AUTO, spsync=0, grid=0, wg=0, flags=0, shift=0):
    base = torch.zeros(x.size + 8, dtype=torch.float32, device="cuda")
    u = base[shift:shift + x.size]
    u.copy_(torch.from_numpy(x))
    scratch = torch.full((max(x.size, 1),), float("nan"), dtype=torch.float32, device="cuda")
    opts = lib.make_opts(variant=variant, wg=wg, grid=grid, flags=flags)
    lib.stencil_jacobi_1d(u.data_ptr(), scratch.data_ptr(), x.size, steps, r, spsync, lib.current_stream(), opts)
    torch.cuda.synchronize()
    assert lib.red_check_error(lib.current_stream()) == lib.RED_OK
    return u.cpu().numpy()


FORMS = [dict(variant=RELAUNCH), dict(variant=PERSISTENT, spsync=1), dict(variant=PERSISTENT, spsync=3),
         dict(variant=PERSISTENT), dict(variant=PERSISTENT, spsync=32, grid=7),
         dict(variant=PERSISTENT, spsync=5, grid=64, wg=256), dict(variant=PERSISTENT, flags=16),
         dict(variant=PERSISTENT, spsync=4, flags=4), dict(variant=AUTO)]


@pytest.mark.parametrize("form", range(len(FORMS)))
def test_small_sizes_bit_exact(lib, form):
    f = FORMS[form]
    for n in (3, 4, 5, 64, 65, 1000, 4099):
        x = inputs.normal_f32(n, sub=60 + n % 7)
        for steps in (1, 2, 9, 40):
            want = oracle.jacobi_1d_f32(x, steps, 0.3)
            got = run(lib, x, steps, 0.3, **f)
            assert np.array_equal(got, want), (f, n, steps, np.flatnonzero(got != want)[:5])


@pytest.mark.parametrize("n,wg,grid", [(1000, 512, 0), (9_001, 128, 4), (100_003, 512, 16), (100_003, 1024, 16),
                                        ((1 << 20) + 3, 256, 256), (4099, 64, 4)])
def test_caller_workgroup_sizes(lib, n, wg, grid):
    """A caller's workgroup size sets the values each thread holds (4 to 32
    here: the fewest that cover the window), bit for bit for the library's
    halo and a short one."""
    x = inputs.normal_f32(n, sub=67)
    for spsync in (0, 7):
        want = oracle.jacobi_1d_f32(x, 40, 0.3)
        got = run(lib, x, 40, 0.3, variant=PERSISTENT, spsync=spsync, wg=wg, grid=grid)
        assert np.array_equal(got, want), (n, wg, grid, spsync, np.flatnonzero(got != want)[:5])


def test_no_op_cases(lib):
    for n in (0, 1, 2):
        x = np.arange(n, dtype=np.float32)
        assert np.array_equal(run(lib, x, 5, 0.25), x)
    x = inputs.normal_f32(500, sub=61)
    for v in (RELAUNCH, PERSISTENT):
        assert np.array_equal(run(lib, x, 0, 0.25, variant=v), x)


@pytest.mark.parametrize("shift", [1, 3])
def test_misaligned_values(lib, shift):
    x = inputs.normal_f32(100003, sub=62)
    want = oracle.jacobi_1d_f32(x, 17, 0.25)
    for v in (RELAUNCH, PERSISTENT):
        assert np.array_equal(run(lib, x, 17, 0.25, variant=v, shift=shift), want)


def test_binomial_impulse(lib):
    """r = 1/4 from a unit impulse: C(2T, T+k) / 4^T, exact (T <= 12)."""
    n, T = 4097, 12
    x = np.zeros(n, np.float32)
    x[n // 2] = 1.0
    got = run(lib, x, T, 0.25, variant=PERSISTENT, spsync=5)
    import math
    for k in range(-T, T + 1):
        assert got[n // 2 + k] == math.comb(2 * T, T + k) / 4.0 ** T
    assert np.count_nonzero(got) == 2 * T + 1


def test_large_persistent_and_auto_fallback(lib):
    """A million values for 200 steps in one persistent launch; an array
    larger than the co-resident windows is refused by the persistent
    form and run by one launch per step under AUTO."""
    x = inputs.normal_f32((1 << 20) + 5, sub=63)
    want = oracle.jacobi_1d_f32(x, 200, 0.4)
    for spsync in (1, 16):
        assert np.array_equal(run(lib, x, 200, 0.4, variant=PERSISTENT, spsync=spsync), want)
    big = inputs.normal_f32(12_000_001, sub=64)
    t = torch.from_numpy(big).to("cuda")
    s = torch.empty_like(t)
    with pytest.raises(lib.RedError) as e:
        lib.stencil_jacobi_1d(t.data_ptr(), s.data_ptr(), t.numel(), 3, 0.25, 0, lib.current_stream(),
                              lib.make_opts(variant=PERSISTENT))
    assert e.value.code == lib.RED_EINVAL
    lib.stencil_jacobi_1d(t.data_ptr(), s.data_ptr(), t.numel(), 3, 0.25, 0, lib.current_stream(),
                          lib.make_opts(variant=AUTO))
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.jacobi_1d_f32(big, 3, 0.25))


@pytest.mark.parametrize("n,steps,spsync,flags", [(1 << 22, 200, 0, 0), (1 << 22, 200, 32, 0), (1 << 22, 130, 0, 16),
                                                  (8_000_000, 60, 0, 0)])
def test_bench_sizes_default_geometry(lib, n, steps, spsync, flags):
    """The 4 M-value workload of the bench line and the 8 M-value table size
    in the default geometry (a whole number of workgroups per CU, the
    library's halo, or k = 32; XCD-aggregated barrier), bit for bit."""
    x = inputs.normal_f32(n, sub=66)
    say("stencil", n, "values,", steps, "steps, steps_per_sync", spsync, "flags", flags)
    want = oracle.jacobi_1d_f32(x, steps, 0.25)
    got = run(lib, x, steps, 0.25, variant=PERSISTENT, spsync=spsync, flags=flags)
    assert np.array_equal(got, want), np.flatnonzero(got != want)[:5]


def test_repeat_and_graph_capture(lib):
    """The persistent launch recorded into a caller's graph and replayed:
    each replay continues from the previous state, like eager calls."""
    n, steps = 300_007, 11
    x = inputs.normal_f32(n, sub=65)
    u = torch.from_numpy(x).to("cuda")
    sc = torch.empty_like(u)
    st = torch.cuda.Stream()
    o = lib.make_opts(variant=PERSISTENT, flags=4)
    with torch.cuda.stream(st):
        lib.stencil_jacobi_1d(u.data_ptr(), sc.data_ptr(), n, steps, 0.3, 4, st.cuda_stream, o)
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        lib.stencil_jacobi_1d(u.data_ptr(), sc.data_ptr(), n, steps, 0.3, 4, st.cuda_stream, o)
    want = oracle.jacobi_1d_f32(x, steps, 0.3)
    assert np.array_equal(u.cpu().numpy(), want)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        want = oracle.jacobi_1d_f32(want, steps, 0.3)
        assert np.array_equal(u.cpu().numpy(), want), rep


def test_runs_shorter_than_one_exchange_repeated(lib):
    """Fewer steps than steps_per_sync: no exchange happens, and the final
    write-back of every block must still wait until all neighbours have
    read their initial halos from u (regression: it once did not)."""
    for rep in range(20):
        n = 1000 + 37 * rep
        x = inputs.normal_f32(n, sub=70 + rep)
        for steps in (1, 2, 7):
            want = oracle.jacobi_1d_f32(x, steps, 0.3)
            for flags in (0, 16, 4):
                got = run(lib, x, steps, 0.3, variant=PERSISTENT, flags=flags)
                assert np.array_equal(got, want), (rep, steps, flags, np.flatnonzero(got != want)[:5])
