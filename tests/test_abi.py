"""C-ABI library checks that need no GPU: the library loads, exports every
symbol that include/redsum.h declares, validates arguments before touching
HIP, reports RED_ENODEV without a device, and its host-side probe formulas
agree with the oracle's (Eq. 6, 7, 8)."""
import ctypes
import os
import re

import pytest

import oracle
from paper_2004_05371_amd import redsum as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "redsum.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|double|const char\s*\*)\s*\**\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return R.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 20
    assert sorted(R.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


def has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_validation_before_hip(lib):
    # Each of these must fail validation without any HIP call.
    assert lib.red_sum(99, None, 0, None, None) == R.RED_EINVAL
    assert lib.red_sum(R.RED_F32, None, 10, ctypes.c_void_p(64), None) == R.RED_EINVAL
    assert lib.red_sum(R.RED_F32, ctypes.c_void_p(64), -1, ctypes.c_void_p(64), None) == R.RED_EINVAL
    assert lib.red_sum(R.RED_F32, ctypes.c_void_p(64), 1 << 40, ctypes.c_void_p(64), None) == R.RED_EINVAL
    assert lib.red_sum(R.RED_F32, ctypes.c_void_p(66), 4, ctypes.c_void_p(64), None) == R.RED_EINVAL  # misaligned
    assert lib.red_sum(R.RED_F32, ctypes.c_void_p(64), 4, None, None) == R.RED_EINVAL
    assert "out" in R.last_error()
    bad = R.make_opts(variant=R.RED_VARIANT_RELAUNCH, wg=100, ipt=4)
    assert lib.red_sum_ex(R.RED_F32, ctypes.c_void_p(64), 4, ctypes.c_void_p(64), None, ctypes.byref(bad)) == R.RED_EINVAL
    bad = R.make_opts(variant=R.RED_VARIANT_RELAUNCH, wg=256, ipt=3)
    assert lib.red_sum_ex(R.RED_F32, ctypes.c_void_p(64), 4, ctypes.c_void_p(64), None, ctypes.byref(bad)) == R.RED_EINVAL
    bad = R.make_opts(acc=7)
    assert lib.red_sum_ex(R.RED_F32, ctypes.c_void_p(64), 4, ctypes.c_void_p(64), None, ctypes.byref(bad)) == R.RED_EINVAL
    bad = R.make_opts(flags=32)
    assert lib.red_sum_ex(R.RED_F32, ctypes.c_void_p(64), 4, ctypes.c_void_p(64), None, ctypes.byref(bad)) == R.RED_EINVAL
    assert lib.red_sum_segmented(None, None, 3, None, None) == R.RED_EINVAL
    big_wg = R.make_opts(variant=R.RED_VARIANT_ATOMIC, wg=1024, ipt=4, grid=8)  # segmented: <= 512 threads
    assert lib.red_sum_segmented_ex(ctypes.c_void_p(64), ctypes.c_void_p(64), 2, ctypes.c_void_p(64), None,
                                    ctypes.byref(big_wg)) == R.RED_EINVAL
    assert lib.red_sum_segmented(ctypes.c_void_p(64), ctypes.c_void_p(64), -1, ctypes.c_void_p(64), None) == R.RED_EINVAL
    assert lib.red_sum_segmented(ctypes.c_void_p(64), ctypes.c_void_p(68), 2, ctypes.c_void_p(64), None) == R.RED_EINVAL
    for f in (R.FLAG_SEG_WORKGROUP | R.FLAG_SEG_RUNS, R.FLAG_SEG_PIECES | R.FLAG_SEG_RUNS, 256):
        two = R.make_opts(flags=f)  # at most one form flag; unknown bits rejected
        assert lib.red_sum_segmented_ex(ctypes.c_void_p(64), ctypes.c_void_p(64), 2, ctypes.c_void_p(64), None,
                                        ctypes.byref(two)) == R.RED_EINVAL
    seg = R.make_opts(variant=R.RED_VARIANT_SINGLE, wg=256, ipt=4)
    assert lib.red_sum_segmented_ex(ctypes.c_void_p(64), ctypes.c_void_p(64), 2, ctypes.c_void_p(64), None,
                                    ctypes.byref(seg)) == R.RED_EINVAL
    n = ctypes.c_int32()
    assert lib.red_max_coresident_segmented(4, 1024, ctypes.byref(n)) == R.RED_EINVAL  # segmented: <= 512
    assert lib.red_max_coresident_segmented(4, 100, ctypes.byref(n)) == R.RED_EINVAL
    assert lib.sync_bench_wave(9, 64, 10, None, None, None, None) == R.RED_EINVAL
    assert lib.sync_bench_wave_ex(0, 5, 64, 10, None, None, None, None) == R.RED_EINVAL
    assert lib.sync_bench_wave_ex(4, 0, 64, 10, None, None, None, None) == R.RED_EINVAL
    assert lib.sync_bench_grid(0, 256, 10, None, None, None, None) == R.RED_EINVAL
    # stencil: negative steps, overlapping arrays, bad variant
    assert lib.stencil_jacobi_1d(ctypes.c_void_p(64), ctypes.c_void_p(1 << 20), 10, -1, ctypes.c_float(0.25), 0,
                                 None, None) == R.RED_EINVAL
    assert lib.stencil_jacobi_1d(ctypes.c_void_p(64), ctypes.c_void_p(64 + 16), 10, 1, ctypes.c_float(0.25), 0,
                                 None, None) == R.RED_EINVAL
    bad = R.make_opts(variant=R.RED_VARIANT_ATOMIC)
    assert lib.stencil_jacobi_1d(ctypes.c_void_p(64), ctypes.c_void_p(1 << 20), 10, 1, ctypes.c_float(0.25), 0,
                                 None, ctypes.byref(bad)) == R.RED_EINVAL
    d = ctypes.c_double()
    for kind in (-1, 3):  # launch types are 0 ordinary, 1 cooperative, 2 graph
        assert lib.sync_bench_relaunch(8, 64, kind, 10, ctypes.byref(d), ctypes.byref(d), None, None) == R.RED_EINVAL
    assert lib.sync_check_watchdog(4, 64, 9, 100, None) == R.RED_EINVAL
    assert lib.red_bw_proxy_ex(ctypes.c_void_p(64), 1024, 4, 256, 2, None) == R.RED_EINVAL  # unknown flag
    e = ctypes.c_int64()
    assert lib.sync_check_grid_visibility(0, 256, 0, 10, ctypes.byref(e), None) == R.RED_EINVAL
    assert lib.sync_check_grid_visibility(4, 256, -3, 10, ctypes.byref(e), None) == R.RED_EINVAL
    assert lib.sync_check_grid_visibility(4, 256, 0, 0, ctypes.byref(e), None) == R.RED_EINVAL
    assert lib.sync_check_grid_visibility_published(0, 256, 0, 10, ctypes.byref(e), None) == R.RED_EINVAL
    assert lib.sync_check_grid_visibility_published(4, 256, 33, 10, ctypes.byref(e), None) == R.RED_EINVAL
    assert lib.sync_check_grid_visibility_published(4, 100, 0, 10, ctypes.byref(e), None) == R.RED_EINVAL
    p = R.Plan(R.RED_VARIANT_PERSISTENT, 256, 16, 0, 0)
    assert lib.red_set_plan(R.RED_F32, 0, 100, ctypes.byref(p)) == R.RED_EINVAL
    # the no-allocation entry point: its grid limit, before any HIP call
    big = R.make_opts(variant=R.RED_VARIANT_RELAUNCH, wg=256, ipt=4, grid=R.RED_NOALLOC_MAX_GRID + 1)
    assert lib.red_sum_noalloc(R.RED_F32, ctypes.c_void_p(64), 4, ctypes.c_void_p(64), None,
                               ctypes.byref(big)) == R.RED_EINVAL
    assert "scratch" in R.last_error()
    assert lib.red_sum_noalloc(R.RED_F32, ctypes.c_void_p(64), -3, ctypes.c_void_p(64), None, None) == R.RED_EINVAL
    # probe validation: repetition counts, launch counts, wait units, wave ops
    dd = ctypes.byref(d)
    assert lib.sync_bench_grid_r(8, 256, 0, 16, 16, 5, dd, dd, None, None) == R.RED_EINVAL  # r1 == r2
    assert lib.sync_bench_grid_r(8, 256, 0, 0, 5, 5, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_grid_r(8, 256, 0, 1 << 20, 5, 5, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_grid_published(8, 256, 0, 16, 16, 5, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_grid_published(8, 256, -3, 0, 0, 5, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_grid_published(0, 256, 0, 0, 0, 5, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_relaunch_ex(8, 64, 0, 4, 4, 0, 10, dd, dd, None, None) == R.RED_EINVAL  # i == j
    assert lib.sync_bench_relaunch_ex(8, 64, 0, 65, 1, 0, 10, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_relaunch_ex(8, 64, 0, 8, 1, -1, 10, dd, dd, None, None) == R.RED_EINVAL
    assert lib.sync_bench_spin(0, 8, 1, 10, dd, dd, None) == R.RED_EINVAL
    assert lib.sync_bench_spin(100, 8, 8, 10, dd, dd, None) == R.RED_EINVAL
    assert lib.sync_bench_spin(10**7, 100, 1, 10, dd, dd, None) == R.RED_EINVAL  # > 1 s of waiting
    buf = (ctypes.c_double * 64)()
    assert lib.sync_check_wave(7, 0, buf, buf, None) == R.RED_EINVAL
    assert lib.sync_check_wave(0, 9, buf, buf, None) == R.RED_EINVAL
    assert lib.sync_check_wave(0, 0, None, buf, None) == R.RED_EINVAL
    # host-side loop baseline validates host offsets
    off = (ctypes.c_int64 * 3)(0, 5, 2)
    assert lib.red_sum_segmented_loop(ctypes.c_void_p(64), off, 2, ctypes.c_void_p(64), None) == R.RED_EINVAL


@pytest.mark.skipif(has_gpu(), reason="checks the no-device path")
def test_no_device_reports_enodev(lib):
    assert lib.red_init(0) == R.RED_ENODEV
    assert lib.red_sum(R.RED_F32, ctypes.c_void_p(64), 4, ctypes.c_void_p(64), None) == R.RED_ENODEV
    assert "device" in R.last_error()


def test_plan_table_roundtrip(lib):
    p = R.Plan(R.RED_VARIANT_ATOMIC, 256, 2, 512, 1)
    R.red_set_plan(R.RED_BF16, R.RED_ACC_COMPENSATED, 1 << 20, p)
    q = R.red_get_plan(R.RED_BF16, R.RED_ACC_COMPENSATED, (1 << 20) - 5)  # same ceil(log2) bucket
    assert (q.variant, q.wg, q.ipt, q.grid, q.flags) == (2, 256, 2, 512, 1)
    d = R.red_get_plan(R.RED_BF16, R.RED_ACC_PLAIN, 1 << 20)  # other bucket key -> default
    assert d.variant in (1, 2, 3) and d.wg % 64 == 0


def test_host_probe_formulas_match_oracle(lib):
    assert R.red_eq6_overhead(9000.0, 2000.0, 8, 1) == pytest.approx(oracle.launch_overhead_eq6(9000.0, 2000.0, 8, 1))
    assert R.red_eq7_latency(5000.0, 1000.0, 4096, 512) == pytest.approx(oracle.per_op_latency_eq7(5000.0, 1000.0, 4096, 512))
    a = [10.0, 12.0, 11.0, 13.0, 9.0, 10.5]
    b = [5.0, 5.5, 4.5, 5.0, 6.0, 5.25]
    assert R.red_eq8_sigma(a, b, 64, 8) == pytest.approx(oracle.sigma_eq8(a, b, 64, 8), rel=1e-12)


def test_default_plan_follows_model_switch_point(lib):
    """Small inputs default to one workgroup (no device-wide sync), large
    ones to the relaunch variant (Eq. 5 switch point)."""
    small = R.red_get_plan(R.RED_F32, R.RED_ACC_COMPENSATED, 1000)
    assert small.variant == R.RED_VARIANT_SINGLE
    mid = R.red_get_plan(R.RED_F32, R.RED_ACC_COMPENSATED, 1 << 18)
    assert mid.variant == R.RED_VARIANT_ATOMIC
    large = R.red_get_plan(R.RED_F32, R.RED_ACC_COMPENSATED, 1 << 28)
    assert large.variant == R.RED_VARIANT_RELAUNCH
    # the same switch point in bytes for 16-bit inputs
    assert R.red_get_plan(R.RED_BF16, R.RED_ACC_COMPENSATED, 2000).variant == R.RED_VARIANT_SINGLE


class _FakeCudaTensor:
    """Stand-in for a CUDA tensor: the fields the wrappers check, and a
    data_ptr that must never be reached when a check fails."""

    def __init__(self, dtype, numel, device="cuda:0", contiguous=True, cuda=True):
        import torch
        self.dtype = dtype
        self._n = numel
        self.device = torch.device(device)
        self._contig = contiguous
        self.is_cuda = cuda

    def is_contiguous(self):
        return self._contig

    def numel(self):
        return self._n

    def dim(self):
        return 1

    def data_ptr(self):
        raise AssertionError("a wrapper passed a pointer on after a failed check")


def test_wrappers_reject_bad_tensors_before_any_launch():
    import torch
    f32, f64, i64 = torch.float32, torch.float64, torch.int64
    T = _FakeCudaTensor
    # sum: out of the wrong dtype, size, device or layout
    with pytest.raises(ValueError, match="float64"):
        R.sum(T(f32, 100), out=T(f32, 1))
    with pytest.raises(ValueError, match="int64"):
        R.sum(T(torch.int32, 100), out=T(f64, 1))
    with pytest.raises(ValueError, match="holds 0"):
        R.sum(T(f32, 100), out=T(f64, 0))
    with pytest.raises(ValueError, match="is on"):
        R.sum(T(f32, 100), out=T(f64, 1, device="cuda:1"))
    with pytest.raises(ValueError, match="contiguous"):
        R.sum(T(f32, 100), out=T(f64, 1, contiguous=False))
    with pytest.raises(ValueError):
        R.sum(T(f32, 100, cuda=False))
    # segmented: host offsets, non-contiguous values, devices, out
    with pytest.raises(ValueError, match="offsets"):
        R.segmented_sum(T(f32, 100), T(i64, 11, device="cpu", cuda=False))
    with pytest.raises(ValueError, match="values"):
        R.segmented_sum(T(f32, 100, contiguous=False), T(i64, 11))
    with pytest.raises(ValueError, match="devices"):
        R.segmented_sum(T(f32, 100), T(i64, 11, device="cuda:1"))
    with pytest.raises(ValueError, match="nseg"):
        R.segmented_sum(T(f32, 100), T(i64, 0))
    with pytest.raises(ValueError, match="holds 9"):
        R.segmented_sum(T(f32, 100), T(i64, 11), out=T(f64, 9))
    with pytest.raises(ValueError, match="float64"):
        R.segmented_sum(T(f32, 100), T(i64, 11), out=T(f32, 10))
    with pytest.raises(TypeError):
        R.segmented_sum(T(f32, 100), T(torch.int32, 11))


def test_xcd_tree_layout_covers_every_grid():
    """The arrival tree's first-level lines (class r = g mod nxcc, node
    (g / nxcc) / 64, line r + nxcc * node) for every grid the library
    launches: every line index is inside the 144 lines, and each node's
    expected count is the number of workgroups that map to it."""
    import numpy as np
    fan, max_lines = 64, 144
    for nxcc in (2, 4, 8, 14):
        for n in list(range(1, 70)) + [100, 255, 256, 257, 511, 512, 1000, 1024, 2047, 2048, 4096, 8191, 8192]:
            g = np.arange(n)
            r, j = g % nxcc, g // nxcc
            members = (n - r + nxcc - 1) // nxcc
            node = j // fan
            line = r + nxcc * node
            assert line.max() < max_lines, (nxcc, n)
            nsize = np.minimum(fan, members - node * fan)
            counts = np.bincount(line, minlength=max_lines)
            assert (counts[line] == nsize).all(), (nxcc, n)
            nodes = (members + fan - 1) // fan
            for cls in range(min(n, nxcc)):
                assert len(set(node[r == cls])) == nodes[r == cls][0]
