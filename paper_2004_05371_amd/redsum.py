"""Python binding of libredsum (ctypes).  Argument marshalling only: every
step of a reduction runs in the HIP kernels of the library.

The C entry points are exposed under the same names (``red_sum``,
``red_sum_segmented``, ``sync_bench_grid``, ...), taking integer device
addresses and stream handles.  ``sum`` / ``segmented_sum`` are conveniences
for torch tensors (torch supplies device memory and the current stream
only).

Loading fails loudly if the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libredsum.so")

# enums (mirror include/redsum.h)
RED_I32, RED_F32, RED_F16, RED_BF16 = 0, 1, 2, 3
RED_OK, RED_EINVAL, RED_ENOTSUP, RED_EHIP, RED_ETIMEOUT, RED_ENOMEM, RED_ENODEV = 0, -1, -2, -3, -4, -5, -6
RED_VARIANT_AUTO, RED_VARIANT_RELAUNCH, RED_VARIANT_ATOMIC, RED_VARIANT_PERSISTENT = 0, 1, 2, 3
RED_VARIANT_SINGLE = 4
RED_ACC_COMPENSATED, RED_ACC_PLAIN = 0, 1
RED_WAVE_DPP, RED_WAVE_SWIZZLE, RED_WAVE_BPERMUTE, RED_WAVE_DPP_STEP = 0, 1, 2, 3
RED_MAX_GRID = 8192
RED_NOALLOC_MAX_GRID = 2048
FLAG_NONTEMPORAL = 1
FLAG_NO_GRAPH = 2
FLAG_PLAIN_LAUNCH = 4
FLAG_PIPELINE = 8
FLAG_XCD = 16
FLAG_SEG_WORKGROUP = 32
FLAG_SEG_PIECES = 64
FLAG_SEG_RUNS = 128

STATUS_NAMES = {0: "RED_OK", -1: "RED_EINVAL", -2: "RED_ENOTSUP", -3: "RED_EHIP",
                -4: "RED_ETIMEOUT", -5: "RED_ENOMEM", -6: "RED_ENODEV"}
VARIANT_NAMES = {1: "relaunch", 2: "atomic", 3: "persistent", 4: "single"}

# every symbol declared in include/redsum.h
EXPORTS = [
    "red_init", "red_shutdown", "red_last_error", "red_check_error",
    "red_sum", "red_sum_ex", "red_sum_noalloc", "red_sum_segmented", "red_sum_segmented_ex",
    "red_sum_segmented_loop", "red_set_plan", "red_get_plan", "red_autotune", "red_autotune_search",
    "red_autotune_segmented", "red_set_segmented_plan", "red_get_segmented_plan",
    "red_kernel_timer", "red_kernel_timer_read", "sync_bench_wave", "sync_bench_wave_ex", "sync_bench_block",
    "sync_bench_grid", "sync_bench_grid_ex", "sync_bench_grid_r", "sync_bench_relaunch",
    "sync_bench_relaunch_ex", "sync_bench_spin", "sync_bench_block_tput", "sync_check_wave", "sync_check_grid_order",
    "sync_check_grid_visibility", "sync_bench_grid_published", "sync_check_grid_visibility_published",
    "sync_check_watchdog", "sync_xcc_map", "red_max_coresident", "red_max_coresident_segmented",
    "red_device_info",
    "red_bw_proxy", "red_bw_proxy_ex", "red_eq6_overhead", "red_eq7_latency", "red_eq8_sigma", "stencil_jacobi_1d",
]


class Plan(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("wg", ctypes.c_int32),
                ("ipt", ctypes.c_int32), ("grid", ctypes.c_int32), ("flags", ctypes.c_int32)]

    def as_dict(self):
        return {"variant": VARIANT_NAMES.get(self.variant, self.variant), "wg": self.wg,
                "ipt": self.ipt, "grid": self.grid, "flags": self.flags}


class Opts(ctypes.Structure):
    _fields_ = [("plan", Plan), ("acc", ctypes.c_int32), ("flags", ctypes.c_int32)]


class RedError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__("%s -> %s: %s" % (fn, STATUS_NAMES.get(code, code), msg))
        self.code = code


_lib: Optional[ctypes.CDLL] = None

# double (*red_cost_fn)(red_plan *plan, void *ctx)
COST_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(Plan), ctypes.c_void_p)

_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "red_init": ([_i32], _i32),
    "red_shutdown": ([], None),
    "red_last_error": ([], ctypes.c_char_p),
    "red_check_error": ([_vp], _i32),
    "red_sum": ([_i32, _vp, _i64, _vp, _vp], _i32),
    "red_sum_ex": ([_i32, _vp, _i64, _vp, _vp, ctypes.POINTER(Opts)], _i32),
    "red_sum_noalloc": ([_i32, _vp, _i64, _vp, _vp, ctypes.POINTER(Opts)], _i32),
    "red_sum_segmented": ([_vp, _vp, _i64, _vp, _vp], _i32),
    "red_sum_segmented_ex": ([_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(Opts)], _i32),
    "red_sum_segmented_loop": ([_vp, _i64p, _i64, _vp, _vp], _i32),
    "red_set_plan": ([_i32, _i32, _i64, ctypes.POINTER(Plan)], _i32),
    "red_get_plan": ([_i32, _i32, _i64, ctypes.POINTER(Plan)], _i32),
    "red_autotune": ([_i32, _i32, _vp, _i64, _vp, _vp, _i32, ctypes.POINTER(Plan), _dp], _i32),
    "red_autotune_segmented": ([_vp, _vp, _i64, _vp, _vp, _i32, ctypes.POINTER(Plan), _dp], _i32),
    "red_autotune_search": ([_i32, _i64, _i32, _i32, _i32, _i32, COST_FN, _vp, ctypes.POINTER(Plan), _dp], _i32),
    "red_set_segmented_plan": ([_i64, ctypes.POINTER(Plan)], _i32),
    "red_get_segmented_plan": ([_i64, ctypes.POINTER(Plan)], _i32),
    "red_kernel_timer": ([_vp, _i32], _i32),
    "red_kernel_timer_read": ([_vp, _dp, _dp, _i64p], _i32),
    "sync_bench_wave": ([_i32, _i32, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_wave_ex": ([_i32, _i32, _i32, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_block": ([_i32, _i32, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_grid": ([_i32, _i32, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_grid_ex": ([_i32, _i32, _i32, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_relaunch": ([_i32, _i32, _i32, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_grid_r": ([_i32, _i32, _i32, _i64, _i64, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_relaunch_ex": ([_i32, _i32, _i32, _i32, _i32, _i64, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_bench_spin": ([_i64, _i64, _i64, _i32, _dp, _dp, _vp], _i32),
    "sync_bench_block_tput": ([_i32, _i32, _i64, _dp, _dp, _vp], _i32),
    "sync_check_wave": ([_i32, _i32, _vp, _vp, _vp], _i32),
    "sync_check_grid_order": ([_i32, _i32, _i64p, _i64p, _vp], _i32),
    "sync_check_grid_visibility": ([_i32, _i32, _i32, _i32, _i64p, _vp], _i32),
    "sync_bench_grid_published": ([_i32, _i32, _i32, _i64, _i64, _i32, _dp, _dp, _dp, _vp], _i32),
    "sync_check_grid_visibility_published": ([_i32, _i32, _i32, _i32, _i64p, _vp], _i32),
    "sync_check_watchdog": ([_i32, _i32, _i32, _i32, _vp], _i32),
    "red_max_coresident": ([_i32, _i32p], _i32),
    "red_max_coresident_segmented": ([_i32, _i32, _i32p], _i32),
    "red_device_info": ([_i32p, _i64p, _i64p, _i64p, _i64p, _i32p], _i32),
    "sync_xcc_map": ([_i32, _i32, _i32p, _vp], _i32),
    "red_bw_proxy": ([_vp, _i64, _i32, _i32, _vp], _i32),
    "red_bw_proxy_ex": ([_vp, _i64, _i32, _i32, _i32, _vp], _i32),
    "red_eq6_overhead": ([_d, _d, _i32, _i32], _d),
    "red_eq7_latency": ([_d, _d, _i64, _i64], _d),
    "red_eq8_sigma": ([_dp, _dp, _i32, _i64, _i64], _d),
    "stencil_jacobi_1d": ([_vp, _vp, _i64, _i32, ctypes.c_float, _i32, _vp, _vp], _i32),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libredsum.so (raises if it is missing: no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libredsum.so is not built (%s); run "
                              "`python -m paper_2004_05371_amd.build`" % path)
        lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        # Release the library's graphs, events, streams and workspaces while
        # the HIP runtime is still whole: Python's exit handlers run before
        # the runtime's own teardown (and before a profiler's).
        atexit.register(lib.red_shutdown)
    return _lib


def last_error() -> str:
    return load().red_last_error().decode()


def _check(rc: int, fn: str) -> int:
    if rc != RED_OK:
        raise RedError(rc, fn, last_error())
    return rc


# ---------------------------------------------------------------- raw C ABI
def red_init(device: int = 0) -> int:
    return _check(load().red_init(device), "red_init")


def red_shutdown() -> None:
    load().red_shutdown()


def red_check_error(stream: int = 0) -> int:
    return load().red_check_error(stream)


def red_sum(dtype: int, x: int, n: int, out: int, stream: int = 0) -> int:
    return _check(load().red_sum(dtype, x, n, out, stream), "red_sum")


def make_opts(variant: int = RED_VARIANT_AUTO, wg: int = 0, ipt: int = 0, grid: int = 0,
              acc: int = RED_ACC_COMPENSATED, flags: int = 0) -> Opts:
    return Opts(Plan(variant, wg, ipt, grid, 0), acc, flags)


def opts_from_plan(plan: Plan, acc: int = RED_ACC_COMPENSATED, flags: int = 0) -> Opts:
    return Opts(Plan(plan.variant, plan.wg, plan.ipt, plan.grid, plan.flags), acc, flags)


def red_sum_ex(dtype: int, x: int, n: int, out: int, stream: int = 0, opts: Optional[Opts] = None) -> int:
    return _check(load().red_sum_ex(dtype, x, n, out, stream,
                                    ctypes.byref(opts) if opts is not None else None), "red_sum_ex")


def red_sum_noalloc(dtype: int, x: int, n: int, out: int, stream: int = 0, opts: Optional[Opts] = None) -> int:
    """red_sum_ex with its partials and barrier words in the library's static
    device scratch (no allocation; calls on one device must not overlap)."""
    return _check(load().red_sum_noalloc(dtype, x, n, out, stream,
                                         ctypes.byref(opts) if opts is not None else None), "red_sum_noalloc")


def red_sum_segmented(x: int, offsets: int, nseg: int, out: int, stream: int = 0) -> int:
    return _check(load().red_sum_segmented(x, offsets, nseg, out, stream), "red_sum_segmented")


def red_sum_segmented_ex(x: int, offsets: int, nseg: int, out: int, stream: int = 0,
                         opts: Optional[Opts] = None) -> int:
    return _check(load().red_sum_segmented_ex(x, offsets, nseg, out, stream,
                                              ctypes.byref(opts) if opts is not None else None),
                  "red_sum_segmented_ex")


def red_sum_segmented_loop(x: int, host_offsets, nseg: int, out: int, stream: int = 0) -> int:
    import numpy as np
    off = np.ascontiguousarray(host_offsets, dtype=np.int64)
    return _check(load().red_sum_segmented_loop(x, off.ctypes.data_as(_i64p), nseg, out, stream),
                  "red_sum_segmented_loop")


def red_set_plan(dtype: int, acc: int, n: int, plan: Plan) -> int:
    return _check(load().red_set_plan(dtype, acc, n, ctypes.byref(plan)), "red_set_plan")


def red_get_plan(dtype: int, acc: int, n: int) -> Plan:
    p = Plan()
    _check(load().red_get_plan(dtype, acc, n, ctypes.byref(p)), "red_get_plan")
    return p


def red_autotune(dtype: int, acc: int, x: int, n: int, out: int, stream: int = 0, budget: int = 0):
    p = Plan()
    us = ctypes.c_double()
    _check(load().red_autotune(dtype, acc, x, n, out, stream, budget, ctypes.byref(p), ctypes.byref(us)),
           "red_autotune")
    return p, us.value


def red_autotune_search(dtype: int, n: int, cost, cus: int = 256, nxcc: int = 8, allow_xcd: bool = False,
                        budget: int = 0):
    """The library's candidate search with a caller-supplied cost: `cost`
    takes a Plan (it may lower plan.grid) and returns microseconds, or a
    negative status to stop.  -> (best Plan, its cost)."""
    errors = []

    def trampoline(pp, _ctx):
        try:
            return float(cost(pp.contents))
        except Exception as e:  # an exception must not cross the C frames
            errors.append(e)
            return float(RED_EINVAL)

    fn = COST_FN(trampoline)
    p = Plan()
    us = ctypes.c_double()
    rc = load().red_autotune_search(dtype, n, cus, nxcc, int(allow_xcd), budget, fn, None, ctypes.byref(p),
                                    ctypes.byref(us))
    if errors:
        raise errors[0]
    _check(rc, "red_autotune_search")
    return p, us.value


def red_autotune_segmented(x: int, offsets: int, nseg: int, out: int, stream: int = 0, budget: int = 0):
    p = Plan()
    us = ctypes.c_double()
    _check(load().red_autotune_segmented(x, offsets, nseg, out, stream, budget, ctypes.byref(p),
                                         ctypes.byref(us)), "red_autotune_segmented")
    return p, us.value


def red_set_segmented_plan(nseg: int, plan: Plan) -> int:
    return _check(load().red_set_segmented_plan(nseg, ctypes.byref(plan)), "red_set_segmented_plan")


def red_get_segmented_plan(nseg: int) -> Plan:
    p = Plan()
    _check(load().red_get_segmented_plan(nseg, ctypes.byref(p)), "red_get_segmented_plan")
    return p


def red_kernel_timer(stream: int = 0, enable=True) -> int:
    """enable: False/0 off, True/1 every launch, k > 1 every k-th launch."""
    return _check(load().red_kernel_timer(stream, int(enable)), "red_kernel_timer")


def red_kernel_timer_read(stream: int = 0):
    """-> (mean us, min us, launches timed) of the dominant kernel."""
    m, mn, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(load().red_kernel_timer_read(stream, ctypes.byref(m), ctypes.byref(mn), ctypes.byref(n)),
           "red_kernel_timer_read")
    return m.value, mn.value, n.value


def _probe3(name, *args, stream=0):
    ns, sg, cy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(getattr(load(), name)(*args, ctypes.byref(ns), ctypes.byref(sg), ctypes.byref(cy), stream), name)
    return ns.value, sg.value, cy.value


WAVE_TYPES = {"f32": 0, "i32": 1, "f64": 2, "i64": 3, "comp": 4}


def sync_bench_wave_ex(op: int, vtype: int, wg_size: int = 64, reps: int = 20, stream: int = 0):
    """-> (ns per op, sigma ns, shader-clock cycles per op) on values of
    type vtype (WAVE_TYPES)."""
    return _probe3("sync_bench_wave_ex", op, vtype, wg_size, reps, stream=stream)


def sync_bench_wave(op: int, wg_size: int = 64, reps: int = 20, stream: int = 0):
    """-> (ns per op, sigma ns, shader-clock cycles per op)"""
    return _probe3("sync_bench_wave", op, wg_size, reps, stream=stream)


def sync_bench_block(wg_size: int, n_wg: int = 1, reps: int = 20, stream: int = 0):
    """-> (ns per barrier, sigma ns, cycles per barrier)"""
    return _probe3("sync_bench_block", wg_size, n_wg, reps, stream=stream)


def sync_bench_block_tput(wg_size: int, wg_per_cu: int, window_ticks: int = 20000, stream: int = 0):
    """-> (barriers completed per microsecond per CU, cycles per barrier of one workgroup)"""
    r, c = ctypes.c_double(), ctypes.c_double()
    _check(load().sync_bench_block_tput(wg_size, wg_per_cu, window_ticks, ctypes.byref(r), ctypes.byref(c), stream),
           "sync_bench_block_tput")
    return r.value, c.value


def sync_bench_grid(n_wg: int, wg_size: int = 256, reps: int = 20, stream: int = 0):
    """-> (ns per grid barrier by Eq. 7, sigma ns by Eq. 8, in-kernel wall-clock ns per barrier)"""
    return _probe3("sync_bench_grid", n_wg, wg_size, reps, stream=stream)


def sync_bench_grid_ex(n_wg: int, wg_size: int = 256, groups: int = 0, reps: int = 20, stream: int = 0):
    """Grid barrier with an explicit shape (groups = 1 flat, > 1 two-level)."""
    return _probe3("sync_bench_grid_ex", n_wg, wg_size, groups, reps, stream=stream)


def sync_bench_grid_r(n_wg: int, wg_size: int, groups: int, r1: int, r2: int, reps: int = 20, stream: int = 0):
    """Grid barrier with the two repetition counts of Eq. 7 fixed (r1 > r2 > 0)."""
    return _probe3("sync_bench_grid_r", n_wg, wg_size, groups, r1, r2, reps, stream=stream)


def sync_bench_grid_published(n_wg: int, wg_size: int = 256, groups: int = 0, r1: int = 0, r2: int = 0,
                              reps: int = 20, stream: int = 0):
    """Grid barrier for data published by device-scope atomics (no L2
    write-back or invalidation); r1 = r2 = 0 calibrates."""
    return _probe3("sync_bench_grid_published", n_wg, wg_size, groups, r1, r2, reps, stream=stream)


LAUNCH_ORDINARY, LAUNCH_COOPERATIVE, LAUNCH_GRAPH = 0, 1, 2


def sync_bench_relaunch(n_wg: int = 256, wg_size: int = 256, cooperative=False, reps: int = 20,
                        stream: int = 0):
    """-> (launch overhead ns by Eq. 6, sigma ns, null-kernel total latency ns).
    cooperative: False/True, or a launch type LAUNCH_ORDINARY /
    LAUNCH_COOPERATIVE / LAUNCH_GRAPH."""
    return _probe3("sync_bench_relaunch", n_wg, wg_size, int(cooperative), reps, stream=stream)


def sync_bench_relaunch_ex(n_wg: int, wg_size: int, launch_type: int, i: int, j: int, unit_ticks: int = 0,
                           reps: int = 20, stream: int = 0):
    """Eq. 6 with launch counts (i, j) and a wait unit of unit_ticks 100 MHz
    ticks (0 = 5 us) -> (overhead ns, sigma ns, null-kernel ns)."""
    return _probe3("sync_bench_relaunch_ex", n_wg, wg_size, launch_type, i, j, unit_ticks, reps, stream=stream)


def sync_bench_spin(unit_ticks: int, r1: int, r2: int, reps: int = 20, stream: int = 0):
    """Eq. 7 over a wait kernel of r x unit_ticks ticks -> (ns per unit, sigma ns)."""
    ns, sg = ctypes.c_double(), ctypes.c_double()
    _check(load().sync_bench_spin(unit_ticks, r1, r2, reps, ctypes.byref(ns), ctypes.byref(sg), stream),
           "sync_bench_spin")
    return ns.value, sg.value


_WAVE_CTYPES = {0: ctypes.c_float, 1: ctypes.c_uint32, 2: ctypes.c_double, 3: ctypes.c_uint64}


def sync_check_wave(op: int, vtype: int, values, stream: int = 0):
    """One wavefront combine of 64 values (list; for the compensated type
    a list of (s, c) pairs) -> the 64 per-lane results."""
    if len(values) != 64:
        raise ValueError("64 values, one per lane")
    if vtype == WAVE_TYPES["comp"]:
        flat = [float(v) for pair in values for v in pair]
        buf_in = (ctypes.c_float * 128)(*flat)
        buf_out = (ctypes.c_float * 128)()
    else:
        ct = _WAVE_CTYPES[vtype]
        buf_in = (ct * 64)(*values)
        buf_out = (ct * 64)()
    _check(load().sync_check_wave(op, vtype, ctypes.cast(buf_in, _vp), ctypes.cast(buf_out, _vp), stream),
           "sync_check_wave")
    if vtype == WAVE_TYPES["comp"]:
        return [(buf_out[2 * k], buf_out[2 * k + 1]) for k in range(64)]
    return list(buf_out)


def sync_check_grid_visibility(n_wg: int, wg_size: int = 256, groups: int = 0, rounds: int = 50,
                               stream: int = 0) -> int:
    """Reads that missed the round's value across the grid barrier (0 when correct)."""
    e = ctypes.c_int64()
    _check(load().sync_check_grid_visibility(n_wg, wg_size, groups, rounds, ctypes.byref(e), stream),
           "sync_check_grid_visibility")
    return e.value


def sync_check_grid_visibility_published(n_wg: int, wg_size: int = 256, groups: int = 0, rounds: int = 50,
                                         stream: int = 0) -> int:
    """As sync_check_grid_visibility, with device-scope atomic stores and loads."""
    e = ctypes.c_int64()
    _check(load().sync_check_grid_visibility_published(n_wg, wg_size, groups, rounds, ctypes.byref(e), stream),
           "sync_check_grid_visibility_published")
    return e.value


def sync_check_grid_order(n_wg: int, wg_size: int = 256, stream: int = 0):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().sync_check_grid_order(n_wg, wg_size, ctypes.byref(a), ctypes.byref(b), stream),
           "sync_check_grid_order")
    return a.value, b.value


def sync_check_watchdog(n_wg: int, wg_size: int = 64, skip_wg: int = 1, spin_limit: int = 2000,
                        stream: int = 0) -> int:
    """Returns the status code (RED_ETIMEOUT is the expected outcome)."""
    return load().sync_check_watchdog(n_wg, wg_size, skip_wg, spin_limit, stream)


def red_max_coresident(wg_size: int) -> int:
    n = ctypes.c_int32()
    _check(load().red_max_coresident(wg_size, ctypes.byref(n)), "red_max_coresident")
    return n.value


def red_max_coresident_segmented(ipt: int, wg_size: int) -> int:
    n = ctypes.c_int32()
    _check(load().red_max_coresident_segmented(ipt, wg_size, ctypes.byref(n)), "red_max_coresident_segmented")
    return n.value


def red_device_info() -> dict:
    cus, nx = ctypes.c_int32(), ctypes.c_int32()
    wc, ck, l2, hbm = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().red_device_info(ctypes.byref(cus), ctypes.byref(wc), ctypes.byref(ck), ctypes.byref(l2),
                                  ctypes.byref(hbm), ctypes.byref(nx)), "red_device_info")
    return {"cus": cus.value, "wallclock_khz": wc.value, "clock_khz": ck.value,
            "l2_bytes": l2.value, "hbm_bytes": hbm.value, "nxcc": nx.value}


def sync_xcc_map(n_wg: int, wg_size: int = 64, stream: int = 0):
    """XCD of each workgroup of an ordinary launch (list of ints)."""
    buf = (ctypes.c_int32 * n_wg)()
    _check(load().sync_xcc_map(n_wg, wg_size, buf, stream), "sync_xcc_map")
    return list(buf)


def stencil_jacobi_1d(u: int, scratch: int, n: int, steps: int, r: float, steps_per_sync: int = 0,
                      stream: int = 0, opts: Optional[Opts] = None) -> int:
    return _check(load().stencil_jacobi_1d(u, scratch, n, steps, r, steps_per_sync, stream,
                                           ctypes.byref(opts) if opts is not None else None), "stencil_jacobi_1d")


def jacobi(t, steps: int, r: float, scratch=None, steps_per_sync: int = 0, opts: Optional[Opts] = None):
    """In-place steps of the 1D Jacobi stencil on a contiguous float32 CUDA
    tensor (asynchronous); returns t."""
    import torch
    if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float32:
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if scratch is None:
        scratch = torch.empty_like(t)
    stencil_jacobi_1d(t.data_ptr(), scratch.data_ptr(), t.numel(), steps, r, steps_per_sync, current_stream(), opts)
    return t


def red_bw_proxy(x: int, nbytes: int, n_wg: int, wg_size: int, stream: int = 0) -> int:
    return _check(load().red_bw_proxy(x, nbytes, n_wg, wg_size, stream), "red_bw_proxy")


def red_bw_proxy_ex(x: int, nbytes: int, n_wg: int, wg_size: int, flags: int = 0, stream: int = 0) -> int:
    return _check(load().red_bw_proxy_ex(x, nbytes, n_wg, wg_size, flags, stream), "red_bw_proxy_ex")


def red_eq6_overhead(lat_ij: float, lat_ji: float, i: int, j: int) -> float:
    return load().red_eq6_overhead(lat_ij, lat_ji, i, j)


def red_eq7_latency(lat_k1: float, lat_k2: float, r1: int, r2: int) -> float:
    return load().red_eq7_latency(lat_k1, lat_k2, r1, r2)


def red_eq8_sigma(k1, k2, r1: int, r2: int) -> float:
    a = (ctypes.c_double * len(k1))(*k1)
    b = (ctypes.c_double * len(k2))(*k2)
    return load().red_eq8_sigma(a, b, min(len(k1), len(k2)), r1, r2)


# ---------------------------------------------------------------- torch helpers
_DTYPE_CODES = None


def dtype_code(t) -> int:
    global _DTYPE_CODES
    import torch
    if _DTYPE_CODES is None:
        _DTYPE_CODES = {torch.int32: RED_I32, torch.float32: RED_F32,
                        torch.float16: RED_F16, torch.bfloat16: RED_BF16}
    if t.dtype not in _DTYPE_CODES:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return _DTYPE_CODES[t.dtype]


def _check_out(out, dtype, count: int, device) -> None:
    """A caller's output tensor: `dtype`, contiguous, on `device`, with room
    for `count` results (checked before any launch writes into it)."""
    if not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous CUDA tensor")
    if out.dtype != dtype:
        raise ValueError("out must be %s, not %s" % (dtype, out.dtype))
    if out.device != device:
        raise ValueError("out is on %s, the input on %s" % (out.device, device))
    if out.numel() < count:
        raise ValueError("out holds %d elements, %d are written" % (out.numel(), count))


def current_stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


def sum(t, out=None, opts: Optional[Opts] = None):
    """Sum of a contiguous 1-D CUDA tensor (int32 -> int64, float -> float64),
    returned as a 0-d device tensor (asynchronous)."""
    import torch
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    code = dtype_code(t)
    want = torch.int64 if code == RED_I32 else torch.float64
    if out is None:
        out = torch.empty((), dtype=want, device=t.device)
    else:
        _check_out(out, want, 1, t.device)
    red_sum_ex(code, t.data_ptr(), t.numel(), out.data_ptr(), current_stream(), opts)
    return out


def segmented_sum(values, offsets, out=None, opts: Optional[Opts] = None):
    """Per-segment float64 sums of a float32 CUDA tensor with int64 CSR offsets."""
    import torch
    if values.dtype != torch.float32 or offsets.dtype != torch.int64:
        raise TypeError("values must be float32 and offsets int64")
    for name, t in (("values", values), ("offsets", offsets)):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous CUDA tensor" % name)
    if offsets.device != values.device:
        raise ValueError("values and offsets are on different devices")
    if offsets.dim() != 1 or offsets.numel() < 1:
        raise ValueError("offsets must be 1-D with nseg + 1 entries")
    nseg = offsets.numel() - 1
    if out is None:
        out = torch.empty(nseg, dtype=torch.float64, device=values.device)
    else:
        _check_out(out, torch.float64, nseg, values.device)
    red_sum_segmented_ex(values.data_ptr(), offsets.data_ptr(), nseg, out.data_ptr(), current_stream(), opts)
    return out
