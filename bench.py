#!/usr/bin/env python3
"""Benchmark of the device-wide fp32 sum reduction on one MI355X.

Workload: the sum of 2^28 fp32 values drawn N(0,1) (1 GiB, resident in HBM
before timing starts), TwoSum-compensated fp32 accumulation with a binary64
final combine, launched with the autotuned plan.  One step = one call of
red_sum over the whole array (per-thread accumulation, wavefront and
workgroup combines, device-wide synchronization, final combine).

Prints ONE JSON line: GB/s (= 2^30 bytes / time per step) and the fraction
of the 8 TB/s HBM peak, plus the grid-barrier and relaunch latencies, the
other synchronization variants, the bandwidth-proxy ceiling, the error of
the result against the exact CPU oracle, and the oracle's own CPU time.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
N = 1 << 28
METRIC = "reduction GB/s & % of HBM peak (fp32, 2^28 elems); grid-barrier latency ns"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_f32_2p28.json")
CSRC = os.path.join(ROOT, "paper_2004_05371_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if it is absent or was taken on a
    different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def time_steps(fn, steps, stream):
    """Per-step HIP event times (ms) on `stream` over `steps` calls."""
    import torch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [s.elapsed_time(e) for s, e in zip(starts, ends)], wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2004_05371_amd import inputs, redsum as R

    R.load()
    torch.cuda.set_device(0)
    R.red_init(0)
    dev = R.red_device_info()
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    log("device", dev)

    # ---- input, resident in HBM before timing
    t0 = time.time()
    x = inputs.normal_f32(N)
    xt = torch.from_numpy(x).to("cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    log("input ready in %.1f s" % (time.time() - t0))
    nbytes = N * 4

    # ---- autotune the plan for this workload
    plan, tuned_us = R.red_autotune(R.RED_F32, R.RED_ACC_COMPENSATED, xt.data_ptr(), N, out.data_ptr(), sh)
    log("tuned plan", plan.as_dict(), "%.1f us" % tuned_us)
    opts = R.make_opts(variant=plan.variant, wg=plan.wg, ipt=plan.ipt, grid=plan.grid,
                       acc=R.RED_ACC_COMPENSATED)

    def step():
        R.red_sum_ex(R.RED_F32, xt.data_ptr(), N, out.data_ptr(), sh, opts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times, wall = time_steps(step, args.steps, stream)
    ms_per_step = wall * 1e3 / args.steps
    mean_ms = statistics.fmean(times)
    gbps = nbytes / (ms_per_step * 1e-3) / 1e9
    kernel_gbps = nbytes / (mean_ms * 1e-3) / 1e9
    result = out.item()
    log("steps: wall %.3f ms/step, event mean %.3f ms, median %.3f ms" %
        (ms_per_step, mean_ms, statistics.median(times)))

    extra = {}
    # ---- other variants / accumulation (a few steps each)
    variants = {}
    for v, name in ((1, "relaunch"), (2, "atomic"), (3, "persistent")):
        o = R.make_opts(variant=v, wg=plan.wg, ipt=plan.ipt, grid=plan.grid if v != 3 else min(
            plan.grid or 4 * dev["cus"], R.red_max_coresident(plan.wg)))
        fn = (lambda o=o: R.red_sum_ex(R.RED_F32, xt.data_ptr(), N, out.data_ptr(), sh, o))
        for _ in range(5):
            fn()
        tt, _ = time_steps(fn, 50, stream)
        variants[name] = round(nbytes / (statistics.median(tt) * 1e-3) / 1e9, 1)
    extra["variants_GBps"] = variants
    o = R.make_opts(variant=plan.variant, wg=plan.wg, ipt=plan.ipt, grid=plan.grid, acc=R.RED_ACC_PLAIN)
    tt, _ = time_steps(lambda: R.red_sum_ex(R.RED_F32, xt.data_ptr(), N, out.data_ptr(), sh, o), 50, stream)
    extra["plain_fp32_GBps"] = round(nbytes / (statistics.median(tt) * 1e-3) / 1e9, 1)
    # read-only ceiling (bandwidth proxy)
    g = 4 * dev["cus"]
    tt, _ = time_steps(lambda: R.red_bw_proxy(xt.data_ptr(), nbytes, g, 512, sh), 50, stream)
    extra["bw_proxy_GBps"] = round(nbytes / (statistics.median(tt) * 1e-3) / 1e9, 1)

    # ---- synchronization latencies (ns)
    if not args.no_probes:
        cus = dev["cus"]
        gb = {}
        for n_wg in (cus, 2 * cus):
            ns, sg, wall_ns = R.sync_bench_grid(min(n_wg, R.red_max_coresident(256)), 256, reps=20)
            gb[str(n_wg)] = {"ns": round(ns, 1), "sigma_ns": round(sg, 1), "in_kernel_ns": round(wall_ns, 1)}
        ro, ro_sg, null_ns = R.sync_bench_relaunch(cus, 256, cooperative=False, reps=20)
        rc, rc_sg, null_c = R.sync_bench_relaunch(cus, 256, cooperative=True, reps=20)
        extra["grid_barrier_ns"] = gb
        extra["relaunch_overhead_ns"] = {"traditional": round(ro, 1), "traditional_sigma": round(ro_sg, 1),
                                         "cooperative": round(rc, 1), "cooperative_sigma": round(rc_sg, 1),
                                         "null_kernel_total_ns": round(null_ns, 1),
                                         "null_kernel_total_coop_ns": round(null_c, 1)}

    # ---- correctness of the timed result and the CPU oracle baseline
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ts = []
        ex = None
        for _ in range(3):
            c0 = time.perf_counter()
            ex = oracle.exact_sum(x, "f32")
            ts.append(time.perf_counter() - c0)
        t_cpu = statistics.median(ts)
        extra["rel_err_vs_exact"] = oracle.rel_err(result, ex)
        cpu = {"value": round(nbytes / t_cpu / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": "the full 2^28-element fp32 input, exact exponent-binned sum (median of 3 runs, "
                         "%.2f s each)" % t_cpu}

    roof = {"bound": "hbm", "achieved": round(kernel_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(kernel_gbps / HBM_PEAK_GBPS, 4), "traffic": traffic_per_launch()}
    rec = {
        "metric": METRIC,
        "value": round(gbps, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fp32 sum of 2^28 N(0,1) values (1 GiB), compensated fp32 + fp64 final combine",
                   "n": N, "bytes": nbytes, "plan": plan.as_dict()},
        "pct_hbm_peak": round(100.0 * gbps / HBM_PEAK_GBPS, 2),
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
