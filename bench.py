#!/usr/bin/env python3
"""Benchmark of the device-wide fp32 sum reduction on one MI355X.

Workload: the sum of 2^28 fp32 values drawn N(0,1) (1 GiB, resident in HBM
before timing starts), TwoSum-compensated fp32 accumulation with a binary64
final combine, launched with the tuned plan (from the committed plan cache,
or tuned on the spot).  One step = one call of red_sum over the whole array
(per-thread accumulation, wavefront and workgroup combines, device-wide
synchronization, final combine).

Prints ONE JSON line: GB/s (= 2^30 bytes / wall time per step) and the
fraction of the 8 TB/s HBM peak; the roofline of the dominant (streaming)
kernel from its own HIP-event durations; the grid-barrier and relaunch
latencies, the other synchronization variants and the bandwidth-proxy
ceiling; one figure each for the segmented batch (10,000 log-uniform
segments) and the iterative stencil (4M values); the error of the result
against the exact CPU oracle and the oracle's own CPU time.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20]
    python bench.py --configs out.jsonl [--only-configs]   # every workload + probe sweeps
    python bench.py --retune --save-plans plans.json        # re-run the autotuner
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
# Sources of the dominant streaming kernel (the traffic summary is tied to them).
KERNEL_SOURCES = ("device_prims.h", "reduce.hip")
# The timed loop records kernel events on every timer_period(steps)-th
# step: at least this many launches of the dominant kernel are timed.
KERNEL_LAUNCHES_TIMED = 10


def timer_period(steps: int) -> int:
    return max(1, steps // KERNEL_LAUNCHES_TIMED)



def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch(plan_dict):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if it is absent, was taken on a
    different kernel source, or on a different plan."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("plan") != plan_dict:
        return None
    return d.get("bytes_per_launch")


VARIANT_KERNELS = {"relaunch": "k_partials", "atomic": "k_atomic", "persistent": "k_persistent",
                   "single": "k_single"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
GIB_KIB = float(1 << 20)  # 1 GiB in KiB


def dominant_kernel_name(plan_dict) -> str:
    """Full name, as the profiler prints it, of the kernel that streams the
    fp32 compensated input under `plan_dict`."""
    f = int(plan_dict.get("flags", 0))
    return "void redsum::%s<redsum::ModeF32Comp, %d, %s, %s>(redsum::ReduceArgs)" % (
        VARIANT_KERNELS[plan_dict["variant"]], int(plan_dict["ipt"]), "true" if f & 1 else "false",
        "true" if f & 8 else "false")


def last_json_line(path):
    with open(path) as fh:
        return json.loads([l for l in fh.read().splitlines() if l.startswith("{")][-1])


def counter_values(path, counter):
    """{kernel name: [per-dispatch values]} from a rocprofv3 counter CSV."""
    import csv
    vals = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return vals


def summarize_pmc(fetch_dir, write_dir, bench_json, out_dir):
    """HBM traffic per launch of the dominant kernel from two rocprofv3
    --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by
    the same counter on the 1 GiB device-to-device copies of the same run
    (2^30 bytes read and written).  Writes hbm_traffic_f32_2p28.{json,md}."""
    line = last_json_line(bench_json)
    plan = line["config"]["plan"]
    name = dominant_kernel_name(plan)
    fetch = counter_values(os.path.join(fetch_dir, "run_counter_collection.csv"), "FETCH_SIZE")
    write = counter_values(os.path.join(write_dir, "run_counter_collection.csv"), "WRITE_SIZE")
    kf, kw = fetch[name], write[name]
    # the calibration copies are the 1 GiB ones (other copies move a few bytes)
    cf = [v for v in fetch[COPY_KERNEL] if v > GIB_KIB / 4]
    cw = [v for v in write[COPY_KERNEL] if v > GIB_KIB / 4]
    if not (kf and kw and cf and cw):
        raise SystemExit("counter runs hold no dominant-kernel or 1 GiB copy dispatches")
    f_kib, w_kib = statistics.mean(kf), statistics.mean(kw)
    f_scale, w_scale = GIB_KIB / statistics.median(cf), GIB_KIB / statistics.median(cw)
    traffic = int(round((f_kib * f_scale + w_kib * w_scale) * 1024))
    algo = N * 4 + 8 * int(plan["grid"]) + 8
    cmd = ("rocprofv3 --pmc %s --output-format csv -d <dir> -o run -- python3 bench.py --steps 5 --warmup 2 "
           "--no-cpu-baseline --no-probes --calibrate-copy")
    doc = {"kernel": name, "workload": "fp32 sum of 2^28 N(0,1) values (1 GiB)", "plan": plan,
           "kernel_source_hash": kernel_source_hash(),
           "fetch_kib_per_launch": round(f_kib, 1), "write_kib_per_launch": round(w_kib, 1),
           "launches": [len(kf), len(kw)],
           "calibration": {"kernel": COPY_KERNEL + ", 1 GiB device-to-device copy (torch copy_)",
                           "fetch_kib": round(statistics.median(cf), 1), "write_kib": round(statistics.median(cw), 1),
                           "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5)},
           "bytes_per_launch": traffic, "algorithmic_bytes_per_launch": algo,
           "traffic_over_algorithmic": round(traffic / algo, 5),
           "commands": [cmd % "FETCH_SIZE", cmd % "WRITE_SIZE",
                        "python3 bench.py --summarize-pmc <fetch dir> <write dir> <bench line of the fetch run>"]}
    with open(os.path.join(out_dir, "hbm_traffic_f32_2p28.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    md = ["# HBM traffic: fp32 2^28 compensated sum, dominant kernel", "",
          "Commands (two counter passes, then the summary; repository root):", "", "```"] + doc["commands"] + [
          "```", "",
          "Kernel `%s`, plan `%s`, %d launches per pass." % (name, json.dumps(plan), len(kf)), "",
          "| Counter | Kernel (KiB/launch) | 1 GiB copy (KiB/dispatch) | Scale | Kernel, scaled (KiB) |",
          "|---|---|---|---|---|",
          "| FETCH_SIZE | %.1f | %.1f | %.5f | %.1f |" % (f_kib, statistics.median(cf), f_scale, f_kib * f_scale),
          "| WRITE_SIZE | %.1f | %.1f | %.5f | %.1f |" % (w_kib, statistics.median(cw), w_scale, w_kib * w_scale),
          "",
          "- The calibration copy is torch's 1 GiB device-to-device `copy_` (`%s`), which reads and" % COPY_KERNEL,
          "  writes exactly 1,048,576 KiB. Each counter is scaled by what it reads for that copy.",
          "- Traffic per launch: %d bytes against %d algorithmic bytes (2^30 input, %d partials of 8 B, 8 B"
          % (traffic, algo, int(plan["grid"])),
          "  output): **%.5fx**." % (traffic / algo),
          "- `hbm_traffic_f32_2p28.json` holds these figures with the hash of the kernel's sources; `bench.py`",
          "  reports `roofline.traffic` only while the sources and the plan still match."]
    with open(os.path.join(out_dir, "hbm_traffic_f32_2p28.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    log("traffic %d B per launch (%.5fx algorithmic)" % (traffic, traffic / algo))


def summarize_trace(trace_dir, bench_json, out_dir, plain_json=None):
    """Kernel-trace summary of a profiled bench run: the per-kernel
    statistics of rocprofv3 --kernel-trace --stats beside the bench line's
    own event timing of the dominant kernel."""
    import csv
    line = last_json_line(bench_json)
    plan = line["config"]["plan"]
    name = dominant_kernel_name(plan)
    with open(os.path.join(trace_dir, "run_kernel_stats.csv")) as fh:
        rows = list(csv.DictReader(fh))
    dom = [r for r in rows if r["Name"] == name]
    if not dom:
        raise SystemExit("kernel stats hold no dispatch of " + name)
    avg_ns = float(dom[0]["AverageNs"])
    algo = N * 4 + 8 * int(plan["grid"]) + 8
    md = ["# Kernel trace: fp32 2^28 compensated sum (headline workload)", "",
          "Command (repository root, plans from `paper_2004_05371_amd/tuned_plans.json`), then the summary:", "",
          "```", "rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- python3 bench.py",
          "python3 bench.py --summarize-trace <dir> <bench line of that run> [<bench line of a run of python3 bench.py>]",
          "```", "",
          "Device: %s. Plan `%s`." % ("MI355X (gfx950, 256 CUs, 8 XCDs)", json.dumps(plan)), "",
          "| Kernel | Calls | Average (us) | Min (us) | Max (us) |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        k = r["Name"].replace("|", "/")
        if len(k) > 95:
            k = k[:92] + "..."
        md.append("| `%s` | %s | %.2f | %.2f | %.2f |" % (k, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                          float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    md += ["",
           "- Dominant kernel `%s`: %s launches (timed loop, warm-up, variant table), average **%.2f us** ="
           % (name.split("(")[0].replace("void redsum::", ""), dom[0]["Calls"], avg_ns / 1e3),
           "  %.1f GB/s for %d algorithmic bytes (%.1f %% of 8 TB/s)."
           % (algo / avg_ns, algo, 100 * algo / avg_ns / 8000),
           "- The bench line of the same run: HIP events carried by that kernel's dispatch on its stream, mean %.2f us"
           % line["extra"]["dominant_kernel_mean_us"],
           "  (roofline.achieved %.1f GB/s); wall rate %.1f GB/s." % (line["roofline"]["achieved"], line["value"])]
    if plain_json:
        plain = last_json_line(plain_json)
        md += ["- The same command without the profiler (a separate run): events mean %.2f us, roofline.achieved"
               " %.1f GB/s (frac %.4f); the profiler adds time to the events of every dispatch."
               % (plain["extra"]["dominant_kernel_mean_us"], plain["roofline"]["achieved"],
                  plain["roofline"]["frac"])]
    md += [
           "- Other rows come from the variant table and the probes of the same bench run."]
    with open(os.path.join(out_dir, "k_partials_f32_2p28_kernel_trace.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    log("dominant kernel %.2f us average over %s launches" % (avg_ns / 1e3, dom[0]["Calls"]))
    summarize_extensions(rows, line, out_dir)


def summarize_configs(paths, out_dir):
    """Write profiles/sync_characterization.md from the probe records of
    `bench.py --configs` runs (Sections IV, V and IX: every level of the
    synchronization hierarchy, Tables I, II and V and the grid-barrier heat
    map)."""
    recs = []
    for p in paths:
        with open(p) as fh:
            recs += [json.loads(l) for l in fh if l.strip()]
    machine = next((r for r in recs if r.get("config") == "machine"), None)
    by = lambda kind: [r for r in recs if r.get("probe") == kind]
    out = ["# Synchronization characterization: MI355X (gfx950), one GPU", "",
           "Commands (repository root), then the summary:", "", "```",
           "python3 bench.py --only-configs --configs <jsonl> --config-sections machine,probes",
           "python3 bench.py --summarize-configs <jsonl>", "```", ""]
    if machine:
        d = machine["device"]
        out += ["Device: %d CUs, %d XCDs, shader clock %.2f GHz, wall clock %d kHz; host CPUs %s." %
                (d["cus"], d["nxcc"], d["clock_khz"] / 1e6, d["wallclock_khz"], machine.get("host_cpus")), ""]
    out += ["Latencies are the Eq. 7 differential between kernels of r1 and r2 repetitions (host-side HIP events), "
            "sigma by Eq. 8; cycles are the in-kernel shader clock per operation (Section IX-C's method). "
            "Block throughput is measured as barriers completed in a 200 us window by every co-resident workgroup.",
            ""]
    w = by("wave")
    if w:
        out += ["## Wavefront combines (Section VII-D, Table V)", "",
                "| Op | Type | ns | sigma ns | cycles |", "|---|---|---|---|---|"]
        out += ["| %s | %s | %.2f | %.2f | %.1f |" % (r["op"], r["type"], r["ns"], r["sigma_ns"], r["cycles"]) for r in w]
        out.append("")
    b = by("block")
    if b:
        out += ["## Workgroup barrier latency (Section V, Table II)", "",
                "| Threads per WG | Workgroups | Waves per CU | ns | sigma ns | cycles |", "|---|---|---|---|---|---|"]
        out += ["| %d | %d | %.2f | %.2f | %.2f | %.1f |" % (r["wg"], r["n_wg"], r["waves_per_cu"], r["ns"], r["sigma_ns"],
                                                         r["cycles"]) for r in b]
        out.append("")
    t = by("block_tput")
    if t:
        out += ["## Workgroup barrier throughput under load, measured (Section V, Table II)", "",
                "| Threads per WG | WGs per CU | Waves per CU | Barriers per us per CU | Cycles per barrier (one WG) |",
                "|---|---|---|---|---|"]
        out += ["| %d | %d | %d | %.1f | %.1f |" % (r["wg"], r["wg_per_cu"], r["waves_per_cu"], r["barriers_per_us_per_cu"],
                                                 r["cycles_per_barrier"]) for r in t]
        out.append("")
    g = by("grid")
    if g:
        out += ["## Grid barrier heat map (Section V, grid synchronization)", "",
                "Latency of one grid barrier in ns, by grid size (rows) and workgroup size (columns), one table per "
                "barrier shape: flat (one counter), 8 groups and the default two-level shape (groups of blockIdx mod "
                "g), and the XCD-aggregated shape; then the default and XCD shapes of the barrier for published data "
                "(values stored and loaded with device-scope atomics: no L2 write-back at arrival, no invalidation "
                "after the wait).", ""]
        wgs = sorted({r["wg"] for r in g})
        titles = {"1": "flat", "8": "8 groups", "default_published": "default, published data",
                  "xcd_published": "xcd, published data"}
        for shape in ("1", "8", "default", "xcd", "default_published", "xcd_published"):
            rows = [r for r in g if str(r["groups"]) == shape]
            if not rows:
                continue
            out += ["### Shape: %s" % titles.get(shape, shape), "",
                    "| Workgroups | " + " | ".join("%d threads (WG/CU)" % x for x in wgs) + " |",
                    "|---|" + "---|" * len(wgs)]
            for n in sorted({r["n_wg"] for r in rows}):
                cells = []
                for x in wgs:
                    m = [r for r in rows if r["n_wg"] == n and r["wg"] == x]
                    cells.append("%.0f (%.2f)" % (m[0]["ns"], m[0]["wg_per_cu"]) if m else "-")
                out.append("| %d | %s |" % (n, " | ".join(cells)))
            out.append("")
    rl = by("relaunch")
    if rl:
        out += ["## Kernel boundary (Section IV, Table I; Eq. 6)", "",
                "| Launch | Workgroups | Overhead ns (Eq. 6) | sigma ns | Null kernel ns |", "|---|---|---|---|---|"]
        out += ["| %s | %d | %.1f | %.1f | %.1f |" % (r["launch"], r["n_wg"], r["overhead_ns"], r["sigma_ns"],
                                                  r["null_kernel_total_ns"]) for r in rl]
        out += ["", "Null kernel: the Section IV host-clock formula for ordinary and cooperative launches (median over "
                "the repetitions); for the graph type, the Eq. 7 differential between graphs of 40 and 5 null "
                "kernels.", ""]
        ordinary = {r["n_wg"]: r["overhead_ns"] for r in rl if r["launch"] == "ordinary"}
        if ordinary and g:
            out += ["## Grid barrier against a kernel boundary", "",
                    "| Workgroups (256 threads) | Barrier shape | Barrier ns | Ordinary launch overhead ns | Difference ns |",
                    "|---|---|---|---|---|"]
            for n, ov in sorted(ordinary.items()):
                for r in g:
                    if r["wg"] == 256 and r["n_wg"] == n:
                        out.append("| %d | %s | %.0f | %.0f | %.0f |" % (n, r["groups"], r["ns"], ov, r["ns"] - ov))
            out.append("")
    path = os.path.join(out_dir, "sync_characterization.md")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    log("wrote", path)


def summarize_extensions(rows, line, out_dir):
    """Kernel-trace rows of the extension figures of the same bench run:
    the segmented batch (slice kernel and fix-up) and the stencil."""
    seg = line.get("extra", {}).get("segmented_10000")
    st = line.get("extra", {}).get("stencil_4M")
    if not seg or not st:
        return
    pick = [r for r in rows if "k_segmented<" in r["Name"] or "k_seg_fixup" in r["Name"]
            or "k_jacobi" in r["Name"] or "k_copy_f32" in r["Name"]]
    if not pick:
        return
    seg_bytes = seg["values"] * 4 + (seg["segments"] + 1) * 8 + seg["segments"] * 8
    md = ["# Kernel trace: segmented batch and iterative stencil (extension figures of the bench line)", "",
          "Same command and run as `k_partials_f32_2p28_kernel_trace.md`:", "",
          "```", "rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- python3 bench.py",
          "python3 bench.py --summarize-trace <dir> <bench line of that run>", "```", "",
          "Workloads: %d fp32 values in %d log-uniform segments, plan `%s` (graph replay and direct "
          "launches); a 1D Jacobi stencil on %d values, %d steps per call, one launch per step and "
          "the persistent form with a grid barrier every 32 steps, and every k steps for the halo "
          "width k the library picks."
          % (seg["values"], seg["segments"], json.dumps(seg["plan"]), st["n"], st["steps"]), "",
          "| Kernel | Calls | Average (us) | Min (us) | Max (us) |", "|---|---|---|---|---|"]
    for r in pick:
        k = r["Name"].replace("|", "/")
        md.append("| `%s` | %s | %.2f | %.2f | %.2f |" % (k[:95], r["Calls"], float(r["AverageNs"]) / 1e3,
                                                          float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    # the slice kernel of the bench plan: k_segmented<ipt, nontemporal, fix-up>
    fix = {"atomic": 0, "persistent": 1, "relaunch": 2}.get(seg["plan"]["variant"], 2)
    tmpl = "k_segmented<%d, %s, %d>" % (seg["plan"]["ipt"], "true" if seg["plan"]["flags"] & 1 else "false", fix)
    sk = [r for r in pick if tmpl in r["Name"]]
    fx = [r for r in pick if "k_seg_fixup" in r["Name"]] if fix == 2 else []
    if sk:
        a = float(sk[0]["AverageNs"])
        md += ["", "- Slice kernel: average %.1f us = %.1f GB/s for %d algorithmic bytes (values, offsets, "
               "outputs; %.1f %% of 8 TB/s)%s." % (a / 1e3, seg_bytes / a, seg_bytes, 100 * seg_bytes / a / 8000,
                                                   "; fix-up kernel %.2f us" % (float(fx[0]["AverageNs"]) / 1e3)
                                                   if fx else ""),
               "- The bench line's own event timing of 20 back-to-back calls: %.1f us per call replayed from the "
               "graph, %.1f us launched directly." % (seg["graph_us"], seg["direct_us"])]
    md += ["- Stencil, from the bench line: %.3f us per step with one launch per step, %.3f us in the "
           "persistent form at k = 32%s." % (st["relaunch_us_per_step"], st["persistent_k32_us_per_step"],
                                             ", %.3f us with the library's halo" % st["persistent_auto_us_per_step"]
                                             if "persistent_auto_us_per_step" in st else ""),
           "- The bench-line figures of this run were taken under the profiler, which adds time to every "
           "launch (most visible in the one-launch-per-step stencil)."]
    with open(os.path.join(out_dir, "k_segmented_and_stencil_kernel_trace.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")


def gbps(nbytes, ms):
    return round(nbytes / (ms * 1e-3) / 1e9, 1)


def time_steps(fn, steps, stream):
    """Per-step HIP event times (ms) on `stream` over `steps` calls, and
    the wall time of the whole loop (s)."""
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


def time_loop(fn, steps, stream):
    """Mean HIP event time (ms) per call of `steps` back-to-back calls on
    `stream`, between one pair of events."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


class Flusher:
    """Read-only pass over a 1 GiB buffer before a timed call, so the 256 MB
    memory-side cache holds none of the input (reads leave clean lines, so
    no write-back competes with the timed call)."""

    def __init__(self, R, sh):
        import torch
        self.R, self.sh = R, sh
        self.buf = torch.empty(1 << 28, dtype=torch.float32, device="cuda")

    def __call__(self):
        self.R.red_bw_proxy(self.buf.data_ptr(), self.buf.numel() * 4, 1024, 512, self.sh)


def time_flushed(fn, reps, stream, flush):
    import torch
    out = []
    for _ in range(reps):
        flush()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def variant_table(R, plan, dtype, xt, n, out, sh, stream, dev, reps=50, flush=None):
    """GB/s (median of `reps` event-timed calls) of every synchronization
    variant with the plan's workgroup size, loads per thread and flags."""
    nbytes = xt.numel() * xt.element_size()
    nt = plan.flags & (R.FLAG_NONTEMPORAL | R.FLAG_PIPELINE)
    coresident = R.red_max_coresident(plan.wg)
    g = plan.grid or min(4 * dev["cus"], coresident)
    cands = {
        "relaunch": R.make_opts(variant=1, wg=plan.wg, ipt=plan.ipt, grid=plan.grid, flags=nt),
        "atomic": R.make_opts(variant=2, wg=plan.wg, ipt=plan.ipt, grid=plan.grid, flags=nt),
        "atomic_xcd": R.make_opts(variant=2, wg=plan.wg, ipt=plan.ipt, grid=plan.grid, flags=nt | R.FLAG_XCD),
        "persistent_cooperative": R.make_opts(variant=3, wg=plan.wg, ipt=plan.ipt, grid=min(g, coresident),
                                              flags=nt),
        "persistent_plain_launch": R.make_opts(variant=3, wg=plan.wg, ipt=plan.ipt, grid=min(g, coresident),
                                               flags=nt | R.FLAG_PLAIN_LAUNCH),
        "persistent_xcd_plain_launch": R.make_opts(variant=3, wg=plan.wg, ipt=plan.ipt, grid=min(g, coresident),
                                                   flags=nt | R.FLAG_PLAIN_LAUNCH | R.FLAG_XCD),
    }
    if nbytes <= (64 << 20):
        cands["single_workgroup"] = R.make_opts(variant=4, wg=1024, ipt=2, grid=1)
    res = {}
    for name, o in cands.items():
        fn = (lambda o=o: R.red_sum_ex(dtype, xt.data_ptr(), n, out.data_ptr(), sh, o))
        for _ in range(3):
            fn()
        if flush is None:
            tt, _ = time_steps(fn, reps, stream)
        else:
            tt = time_flushed(fn, reps, stream, flush)
        res[name] = gbps(nbytes, statistics.median(tt))
    if R.red_check_error(sh) != R.RED_OK:
        res["error"] = R.last_error()
    return res


class Plans:
    """Plans from the committed cache, or tuned now (and recorded)."""

    def __init__(self, R, retune: bool):
        from paper_2004_05371_amd import autotune
        self.R, self.at, self.retune = R, autotune, retune
        self.keys = set() if retune else autotune.cached_keys()
        self.installed = 0 if retune else autotune.load()
        self.recorded = []

    def sum_plan(self, t, out, acc, sh):
        R, at = self.R, self.at
        code = R.dtype_code(t)
        inv = {v: k for k, v in at.DTYPES.items()}
        key = ("sum", inv[code], "plain" if acc == R.RED_ACC_PLAIN else "compensated", at.bucket(t.numel()))
        if key not in self.keys:
            self.recorded.append(at.tune_sum(t, out, acc, sh))
            self.keys.add(key)
        return R.red_get_plan(code, acc, t.numel())

    def seg_plan(self, xt, ot, out, sh):
        R, at = self.R, self.at
        nseg = ot.numel() - 1
        key = ("segmented", at.bucket(nseg))
        if key not in self.keys:
            self.recorded.append(at.tune_segmented(xt, ot, out, sh))
            self.keys.add(key)
        return R.red_get_segmented_plan(nseg)


def cpu_oracle_parallel(oracle, x, ex, nbytes):
    """The same oracle call on one contiguous chunk per host CPU, in threads
    (its C binning releases the GIL); the chunks' exact sums are added as
    integers and must equal the single-thread exact sum."""
    from concurrent.futures import ThreadPoolExecutor

    ncpu = len(os.sched_getaffinity(0))
    chunks = [c for c in np_split(x, ncpu) if c.size]
    with ThreadPoolExecutor(max_workers=ncpu) as pool:
        ts = []
        for _ in range(3):
            c0 = time.perf_counter()
            parts = list(pool.map(lambda c: oracle.exact_sum(c, "f32"), chunks))
            ts.append(time.perf_counter() - c0)
    same = (sum(p.num for p in parts) == ex.num and all(p.shift == ex.shift for p in parts)
            and sum(p.n_nan for p in parts) == ex.n_nan)
    t = statistics.median(ts)
    return {"value": round(nbytes / t / 1e9, 3), "unit": "GB/s", "threads": ncpu, "matches_single_thread": same,
            "sample": "the same 1 GiB input in %d contiguous chunks, one thread each, median of 3 runs of %.3f s"
                      % (len(chunks), t)}


def np_split(x, k):
    import numpy as np
    return np.array_split(x, k)


def other_configs(R, dev, stream, sh, plans, inputs):
    """One figure for each of the other workloads, with the cached plans:
    fp32 U[-1,1] and int32 U[-1000,1000] sums of 2^20 values (us per sum,
    back to back), the int32 2^26 sum through every synchronization variant
    (each checked bit for bit against numpy's int64 sum), and bf16 / fp16
    sums of 2^29 N(0,1) values drawn on the device from a fixed seed."""
    import numpy as np
    import torch
    res = {}
    for kind, x in (("f32", inputs.uniform_f32(1 << 20)), ("i32", inputs.uniform_i32(1 << 20))):
        t = torch.from_numpy(x).to("cuda")
        code = R.RED_F32 if kind == "f32" else R.RED_I32
        out = torch.empty((), dtype=torch.float64 if kind == "f32" else torch.int64, device="cuda")
        plan = plans.sum_plan(t, out, R.RED_ACC_COMPENSATED, sh)
        o = R.opts_from_plan(plan)
        fn = lambda: R.red_sum_ex(code, t.data_ptr(), t.numel(), out.data_ptr(), sh, o)
        for _ in range(20):
            fn()
        us = statistics.median(time_loop(fn, 32, stream) for _ in range(7)) * 1e3
        res["%s_2p20_us_per_sum" % kind] = round(us, 2)
        res["%s_2p20_plan" % kind] = plan.as_dict()
        if kind == "i32":
            res["i32_2p20_bit_exact"] = out.item() == int(x.astype(np.int64).sum())
    x = inputs.uniform_i32(1 << 26)
    t = torch.from_numpy(x).to("cuda")
    out = torch.empty((), dtype=torch.int64, device="cuda")
    plan = plans.sum_plan(t, out, R.RED_ACC_COMPENSATED, sh)
    res["i32_2p26_plan"] = plan.as_dict()
    res["i32_2p26_GBps"] = variant_table(R, plan, R.RED_I32, t, t.numel(), out, sh, stream, dev)
    want = int(x.astype(np.int64).sum())
    exact = {}
    for v in (1, 2, 3):
        R.red_sum_ex(R.RED_I32, t.data_ptr(), t.numel(), out.data_ptr(), sh,
                     R.make_opts(variant=v, wg=plan.wg, ipt=plan.ipt,
                                 grid=min(plan.grid or 1024, R.red_max_coresident(plan.wg))))
        torch.cuda.synchronize()
        exact[R.VARIANT_NAMES[v]] = out.item() == want
    res["i32_2p26_bit_exact"] = exact
    del t
    g = torch.Generator(device="cuda")
    for kind, tdt, code in (("bf16", torch.bfloat16, R.RED_BF16), ("f16", torch.float16, R.RED_F16)):
        g.manual_seed(2004 if kind == "bf16" else 5371)
        t = torch.randn(1 << 29, device="cuda", generator=g).to(tdt)
        out = torch.empty((), dtype=torch.float64, device="cuda")
        plan = plans.sum_plan(t, out, R.RED_ACC_COMPENSATED, sh)
        o = R.opts_from_plan(plan, acc=R.RED_ACC_COMPENSATED)
        fn = lambda: R.red_sum_ex(code, t.data_ptr(), t.numel(), out.data_ptr(), sh, o)
        for _ in range(3):
            fn()
        tt, _ = time_steps(fn, 30, stream)
        torch.cuda.synchronize()
        ref = float(t.double().sum())
        res["%s_2p29_GBps" % kind] = gbps(t.numel() * 2, statistics.median(tt))
        res["%s_2p29_plan" % kind] = plan.as_dict()
        res["%s_2p29_rel_diff_vs_torch_f64_sum" % kind] = abs(out.item() - ref) / max(abs(ref), 1e-300)
        del t
        torch.cuda.empty_cache()
    if R.red_check_error(sh) != R.RED_OK:
        raise RuntimeError("other configurations: " + R.last_error())
    return res


def stencil_configs(R, dev, stream, emit, timed):
    """Microseconds per step of the 1D Jacobi stencil: relaunch (one kernel
    per step, u and scratch through the caches / HBM every step) and the
    persistent form with a grid barrier every k steps; the forms' results
    are compared bit for bit on the GPU."""
    import torch

    from paper_2004_05371_amd import inputs

    sh = stream.cuda_stream
    forms = [("relaunch", R.RED_VARIANT_RELAUNCH, 0, 0), ("persistent_k1", R.RED_VARIANT_PERSISTENT, 1, 0),
             ("persistent_k8", R.RED_VARIANT_PERSISTENT, 8, 0), ("persistent_k32", R.RED_VARIANT_PERSISTENT, 32, 0),
             ("persistent_xcd_k8", R.RED_VARIANT_PERSISTENT, 8, R.FLAG_XCD),
             ("persistent_auto", R.RED_VARIANT_PERSISTENT, 0, 0)]
    for n in (1 << 16, 1 << 20, 1 << 22, 8_000_000):
        steps = 1000 if n <= (1 << 20) else 200
        x = torch.from_numpy(inputs.normal_f32(n, sub=66)).to("cuda")
        u = torch.empty_like(x)
        sc = torch.empty_like(x)
        rec = {"config": "stencil", "n": n, "steps": steps, "r": 0.25, "bytes_per_step_relaunch": 8 * n}
        results = {}
        for name, variant, k, flags in forms:
            o = R.make_opts(variant=variant, flags=flags)
            call = lambda: R.stencil_jacobi_1d(u.data_ptr(), sc.data_ptr(), n, steps, 0.25, k, sh, o)
            try:
                u.copy_(x)
                call()
                torch.cuda.synchronize()
                results[name] = u.clone()
                ms = timed(call, 5)
            except R.RedError as e:
                rec[name] = "refused: %s" % e
                continue
            rec[name + "_us_per_step"] = round(ms * 1e3 / steps, 3)
            rec[name + "_GBps_equiv"] = round(8 * n / (ms * 1e-3 / steps) / 1e9, 1)
        ref = results.get("relaunch")
        rec["forms_bit_identical"] = bool(ref is not None and all(torch.equal(ref, v) for v in results.values()))
        emit(rec)
        del x, u, sc, results
        torch.cuda.empty_cache()


def smi_query(args, limit=6000):
    """Output of one read-only amd-smi query as JSON (or its error text)."""
    import subprocess
    try:
        r = subprocess.run(["amd-smi"] + args + ["--json"], capture_output=True, text=True, timeout=30)
    except (OSError, subprocess.SubprocessError) as e:
        return {"error": str(e)}
    try:
        return json.loads(r.stdout)
    except ValueError:
        return {"rc": r.returncode, "stdout": r.stdout[:limit], "stderr": r.stderr[-limit // 4:]}


def time_gpu_side(fn, reps, stream):
    """Per-call device time (ms): each call is queued behind a short spin
    kernel, so the events around it measure the GPU's own latency, not the
    host's launch rate."""
    import torch
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in pairs:
        torch.cuda._sleep(50000)  # about 20 us of spinning
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in pairs]


def model_check(R, stream, emit, lo=10, hi=26):
    """Times one 1024-thread workgroup and the device-wide atomic-ticket
    and relaunch variants on fp32 inputs of 2^lo..2^hi elements (median
    device time per call), takes T and Thr for each as Eq. 1-2 define them,
    and compares the scenario rule's switch point (Section VII-A, Eq. 1-5)
    with the smallest measured size at which the device-wide kernel is
    faster."""
    import torch

    from paper_2004_05371_amd import inputs, model

    sh = stream.cuda_stream
    big = torch.from_numpy(inputs.normal_f32(1 << hi, sub=21)).to("cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    forms = {"single": R.make_opts(variant=R.RED_VARIANT_SINGLE, wg=1024, ipt=2, grid=1),
             "atomic": R.make_opts(variant=R.RED_VARIANT_ATOMIC, wg=256, ipt=4, grid=512, flags=R.FLAG_NONTEMPORAL),
             "relaunch": R.make_opts(variant=R.RED_VARIANT_RELAUNCH, wg=256, ipt=4, grid=512,
                                     flags=R.FLAG_NONTEMPORAL)}
    rows = []
    for lg in range(lo, hi + 1):
        n = 1 << lg
        row = {"n": n, "bytes": 4 * n}
        for name, o in forms.items():
            if name == "single" and lg > 22:
                continue  # one workgroup at 100 GB/s: beyond 16 MB only the slope matters
            call = lambda: R.red_sum_ex(R.RED_F32, big.data_ptr(), n, out.data_ptr(), sh, o)
            for _ in range(3):
                call()
            row[name] = statistics.median(time_gpu_side(call, 50 if lg <= 20 else 10, stream)) * 1e3  # us
        rows.append(row)
        emit({"config": "model_sweep", **{k: (round(v, 3) if isinstance(v, float) else v) for k, v in row.items()}})
    # Eq. 1-2 give t(N) = max(T, N / Thr) (T + max(0, N - C) / Thr with
    # C = T Thr): T is the time of the smallest inputs, Thr the slope
    # between the two largest measured sizes.
    fit = {}
    for name in forms:
        pts = [r for r in rows if name in r]
        t0 = min(r[name] for r in pts[:3])
        slope = (pts[-1][name] - pts[-2][name]) / (pts[-1]["bytes"] - pts[-2]["bytes"])  # us per byte
        fit[name] = {"T_us": round(t0, 3), "Thr_GBps": round(1e-3 / slope, 1)}
    pred = {}
    for more in ("atomic", "relaunch"):
        tb, tm = fit["single"]["T_us"], fit[more]["T_us"]
        pred[more] = model.switch_point(tb, max(0.0, tm - tb), fit["single"]["Thr_GBps"] * 1e3,
                                        fit[more]["Thr_GBps"] * 1e3)
    meas = {more: next((r["bytes"] for r in rows if "single" in r and r[more] < r["single"]), None)
            for more in ("atomic", "relaunch")}
    emit({"config": "model", "fit": fit,
          "switch_bytes_predicted": {k: round(v) for k, v in pred.items()},
          "first_power_of_two_where_device_wide_wins_bytes": meas,
          "library_switch_bytes": round(model.mi355x_single_workgroup_switch()),
          "note": "2^%d..2^%d fp32 elements, device time per call; T = time of the smallest inputs, "
                  "Thr = slope over the two largest" % (lo, hi)})
    del big


CONFIG_SECTIONS = ("machine", "small", "int", "f32", "half", "segments", "uniform", "stencil", "model", "probes")


def run_configs(R, dev, stream, path, plans, sections=CONFIG_SECTIONS):
    """Every workload of the study, one JSON record per measurement,
    appended to `path` (JSONL).  Timed regions hold only library calls; the
    oracle timings and errors are the CPU-baseline leg of each record.
    `sections` selects which of CONFIG_SECTIONS run."""
    import numpy as np
    import torch

    import oracle
    from paper_2004_05371_amd import inputs

    sh = stream.cuda_stream
    flush = Flusher(R, sh)

    def emit(rec):
        log(json.dumps(rec))
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")

    last = {}  # statistics of the latest timed() call, in microseconds

    def timed(fn, reps, flushed=False):
        for _ in range(3):
            fn()
        if flushed:
            tt = time_flushed(fn, reps, stream, flush)
        else:
            tt, _ = time_steps(fn, reps, stream)
        last.clear()
        last.update(median=round(statistics.median(tt) * 1e3, 2), min=round(min(tt) * 1e3, 2),
                    sigma=round(statistics.stdev(tt) * 1e3, 3) if len(tt) > 1 else 0.0, reps=len(tt))
        return statistics.median(tt)

    def cpu_exact(x, kind):
        c0 = time.perf_counter()
        ex = oracle.exact_sum(x, kind) if kind != "i32" else oracle.sum_i32(x)
        return ex, time.perf_counter() - c0

    def sec_machine():
        # -- the machine: device properties, partition mode, clocks and power
        #    (amd-smi, read-only queries), host CPUs available to this process
        emit({"config": "machine", "device": dev, "host_cpus": len(os.sched_getaffinity(0)),
              "amd_smi": {k: smi_query(v) for k, v in (("partition", ["static", "--partition"]),
                                                       ("clock_power", ["metric", "--clock", "--power"]))}})

    def sec_small():
        # -- small: 2^20 fp32 U[-1,1] and int32 U[-1000,1000]; the two-launch
        #    variant, and the tuned plan
        for kind, x in (("f32", inputs.uniform_f32(1 << 20)), ("i32", inputs.uniform_i32(1 << 20))):
            t = torch.from_numpy(x).to("cuda")
            code = R.RED_F32 if kind == "f32" else R.RED_I32
            out = torch.empty((), dtype=torch.float64 if kind == "f32" else torch.int64, device="cuda")
            o = R.make_opts(variant=R.RED_VARIANT_RELAUNCH)
            fn = lambda: R.red_sum_ex(code, t.data_ptr(), t.numel(), out.data_ptr(), sh, o)
            warm, cold = timed(fn, 200), timed(fn, 50, flushed=True)
            dev_t = statistics.median(time_gpu_side(fn, 100, stream))
            plan = plans.sum_plan(t, out, R.RED_ACC_COMPENSATED, sh)
            ot = R.opts_from_plan(plan)
            tuned = timed(lambda: R.red_sum_ex(code, t.data_ptr(), t.numel(), out.data_ptr(), sh, ot), 200)
            fn()
            torch.cuda.synchronize()
            ex, tc = cpu_exact(x, kind)
            ok = (out.item() == ex) if kind == "i32" else (oracle.rel_err(out.item(), ex) <= 1e-6)
            emit({"config": "small", "dtype": kind, "n": x.size, "variant": "relaunch", "us_warm": round(warm * 1e3, 2),
                  "us_device": round(dev_t * 1e3, 2),
                  "us_flushed": round(cold * 1e3, 2), "tuned_plan": plan.as_dict(), "us_tuned": round(tuned * 1e3, 2),
                  "matches_oracle": bool(ok), "cpu_oracle_s": round(tc, 4)})

    def sec_int():
        # -- int: 2^26 int32, three synchronization variants, flushed and warm
        x = inputs.uniform_i32(1 << 26)
        t = torch.from_numpy(x).to("cuda")
        out = torch.empty((), dtype=torch.int64, device="cuda")
        plan = plans.sum_plan(t, out, R.RED_ACC_COMPENSATED, sh)
        warm = variant_table(R, plan, R.RED_I32, t, t.numel(), out, sh, stream, dev)
        cold = variant_table(R, plan, R.RED_I32, t, t.numel(), out, sh, stream, dev, reps=30, flush=flush)
        exact, tc = cpu_exact(x, "i32")
        bit_exact = {}
        for v in (1, 2, 3):
            R.red_sum_ex(R.RED_I32, t.data_ptr(), t.numel(), out.data_ptr(), sh,
                         R.make_opts(variant=v, wg=plan.wg, ipt=plan.ipt,
                                     grid=min(plan.grid or 1024, R.red_max_coresident(plan.wg))))
            torch.cuda.synchronize()
            bit_exact[R.VARIANT_NAMES[v]] = out.item() == exact
        emit({"config": "int", "dtype": "i32", "n": x.size, "plan": plan.as_dict(), "GBps_warm": warm,
              "GBps_flushed": cold, "bit_exact": bit_exact, "cpu_oracle_s": round(tc, 4)})
        del t

    def sec_f32():
        # -- f32: 2^28 in two distributions, plain vs compensated
        for gen in ("normal", "mixed"):
            x = inputs.normal_f32(1 << 28) if gen == "normal" else inputs.mixed_f32(1 << 28)
            t = torch.from_numpy(x).to("cuda")
            out = torch.empty((), dtype=torch.float64, device="cuda")
            ex, tc = cpu_exact(x, "f32")
            absx = float(oracle.exact_abs_sum(x, "f32").fraction)
            for acc, name in ((0, "compensated"), (1, "plain")):
                plan = plans.sum_plan(t, out, acc, sh)
                o = R.opts_from_plan(plan, acc=acc)
                ms = timed(lambda: R.red_sum_ex(R.RED_F32, t.data_ptr(), t.numel(), out.data_ptr(), sh, o), 50)
                stats = dict(last)
                torch.cuda.synchronize()
                r = out.item()
                emit({"config": "f32", "dist": gen, "acc": name, "n": x.size, "plan": plan.as_dict(),
                      "GBps": gbps(x.nbytes, ms), "timing_us": stats, "rel_err": oracle.rel_err(r, ex),
                      "err_over_sum_abs": abs(float(ex.fraction) - r) / absx, "cpu_oracle_s": round(tc, 3)})
            del t

    def sec_half():
        # -- half: bf16 / fp16 2^29 N(0,1), compensated (and plain for contrast)
        for kind in ("bf16", "f16"):
            bits = inputs.normal_half_bits(1 << 29, kind)
            tdt = torch.bfloat16 if kind == "bf16" else torch.float16
            t = torch.from_numpy(bits.view(np.int16)).view(tdt).to("cuda")
            code = R.RED_BF16 if kind == "bf16" else R.RED_F16
            out = torch.empty((), dtype=torch.float64, device="cuda")
            ex, tc = cpu_exact(bits, kind)
            res = {}
            for acc, name in ((0, "compensated"), (1, "plain")):
                plan = plans.sum_plan(t, out, acc, sh)
                o = R.opts_from_plan(plan, acc=acc)
                ms = timed(lambda: R.red_sum_ex(code, t.data_ptr(), t.numel(), out.data_ptr(), sh, o), 50)
                torch.cuda.synchronize()
                res[name] = {"plan": plan.as_dict(), "GBps": gbps(bits.nbytes, ms), "timing_us": dict(last),
                             "Gelem_per_s": round(bits.size / (ms * 1e-3) / 1e9, 1),
                             "rel_err": oracle.rel_err(out.item(), ex)}
            emit({"config": "half", "dtype": kind, "n": bits.size, **res, "cpu_oracle_s": round(tc, 3)})
            del t
            torch.cuda.empty_cache()

    def sec_segments():
        # -- segmented: 10,000 log-uniform segments, one graph launch vs a loop;
        #    the drawn lengths (about 7.4e8 elements) and the same draws scaled
        #    to a total of about 2^28
        for label, total in (("segments", None), ("segments_2p28", 1 << 28)):
            x, off = inputs.segments(10000, total=total)
            xt = torch.from_numpy(x).to("cuda")
            ot = torch.from_numpy(off).to("cuda")
            nseg = off.size - 1
            out = torch.empty(nseg, dtype=torch.float64, device="cuda")
            plan = plans.seg_plan(xt, ot, out, sh)
            nbytes = x.nbytes + off.nbytes + out.numel() * 8
            ms_graph = timed(lambda: R.red_sum_segmented(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), sh), 30)
            graph_stats = dict(last)
            o = R.make_opts(variant=R.RED_VARIANT_PERSISTENT, wg=plan.wg, ipt=plan.ipt,
                            grid=min(plan.grid, R.red_max_coresident_segmented(plan.ipt, plan.wg)),
                            flags=R.FLAG_PLAIN_LAUNCH | (plan.flags & R.FLAG_NONTEMPORAL))
            ms_barrier = timed(lambda: R.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), sh, o),
                               30)
            fixups = {}
            for vname, v in (("relaunch", R.RED_VARIANT_RELAUNCH), ("ticket", R.RED_VARIANT_ATOMIC)):
                ov = R.make_opts(variant=v, wg=plan.wg, ipt=plan.ipt, grid=plan.grid, flags=plan.flags)
                fixups[vname] = round(timed(lambda: R.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg,
                                                                           out.data_ptr(), sh, ov), 30) * 1e3, 1)
            ms_loop = timed(lambda: R.red_sum_segmented_loop(xt.data_ptr(), off, nseg, out.data_ptr(), sh), 3)
            R.red_sum_segmented(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), sh)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            c0 = time.perf_counter()
            sums = oracle.segmented_sums(x, off)
            tc = time.perf_counter() - c0
            worst = max(oracle.rel_err(float(got[k]), e) if e.fraction != 0 else abs(got[k]) for k, e in enumerate(sums))
            emit({"config": label, "nseg": nseg, "total_elems": int(off[-1]), "bytes": nbytes, "plan": plan.as_dict(),
                  "graph_us": round(ms_graph * 1e3, 1), "graph_GBps": gbps(nbytes, ms_graph), "graph_timing_us": graph_stats,
                  "grid_barrier_fixup_us": round(ms_barrier * 1e3, 1), "plan_with_fixup_us": fixups,
                  "loop_per_segment_us": round(ms_loop * 1e3, 1), "speedup_vs_loop": round(ms_loop / ms_graph, 1),
                  "max_rel_err": worst, "cpu_oracle_s": round(tc, 2)})
            del xt, ot
            torch.cuda.empty_cache()

    def sec_uniform():
        # -- segmented batches of uniform lengths over 2^28 values: the cost of
        #    short segments, the slice granularity switch
        xs = torch.from_numpy(inputs.normal_f32(1 << 28, sub=3)).to("cuda")
        splan = dict(wg=512, ipt=4, grid=2 * dev["cus"])
        forms = {"workgroup": R.FLAG_SEG_WORKGROUP, "pieces": R.FLAG_SEG_PIECES, "runs": R.FLAG_SEG_RUNS}
        for L in (16, 32, 64, 256, 768, 1024, 4096, 16384, 65536, 262144, 1 << 28):
            nseg = (1 << 28) // L
            ntot = nseg * L
            offs = torch.arange(0, ntot + 1, L, dtype=torch.int64, device="cuda")
            outs = torch.empty(nseg, dtype=torch.float64, device="cuda")
            nb = ntot * 4 + (nseg + 1) * 8 + nseg * 8
            row = {}
            for fname, ff in [("auto", 0)] + list(forms.items()):
                if (fname == "workgroup" and L < 4096) or (fname == "pieces" and L < 64) or (fname == "runs" and L > 16384):
                    continue
                for vname, v in (("relaunch", R.RED_VARIANT_RELAUNCH), ("ticket", R.RED_VARIANT_ATOMIC)):
                    if fname != "auto" and vname == "ticket":
                        continue
                    o = R.make_opts(variant=v, flags=R.FLAG_NONTEMPORAL | ff, **splan)
                    ms = timed(lambda: R.red_sum_segmented_ex(xs.data_ptr(), offs.data_ptr(), nseg, outs.data_ptr(),
                                                              sh, o), 20)
                    row["%s_%s_us" % (fname, vname)] = round(ms * 1e3, 1)
            ms = row["auto_relaunch_us"] / 1e3
            ref = xs[:ntot].view(nseg, L).double().sum(1)  # torch check on the GPU (the oracle covers parity in the tests)
            emit({"config": "segments_uniform", "length": L, "nseg": nseg, "plan": splan, "us": row["auto_relaunch_us"],
                  "GBps": gbps(nb, ms), "by_form_and_fixup_us": row,
                  "form": "workgroup" if L >= 16384 else "runs" if L < 1024 else "pieces",
                  "max_abs_diff_vs_fp64_torch": float((outs - ref).abs().max())})
            del offs, outs, ref
        del xs
        torch.cuda.empty_cache()

    def sec_stencil():
        # -- iterative stencil: one launch per step against the time loop inside
        #    one persistent kernel (values kept in LDS across grid barriers)
        stencil_configs(R, dev, stream, emit, timed)

    def sec_model():
        # -- model: the Eq. 1-5 switch point between one workgroup ("basic")
        #    and the whole device ("more") from constants fitted on this GPU,
        #    against the crossover measured directly
        model_check(R, stream, emit)

    def sec_probes():
        # -- probes
        for vname, vt in R.WAVE_TYPES.items():
            for op, name in ((0, "dpp_reduce"), (1, "swizzle_reduce"), (2, "bpermute_reduce"), (3, "dpp_step")):
                ns, sg, cyc = R.sync_bench_wave_ex(op, vt, 64, reps=20)
                emit({"probe": "wave", "op": name, "type": vname, "ns": round(ns, 2), "sigma_ns": round(sg, 2),
                      "cycles": round(cyc, 1)})
        for wg in (64, 128, 256, 512, 1024):
            for n_wg in (1, dev["cus"], 4 * dev["cus"]):
                ns, sg, cyc = R.sync_bench_block(wg, n_wg, reps=20)
                # Table II's throughput view: barriers completed per CU per
                # microsecond with n_wg / cus resident workgroups per CU
                emit({"probe": "block", "wg": wg, "n_wg": n_wg, "waves_per_wg": wg // 64,
                      "waves_per_cu": round(n_wg / dev["cus"] * wg / 64, 2), "ns": round(ns, 2),
                      "sigma_ns": round(sg, 2), "cycles": round(cyc, 1),
                      "barriers_per_us_per_cu_from_latency": round(n_wg / dev["cus"] / (ns * 1e-3), 2)
                      if ns > 0 else None})
        # Table II's throughput, measured: barriers completed per CU per
        # microsecond with 1..8 co-resident workgroups per CU
        for wg in (64, 128, 256, 512, 1024):
            for k in (1, 2, 4, 8):
                if k * dev["cus"] > R.red_max_coresident(wg):
                    continue
                rate, cyc = R.sync_bench_block_tput(wg, k, window_ticks=20000)
                emit({"probe": "block_tput", "wg": wg, "wg_per_cu": k, "waves_per_cu": k * wg // 64,
                      "barriers_per_us_per_cu": round(rate, 2), "cycles_per_barrier": round(cyc, 1)})
        for wg in (64, 256, 1024):
            cores = R.red_max_coresident(wg)
            n = 1
            while n <= min(2048, cores):
                shapes = [(g, False) for g in ((1, 8, 0, -1) if n >= 64 else (1, -1))] + [(0, True), (-1, True)]
                for groups, pub in shapes:
                    if pub:
                        ns, sg, wall = R.sync_bench_grid_published(n, wg, groups, reps=20)
                    else:
                        ns, sg, wall = R.sync_bench_grid_ex(n, wg, groups, reps=20)
                    name = {0: "default", -1: "xcd"}.get(groups, groups)
                    emit({"probe": "grid", "wg": wg, "n_wg": n, "wg_per_cu": round(n / dev["cus"], 3),
                          "groups": "%s_published" % name if pub else name, "ns": round(ns, 1),
                          "sigma_ns": round(sg, 1), "in_kernel_ns": round(wall, 1)})
                n *= 2
        for kind, name in ((0, "ordinary"), (1, "cooperative"), (2, "graph")):
            for n_wg in (1, dev["cus"], 4 * dev["cus"]):
                if kind == 1 and n_wg > R.red_max_coresident(256):
                    continue
                ns, sg, null_ns = R.sync_bench_relaunch(n_wg, 256, cooperative=kind, reps=30)
                emit({"probe": "relaunch", "launch": name, "n_wg": n_wg, "overhead_ns": round(ns, 1),
                      "sigma_ns": round(sg, 1), "null_kernel_total_ns": round(null_ns, 1)})

    run = {"machine": sec_machine, "small": sec_small, "int": sec_int, "f32": sec_f32, "half": sec_half,
           "segments": sec_segments, "uniform": sec_uniform, "stencil": sec_stencil, "model": sec_model,
           "probes": sec_probes}
    for name in CONFIG_SECTIONS:
        if name in sections:
            log("configs section", name)
            run[name]()

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--configs", metavar="JSONL", help="also measure every workload and probe sweep into JSONL")
    ap.add_argument("--only-configs", action="store_true", help="skip the headline (with --configs)")
    ap.add_argument("--config-sections", default=",".join(CONFIG_SECTIONS),
                    help="comma-separated sections of --configs to run (default: all of %s)" % ",".join(CONFIG_SECTIONS))
    ap.add_argument("--summarize-configs", nargs="+", metavar="JSONL",
                    help="no GPU: write the synchronization characterization summary from configs records")
    ap.add_argument("--retune", action="store_true", help="ignore the plan cache and autotune")
    ap.add_argument("--save-plans", metavar="JSON", help="write the plans tuned in this run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the headline, copy the 1 GiB input 3 times (byte-counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "BENCH_JSON"),
                    help="no GPU: write the HBM traffic summary from two rocprofv3 --pmc runs")
    ap.add_argument("--summarize-trace", nargs="+", metavar="TRACE_DIR BENCH_JSON [PLAIN_BENCH_JSON]",
                    help="no GPU: write the kernel-trace summary of a profiled bench run (optionally beside "
                         "the bench line of a run without the profiler)")
    ap.add_argument("--summary-out", default=os.path.join(ROOT, "profiles"), metavar="DIR")
    args = ap.parse_args()
    if args.summarize_pmc or args.summarize_trace or args.summarize_configs:
        os.makedirs(args.summary_out, exist_ok=True)
        if args.summarize_configs:
            summarize_configs(args.summarize_configs, args.summary_out)
        if args.summarize_pmc:
            summarize_pmc(*args.summarize_pmc, args.summary_out)
        if args.summarize_trace:
            if len(args.summarize_trace) not in (2, 3):
                ap.error("--summarize-trace takes TRACE_DIR BENCH_JSON [PLAIN_BENCH_JSON]")
            summarize_trace(*args.summarize_trace[:2], args.summary_out,
                            args.summarize_trace[2] if len(args.summarize_trace) == 3 else None)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_05371_amd import autotune, inputs, redsum as R

    R.load()
    torch.cuda.set_device(0)
    R.red_init(0)
    dev = R.red_device_info()
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    plans = Plans(R, args.retune)
    log("device", dev, "cached plans installed:", plans.installed)

    if args.configs:
        sections = [x for x in args.config_sections.split(",") if x]
        bad = [x for x in sections if x not in CONFIG_SECTIONS]
        if bad:
            ap.error("unknown config sections %s" % bad)
        run_configs(R, dev, stream, args.configs, plans, sections)
    if not args.only_configs:
        headline(args, R, dev, stream, sh, plans, inputs)
    if args.save_plans and plans.recorded:
        autotune.save(plans.recorded, args.save_plans, cus=dev["cus"])
        log("saved %d plans to %s" % (len(plans.recorded), args.save_plans))


def headline(args, R, dev, stream, sh, plans, inputs):
    import torch

    # ---- input, resident in HBM before timing
    t0 = time.time()
    x = inputs.normal_f32(N)
    xt = torch.from_numpy(x).to("cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    log("input ready in %.1f s" % (time.time() - t0))
    nbytes = N * 4

    plan = plans.sum_plan(xt, out, R.RED_ACC_COMPENSATED, sh)
    log("plan", plan.as_dict())
    opts = R.opts_from_plan(plan, acc=R.RED_ACC_COMPENSATED)

    def step():
        R.red_sum_ex(R.RED_F32, xt.data_ptr(), N, out.data_ptr(), sh, opts)

    for _ in range(args.warmup):
        step()
    # Timed region: K steps between two synchronizations, with the library
    # timing the dominant kernel of every period-th step by HIP events
    # carried in its own dispatch (on the stream it runs on) for the roofline.
    torch.cuda.synchronize()
    period = timer_period(args.steps)
    R.red_kernel_timer(sh, period)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_mean_us, k_min_us, k_count = R.red_kernel_timer_read(sh)
    R.red_kernel_timer(sh, False)
    if k_count < min(KERNEL_LAUNCHES_TIMED, args.steps):
        raise RuntimeError("only %d launches of the dominant kernel were timed" % k_count)
    ms_per_step = wall * 1e3 / args.steps
    value = nbytes / (ms_per_step * 1e-3) / 1e9
    result = out.item()
    kernel_gbps = nbytes / (k_mean_us * 1e-6) / 1e9
    # The same loop without the dominant-kernel events, and with per-step
    # events (for reference only).
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    times, _ = time_steps(step, args.steps, stream)
    log("steps: wall %.4f ms/step (%.4f without kernel events), step events mean %.4f ms; "
        "dominant kernel mean %.2f us (min %.2f, %d launches)" %
        (ms_per_step, wall_plain * 1e3 / args.steps, statistics.fmean(times), k_mean_us, k_min_us, k_count))

    extra = {"GBps_without_kernel_events": round(nbytes / (wall_plain / args.steps) / 1e9, 1),
             "kernel_events_every_n_steps": period, "kernel_launches_timed": k_count,
             "step_event_mean_us": round(statistics.fmean(times) * 1e3, 2),
             "dominant_kernel_mean_us": round(k_mean_us, 2), "dominant_kernel_min_us": round(k_min_us, 2)}
    extra["variants_GBps"] = variant_table(R, plan, R.RED_F32, xt, N, out, sh, stream, dev)
    o = R.opts_from_plan(plan, acc=R.RED_ACC_PLAIN)
    tt, _ = time_steps(lambda: R.red_sum_ex(R.RED_F32, xt.data_ptr(), N, out.data_ptr(), sh, o), 50, stream)
    extra["plain_fp32_GBps"] = gbps(nbytes, statistics.median(tt))
    tt, _ = time_steps(lambda: R.red_bw_proxy(xt.data_ptr(), nbytes, 1024, 512, sh), 50, stream)
    extra["bw_proxy_GBps"] = gbps(nbytes, statistics.median(tt))
    # the same read-only loop with the nontemporal hint, in the headline plan's shape
    tt, _ = time_steps(lambda: R.red_bw_proxy_ex(xt.data_ptr(), nbytes, plan.grid or 512, plan.wg,
                                                 R.FLAG_NONTEMPORAL, sh), 50, stream)
    extra["bw_proxy_nt_GBps"] = gbps(nbytes, statistics.median(tt))

    # ---- synchronization latencies (ns)
    if not args.no_probes:
        cus = dev["cus"]
        gb = {}
        for n_wg in (cus, 2 * cus, 4 * cus):
            n = min(n_wg, R.red_max_coresident(256))
            # fenced barriers (ordinary data) at 1 and 4 workgroups per CU;
            # the barrier for published data (device-scope atomics) at 1, 2, 4
            shapes = ([(1, "flat", False), (0, "two_level", False), (-1, "xcd", False)] if n_wg != 2 * cus else [])
            for groups, name, pub in shapes + [(0, "two_level_published", True), (-1, "xcd_published", True)]:
                probe = R.sync_bench_grid_published if pub else R.sync_bench_grid_ex
                ns, sg, wall_ns = probe(n, 256, groups, reps=20)
                gb["%d_wg_%s" % (n, name)] = {"ns": round(ns, 1), "sigma_ns": round(sg, 1),
                                              "in_kernel_ns": round(wall_ns, 1)}
        ro, ro_sg, null_ns = R.sync_bench_relaunch(cus, 256, cooperative=0, reps=20)
        rc, rc_sg, null_c = R.sync_bench_relaunch(cus, 256, cooperative=1, reps=20)
        rg, rg_sg, null_g = R.sync_bench_relaunch(cus, 256, cooperative=2, reps=20)
        extra["grid_barrier_ns"] = gb
        extra["relaunch_overhead_ns"] = {"traditional": round(ro, 1), "traditional_sigma": round(ro_sg, 1),
                                         "cooperative": round(rc, 1), "cooperative_sigma": round(rc_sg, 1),
                                         "graph": round(rg, 1), "graph_sigma": round(rg_sg, 1),
                                         "null_kernel_total_ns": round(null_ns, 1),
                                         "null_kernel_total_coop_ns": round(null_c, 1),
                                         "null_kernel_total_graph_ns": round(null_g, 1)}

    # ---- the extensions, one figure each: the segmented batch of 10,000
    #      log-uniform segments (cached plan; graph replay and direct
    #      launches) and the iterative stencil on 4M values (one launch per
    #      step against the persistent form with a grid barrier every 32 steps)
    if not args.no_probes:
        xs, off = inputs.segments(10000)
        xst = torch.from_numpy(xs).to("cuda")
        del xs
        ot = torch.from_numpy(off).to("cuda")
        nseg = off.size - 1
        so = torch.empty(nseg, dtype=torch.float64, device="cuda")
        sp = plans.seg_plan(xst, ot, so, sh)
        od = R.make_opts(variant=sp.variant, wg=sp.wg, ipt=sp.ipt, grid=sp.grid, flags=sp.flags | R.FLAG_NO_GRAPH)
        seg_bytes = xst.numel() * 4 + ot.numel() * 8 + nseg * 8
        seg = {"values": int(off[-1]), "segments": nseg, "plan": sp.as_dict()}
        # the same shape as one persistent kernel (grid-barrier fix-up,
        # ordinary occupancy-capped launch) replayed from a graph
        pg = min(sp.grid or 2 * dev["cus"], R.red_max_coresident_segmented(sp.ipt, sp.wg))
        opg = R.make_opts(variant=R.RED_VARIANT_PERSISTENT, wg=sp.wg, ipt=sp.ipt, grid=pg,
                          flags=R.FLAG_PLAIN_LAUNCH | (sp.flags & R.FLAG_NONTEMPORAL))
        seg["persistent_graph_grid"] = pg
        forms = (("graph", lambda: R.red_sum_segmented(xst.data_ptr(), ot.data_ptr(), nseg, so.data_ptr(), sh)),
                 ("direct", lambda: R.red_sum_segmented_ex(xst.data_ptr(), ot.data_ptr(), nseg, so.data_ptr(), sh, od)),
                 ("persistent_graph",
                  lambda: R.red_sum_segmented_ex(xst.data_ptr(), ot.data_ptr(), nseg, so.data_ptr(), sh, opg)))
        # Two rounds over both forms, the second one kept (the first series
        # after a pause runs slower): back-to-back calls (batch throughput),
        # and each call between its own pair of events (which delays the
        # next graph replay).
        for _ in range(2):
            for name, fn in forms:
                for _ in range(3):
                    fn()
                ms = time_loop(fn, 20, stream)
                seg[name + "_us"] = round(ms * 1e3, 1)
                seg[name + "_GBps"] = gbps(seg_bytes, ms)
                tt, _ = time_steps(fn, 20, stream)
                seg[name + "_us_events_per_call"] = round(statistics.median(tt) * 1e3, 1)
        # The baseline the batch replaces: one red_sum launch per segment
        # (10,000 launches, offsets read on the host).
        loop = lambda: R.red_sum_segmented_loop(xst.data_ptr(), off, nseg, so.data_ptr(), sh)
        loop()
        ms = time_loop(loop, 3, stream)
        seg["per_segment_launches_us"] = round(ms * 1e3, 1)
        seg["per_segment_launches_GBps"] = gbps(seg_bytes, ms)
        seg["graph_speedup_vs_per_segment_launches"] = round(ms * 1e3 / seg["graph_us"], 1)
        if R.red_check_error(sh) != R.RED_OK:
            raise RuntimeError("segmented batch: " + R.last_error())
        extra["segmented_10000"] = seg
        del xst, ot, so
        torch.cuda.empty_cache()
        n_st, steps_st = 1 << 22, 200
        u = torch.from_numpy(inputs.normal_f32(n_st, sub=66)).to("cuda")
        sc = torch.empty_like(u)
        st = {"n": n_st, "steps": steps_st}
        for name, variant, k in (("relaunch", R.RED_VARIANT_RELAUNCH, 0), ("persistent_k32", R.RED_VARIANT_PERSISTENT, 32),
                                 ("persistent_auto", R.RED_VARIANT_PERSISTENT, 0)):
            o = R.make_opts(variant=variant)
            fn = lambda: R.stencil_jacobi_1d(u.data_ptr(), sc.data_ptr(), n_st, steps_st, 0.25, k, sh, o)
            fn()
            tt, _ = time_steps(fn, 5, stream)
            st[name + "_us_per_step"] = round(statistics.median(tt) * 1e3 / steps_st, 3)
        extra["stencil_4M"] = st
        del u, sc
        torch.cuda.empty_cache()
        extra["other_configs"] = other_configs(R, dev, stream, sh, plans, inputs)

    # ---- CPU baseline: the oracle on the same input (and the result's error)
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
               "sample": "the full 2^28-element fp32 input (1 GiB), exact exponent-binned sum, "
                         "single thread, median of 3 runs of %.2f s" % t_cpu}
        extra["cpu_oracle_all_cores"] = cpu_oracle_parallel(oracle, x, ex, nbytes)

    roof = {"bound": "hbm", "achieved": round(kernel_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(kernel_gbps / HBM_PEAK_GBPS, 4), "traffic": traffic_per_launch(plan.as_dict())}
    rec = {
        "metric": METRIC,
        "value": round(value, 1),
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
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)
    if args.calibrate_copy:
        y = torch.empty_like(xt)
        for _ in range(3):
            y.copy_(xt)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
