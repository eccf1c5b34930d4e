"""bench.py's summary writers (no GPU): the synchronization
characterization summary from configs records."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_summarize_configs_writes_every_table(tmp_path):
    recs = [
        {"config": "machine", "device": {"cus": 256, "nxcc": 8, "clock_khz": 2400000, "wallclock_khz": 100000},
         "host_cpus": 16},
        {"probe": "wave", "op": "dpp_reduce", "type": "f32", "ns": 50.1, "sigma_ns": 1.0, "cycles": 120.0},
        {"probe": "block", "wg": 256, "n_wg": 256, "waves_per_wg": 4, "waves_per_cu": 4.0, "ns": 30.0,
         "sigma_ns": 0.5, "cycles": 70.0},
        {"probe": "block_tput", "wg": 256, "wg_per_cu": 2, "waves_per_cu": 8, "barriers_per_us_per_cu": 61.5,
         "cycles_per_barrier": 78.0},
        {"probe": "grid", "wg": 256, "n_wg": 256, "wg_per_cu": 1.0, "groups": "xcd", "ns": 4500.0, "sigma_ns": 100.0,
         "in_kernel_ns": 4400.0},
        {"probe": "grid", "wg": 64, "n_wg": 512, "wg_per_cu": 2.0, "groups": 1, "ns": 9000.0, "sigma_ns": 100.0,
         "in_kernel_ns": 8900.0},
        {"probe": "relaunch", "launch": "ordinary", "n_wg": 256, "overhead_ns": 1200.0, "sigma_ns": 90.0,
         "null_kernel_total_ns": 1600.0},
    ]
    src = tmp_path / "c.jsonl"
    src.write_text("\n".join(json.dumps(r) for r in recs) + "\n")
    subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-configs", str(src),
                    "--summary-out", str(tmp_path)], check=True, capture_output=True)
    text = (tmp_path / "sync_characterization.md").read_text()
    for heading in ("Wavefront combines", "Workgroup barrier latency", "throughput under load", "heat map",
                    "Shape: xcd", "Shape: flat", "Kernel boundary", "against a kernel boundary"):
        assert heading in text, heading
    assert "| 256 | 2 | 8 | 61.5 | 78.0 |" in text
    assert "| 256 | xcd | 4500 | 1200 | 3300 |" in text
