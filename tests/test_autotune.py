"""Plan cache of the autotuner (no GPU): round trip, corrupt and foreign
caches fall back to the default plans, invalid entries are skipped."""
import json
import warnings

import pytest

from paper_2004_05371_amd import autotune, redsum as R


def test_roundtrip_installs_plans(tmp_path):
    entries = [
        {"kind": "sum", "dtype": "bf16", "acc": "plain", "n": 1 << 30,
         "plan": {"variant": "atomic", "wg": 256, "ipt": 8, "grid": 1536, "flags": 1}, "us": 1.0},
        {"kind": "segmented", "nseg": 1 << 17,
         "plan": {"variant": "atomic", "wg": 512, "ipt": 2, "grid": 512, "flags": 1}, "us": 2.0},
    ]
    p = autotune.save(entries, str(tmp_path / "c.json"))
    assert autotune.load(p) == 2
    q = R.red_get_plan(R.RED_BF16, R.RED_ACC_PLAIN, 1 << 30)
    assert (q.variant, q.wg, q.ipt, q.grid, q.flags) == (2, 256, 8, 1536, 1)
    s = R.red_get_segmented_plan(1 << 17)
    assert (s.variant, s.wg, s.ipt, s.grid, s.flags) == (2, 512, 2, 512, 1)


def test_corrupt_cache_keeps_defaults(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    before = R.red_get_plan(R.RED_F16, R.RED_ACC_COMPENSATED, 12345)
    with warnings.catch_warnings(record=True):
        warnings.simplefilter("always")
        assert autotune.load(str(p)) == 0
    after = R.red_get_plan(R.RED_F16, R.RED_ACC_COMPENSATED, 12345)
    assert before.as_dict() == after.as_dict()


def test_foreign_arch_and_bad_entries(tmp_path):
    p = tmp_path / "x.json"
    p.write_text(json.dumps({"format": 1, "arch": "gfx942", "cus": 304, "entries": []}))
    with warnings.catch_warnings(record=True):
        warnings.simplefilter("always")
        assert autotune.load(str(p)) == 0
    p.write_text(json.dumps({"format": 1, "arch": "gfx950", "cus": 256, "entries": [
        {"kind": "sum", "dtype": "f32", "acc": "compensated", "n": 77,
         "plan": {"variant": "relaunch", "wg": 100, "ipt": 4, "grid": 0}},  # wg not a multiple of 64
        {"kind": "sum", "dtype": "nope", "acc": "compensated", "n": 77,
         "plan": {"variant": "relaunch", "wg": 256, "ipt": 4, "grid": 0}},
        {"kind": "segmented", "nseg": 5, "plan": {"variant": "single", "wg": 256, "ipt": 4, "grid": 0}},
        {"kind": "sum", "dtype": "i32", "acc": "compensated", "n": 77,
         "plan": {"variant": "persistent", "wg": 512, "ipt": 2, "grid": 64}},
    ]}))
    with warnings.catch_warnings(record=True):
        warnings.simplefilter("always")
        assert autotune.load(str(p)) == 1
    q = R.red_get_plan(R.RED_I32, R.RED_ACC_COMPENSATED, 77)
    assert (q.variant, q.wg, q.ipt, q.grid) == (3, 512, 2, 64)


def test_missing_cache_is_silent(tmp_path):
    assert autotune.load(str(tmp_path / "none.json")) == 0
