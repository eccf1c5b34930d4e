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


# ---------------------------------------------------------------- the search itself, with a fake cost
# (red_autotune_search: the candidate order and selection of red_autotune,
# costed by a function of the test's choosing instead of GPU timings)

def _rule(v, w, i, g, f):
    return 10.0 + g / 100.0 + w / 1000.0 + i / 10.0 + v + (f & 8) / 8.0 - (f & 1) / 2.0


def _fake(best=None, persistent_cap=None, fail_at=None):
    """A cost function that records the plans it sees; `best` (a dict of
    plan fields) costs 1 us, everything else more, by a fixed rule."""
    seen = []

    def cost(p):
        seen.append((p.variant, p.wg, p.ipt, p.grid, p.flags))
        if fail_at is not None and len(seen) == fail_at:
            return float(R.RED_EHIP)
        if persistent_cap is not None and p.variant == R.RED_VARIANT_PERSISTENT and p.grid > persistent_cap:
            p.grid = persistent_cap
        if best and all(getattr(p, k) == v for k, v in best.items()):
            return 1.0
        # deterministic, larger than 1: prefers the nontemporal hint, small
        # grids and workgroups, the relaunch variant, no pipelining
        return _rule(p.variant, p.wg, p.ipt, p.grid, p.flags)
    return cost, seen


def test_search_order_and_choice_for_a_large_input():
    n = 1 << 28
    target = dict(variant=R.RED_VARIANT_RELAUNCH, wg=512, ipt=2, grid=768, flags=R.FLAG_NONTEMPORAL)
    cost, seen = _fake(best=target)
    plan, us = R.red_autotune_search(R.RED_F32, n, cost, cus=256, nxcc=8)
    assert (plan.variant, plan.wg, plan.ipt, plan.grid, plan.flags) == tuple(target.values()) and us == 1.0
    # default shape without, then with, the nontemporal hint
    d = R.red_get_plan(R.RED_F32, R.RED_ACC_PLAIN, 1 << 40)  # an untouched bucket: the default plan
    assert seen[0][1:3] == (d.wg, d.ipt) and seen[0][4] & R.FLAG_NONTEMPORAL == 0
    assert seen[1][4] & R.FLAG_NONTEMPORAL
    # then 2 (pipelined?) x 4 wg x 4 ipt x 8 grid multiples of the CU count
    # (2^26 vectors never fit in 16 x 256 tiles), then atomic, persistent,
    # persistent by plain launch on the best shape; no XCD form by default
    relaunch = seen[2:2 + 256]
    assert all(v == R.RED_VARIANT_RELAUNCH for v, *_ in relaunch)
    assert sorted({g for *_, g, f in relaunch}) == [256 * m for m in (1, 2, 3, 4, 6, 8, 12, 16)]
    assert {(w, i) for _, w, i, _, _ in relaunch} == {(w, i) for w in (128, 256, 512, 1024) for i in (1, 2, 4, 8)}
    tail = seen[258:]
    assert [t[0] for t in tail] == [R.RED_VARIANT_ATOMIC, R.RED_VARIANT_PERSISTENT, R.RED_VARIANT_PERSISTENT]
    assert all(t[1:4] == (512, 2, 768) for t in tail)
    assert tail[2][4] & R.FLAG_PLAIN_LAUNCH and not tail[1][4] & R.FLAG_PLAIN_LAUNCH
    assert len(seen) == 261
    assert not any(f & R.FLAG_XCD for *_, f in seen)


def test_search_xcd_candidates_only_when_allowed():
    cost, seen = _fake()
    R.red_autotune_search(R.RED_F32, 1 << 28, cost, cus=256, nxcc=8, allow_xcd=True)
    xcd = [s for s in seen if s[4] & R.FLAG_XCD]
    assert [s[0] for s in xcd] == [R.RED_VARIANT_ATOMIC, R.RED_VARIANT_PERSISTENT, R.RED_VARIANT_PERSISTENT]
    cost, seen = _fake()
    R.red_autotune_search(R.RED_F32, 1 << 28, cost, cus=256, nxcc=1, allow_xcd=True)  # one XCD: none
    assert not any(s[4] & R.FLAG_XCD for s in seen)


def test_search_budget_caps_the_candidates():
    cost, seen = _fake()
    plan, us = R.red_autotune_search(R.RED_I32, 1 << 26, cost, budget=7)
    assert len(seen) == 7
    costs = [_rule(*t) for t in seen]
    assert us == min(costs)


def test_search_keeps_the_grid_the_cost_function_lowered():
    cost, seen = _fake(best=dict(variant=R.RED_VARIANT_PERSISTENT, flags=R.FLAG_NONTEMPORAL), persistent_cap=100)
    plan, us = R.red_autotune_search(R.RED_F32, 1 << 28, cost, cus=256)
    assert plan.variant == R.RED_VARIANT_PERSISTENT and plan.grid == 100 and us == 1.0


def test_search_small_inputs_try_one_workgroup():
    target = dict(variant=R.RED_VARIANT_SINGLE, wg=512, ipt=1)
    cost, seen = _fake(best=target)
    plan, us = R.red_autotune_search(R.RED_F32, 5000, cost, cus=256)
    assert (plan.variant, plan.wg, plan.ipt, plan.grid) == (R.RED_VARIANT_SINGLE, 512, 1, 1)
    singles = [s for s in seen if s[0] == R.RED_VARIANT_SINGLE]
    assert len(singles) >= 18  # 3 wg x 3 ipt x 2 (pipelined?), plus the default plan's own
    # small input: each relaunch shape stops at the grid that covers the work
    big = [s for s in seen if s[0] == R.RED_VARIANT_RELAUNCH]
    assert max(g for *_, g, _ in big) <= 5000 // 4
    # the best shape is one workgroup: no device-wide variants follow it
    assert seen[-1][0] == R.RED_VARIANT_SINGLE
    cost, seen = _fake()
    R.red_autotune_search(R.RED_F32, 1 << 28, cost)
    assert not any(s[0] == R.RED_VARIANT_SINGLE for s in seen)


def test_search_stops_on_the_cost_functions_status():
    cost, seen = _fake(fail_at=5)
    with pytest.raises(R.RedError) as e:
        R.red_autotune_search(R.RED_F32, 1 << 28, cost)
    assert e.value.code == R.RED_EHIP and len(seen) == 5
    with pytest.raises(R.RedError):
        R.red_autotune_search(R.RED_F32, 1 << 28, cost, cus=0)  # invalid device description


def test_searched_plan_round_trips_through_the_cache(tmp_path):
    target = dict(variant=R.RED_VARIANT_ATOMIC, wg=256, ipt=8, grid=512, flags=R.FLAG_NONTEMPORAL)
    cost, _ = _fake(best=dict(variant=R.RED_VARIANT_RELAUNCH, wg=256, ipt=8, grid=512, flags=R.FLAG_NONTEMPORAL))
    shape, _ = R.red_autotune_search(R.RED_BF16, 3 << 27, cost)
    assert (shape.wg, shape.ipt, shape.grid) == (256, 8, 512)
    shape.variant = target["variant"]
    entry = {"kind": "sum", "dtype": "bf16", "acc": "compensated", "n": 3 << 27, "plan": shape.as_dict(), "us": 1.0}
    p = autotune.save([entry], str(tmp_path / "t.json"))
    assert autotune.load(p) == 1
    q = R.red_get_plan(R.RED_BF16, R.RED_ACC_COMPENSATED, (3 << 27) + 1)  # same ceil(log2 n) bucket
    assert (q.variant, q.wg, q.ipt, q.grid, q.flags) == tuple(target.values())
