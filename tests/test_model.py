"""Performance model (Eq. 1-5) against the paper's Tables III and IV."""
import json
import os

import pytest

from paper_2004_05371_amd import model

T = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("gpu", ["V100", "P100"])
def test_table3_concurrency_little_law(gpu):
    for row, (bw, lat, conc) in T["table3_concurrency"][gpu].items():
        assert model.concurrency(lat, bw) == pytest.approx(conc, rel=0.02), row


def scenarios(gpu):
    t3 = T["table3_concurrency"][gpu]
    t4 = T["table4_switch_points"][gpu]
    lat = t3["1 thread"][1]
    s1 = model.Scenario("1 warp", lat, t3["1 thread"][0], t3["1 warp"][0], t4["1 warp"]["t_sync"])
    s2 = model.Scenario("1024 threads", lat, t3["32 threads"][0], t3["1024 threads"][0], t4["1024 threads"]["t_sync"])
    return (s1, t4["1 warp"]), (s2, t4["1024 threads"])


@pytest.mark.parametrize("gpu", ["V100", "P100"])
def test_table4_switch_points(gpu):
    for s, row in scenarios(gpu):
        assert s.n_l() == pytest.approx(row["N_l"], rel=0.02), (gpu, s.name)
        assert s.n_m() == pytest.approx(row["N_m"], rel=0.02), (gpu, s.name)


@pytest.mark.parametrize("gpu", ["V100", "P100"])
def test_paper_conclusions(gpu):
    """Section VII-B: 32 doubles (256 B) are better summed by a warp than by
    one thread; 1024 doubles (8 KiB) gain nothing from 1024 threads over 32."""
    (s1, _), (s2, _) = scenarios(gpu)
    assert not s1.use_basic(32 * 8)
    assert s2.use_basic(1024 * 8)


def test_eq2_matches_switch_point():
    # Eq. 2 evaluated directly agrees with the closed-form N_l beyond both
    # concurrencies
    t, ts, tb, tm = 13.0, 420.0, 19.6, 215.0
    nl = model.switch_point_l(ts, tm, tb)
    assert model.prefer_basic(nl * 0.98, t, ts, tb, tm)
    assert not model.prefer_basic(nl * 1.02, t, ts, tb, tm)


def test_scenario_rule_matches_eq2():
    """The closed-form switch point agrees with Eq. 2 evaluated directly, in
    the scenario it selects."""
    for t, ts, tb, tm in [(4.2, 0.8, 100e3, 7000e3), (13.0, 110.0, 0.62, 19.6), (13.0, 420.0, 19.6, 215.0)]:
        n = model.switch_point(t, ts, tb, tm)
        assert model.prefer_basic(n * 0.97, t, ts, tb, tm)
        assert not model.prefer_basic(n * 1.03, t, ts, tb, tm)


def test_mi355x_switch_points():
    """With the measured MI355X constants the model puts the one-workgroup /
    whole-device switch between the measured crossovers (2^16 and 2^17
    fp32 elements against the atomic ticket, about 2^17 against relaunch)."""
    n_atomic = model.mi355x_single_workgroup_switch("atomic")
    n_relaunch = model.mi355x_single_workgroup_switch("relaunch")
    assert 2**16 * 4 <= n_atomic <= 2**17 * 4 * 1.1
    assert 2**17 * 4 * 0.9 <= n_relaunch <= 2**18 * 4
    assert n_relaunch > n_atomic
