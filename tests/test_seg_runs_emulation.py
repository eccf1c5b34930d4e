"""Lane-level CPU emulation of the segmented batch's reduce-by-key form
(seg_wave_runs) and relaunch fix-up (k_seg_fixup), tests/emu/seg_runs_emu.cpp:
every global, LDS and cross-lane access bounds-checked, the kernel's own
invariants checked, every segment's sum compared exactly (integer values).

Covered geometries include the one of a GPU memory fault seen while two
changes to this form were under test: 2^28 values in segments of 3, 4 and
5 values, 512-thread workgroups with 4 and with 2 loads per lane, a grid
of 512 workgroups (4096 wavefront slices).  The committed code passes
them all; each planted mistake (built with -DMUTATION=k) must fail.
Mutation 4 is the reading of the removed change that admitted parts with
as many starts as visible ring entries: it reads lane 64."""
import concurrent.futures
import json
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "seg_runs_emu.cpp")
CXX = shutil.which("g++")

pytestmark = pytest.mark.skipif(CXX is None, reason="needs g++")


def build(out_dir, mutation=0, sanitize=False):
    exe = os.path.join(out_dir, "emu_m%d%s" % (mutation, "_san" if sanitize else ""))
    cmd = [CXX, "-O2", "-std=c++17", "-Wall", "-Werror", "-DMUTATION=%d" % mutation, "-o", exe, SRC]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    subprocess.run(cmd, check=True)
    return exe


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    return build(str(tmp_path_factory.mktemp("emu")))


def run(exe, E, L, layout, grid, wg, ipt, shift=0, seed=1, env=None):
    p = subprocess.run([exe] + [str(a) for a in (E, L, layout, grid, wg, ipt, shift, seed)],
                       capture_output=True, text=True, timeout=600, env=env)
    lines = p.stdout.strip().splitlines()
    rec = json.loads(lines[-1]) if lines else {"ok": False, "violation": p.stderr[-500:]}
    rec["rc"] = p.returncode
    rec["args"] = (E, L, layout, grid, wg, ipt, shift, seed)
    return rec


SMALL = [
    # E, L, layout, grid, wg, ipt, shift
    (0, 5, 0, 8, 512, 4, 0), (1, 1, 0, 8, 512, 4, 3), (63, 1, 1, 3, 64, 1, 1), (1000, 7, 1, 1, 64, 2, 2),
    (100_000, 5, 0, 8, 512, 4, 0), (100_000, 5, 1, 8, 512, 4, 1), (1_000_003, 64, 0, 3, 256, 2, 2),
    (1_000_003, 16, 1, 7, 64, 1, 3), (1_000_003, 3, 0, 16, 512, 4, 0), (1_000_003, 4, 0, 16, 512, 4, 1),
    (1_000_003, 4, 0, 16, 512, 2, 2), (1_000_003, 11, 0, 16, 512, 4, 0), (1_000_003, 31, 0, 16, 512, 4, 3),
    (1_000_003, 33, 1, 16, 256, 4, 0), (1_000_003, 500, 1, 5, 512, 4, 1), (2_000_000, 1000, 0, 300, 64, 1, 0),
    (2_000_000, 2, 1, 64, 512, 4, 2), (4_000_000, 8, 0, 1, 512, 4, 0), (500_000, 3000, 1, 50, 128, 2, 1),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_geometries(emu, case):
    rec = run(emu, *SMALL[case])
    assert rec["rc"] == 0 and rec["ok"], rec


# The fault's geometry (2^28 values, 512-thread workgroups, grid 512) for
# every short length up to 8, both load counts, plus drawn lengths with
# empty segments and misaligned bases; and the default plan's geometry.
FULL = [(1 << 28, L, 0, 512, 512, ipt, 0) for L in (3, 4, 5) for ipt in (4, 2)]
FULL += [(1 << 28, L, 0, 512, 512, 4, 0) for L in (6, 7, 8)]
FULL += [(1 << 28, 4, 1, 512, 512, 4, 1), (1 << 28, 3, 1, 512, 512, 2, 3), ((1 << 28) - 5, 5, 0, 512, 512, 4, 2)]
# the default plan's geometry: 256-thread workgroups, four per CU (grid 1024)
FULL += [(1 << 28, L, 0, 1024, 256, 4, 0) for L in (3, 4, 5, 8)] + [(1 << 28, 4, 1, 1024, 256, 4, 2)]


def test_fault_geometry_is_free_of_out_of_bounds_accesses(emu):
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        recs = list(ex.map(lambda c: run(emu, *c), FULL))
    bad = [r for r in recs if r["rc"] != 0 or not r["ok"]]
    assert not bad, bad
    for r in recs:
        assert r["values"] == r["args"][0] and r["auto_form_is_runs"], r
    # the 512 x 4 plan walks every 4-value tile's quarters with both walks
    four = next(r for r in recs if r["args"][1:7] == (4, 0, 512, 512, 4, 0))
    assert four["parts_reduce_by_key"] > 0 and four["parts_piece_walk"] > 0


MUTATION_CASES = [(1_000_003, 5, 0, 8, 512, 4, 1), (1_000_003, 16, 1, 8, 512, 4, 2),
                  (1_000_003, 40, 1, 8, 512, 2, 3), (2_000_000, 4, 0, 8, 512, 4, 0),
                  (1_000_003, 200, 1, 16, 256, 4, 1)]


@pytest.mark.parametrize("mutation", range(1, 9))
def test_planted_mistakes_are_caught(tmp_path, mutation):
    exe = build(str(tmp_path), mutation)
    recs = [run(exe, *c) for c in MUTATION_CASES]
    assert any(r["rc"] != 0 and not r["ok"] for r in recs), recs
    if mutation == 4:
        # parts with as many starts as visible entries: the walk reads lane 64
        four = next(r for r in recs if r["args"][1] == 4)
        assert four["violation"] == "readlane index out of range" and four["a"] == 64, four


def test_emulation_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The emulator itself, built with ASan and UBSan, over mid-size
    geometries (host-side memory errors in the checker would hide real
    ones)."""
    exe = build(str(tmp_path), 0, sanitize=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    for c in SMALL[4:12] + [(3_000_001, 4, 0, 64, 512, 4, 1), (3_000_001, 3, 1, 64, 512, 2, 0)]:
        rec = run(exe, *c, env=env)
        assert rec["rc"] == 0 and rec["ok"], rec
