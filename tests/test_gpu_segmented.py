"""GPU parity of the segmented batch (red_sum_segmented) against the
oracle's exact per-segment sums, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
from paper_2004_05371_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BOUND = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(lib, x, off, variant=0, wg=0, ipt=0, grid=0, flags=0):
    xt = torch.from_numpy(x).to("cuda") if x.size else torch.zeros(1, dtype=torch.float32, device="cuda")
    ot = torch.from_numpy(off).to("cuda")
    nseg = off.size - 1
    out = torch.full((max(nseg, 1),), float("nan"), dtype=torch.float64, device="cuda")
    opts = lib.make_opts(variant=variant, wg=wg, ipt=ipt, grid=grid, flags=flags)
    lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), lib.current_stream(), opts)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:nseg]


def check(res, x, off, sums=None):
    if sums is None:
        sums = oracle.segmented_sums(x, off)
    for k, ex in enumerate(sums):
        if ex.fraction == 0:
            a = float(oracle.exact_abs_sum(x[off[k]:off[k + 1]], "f32").fraction)
            assert abs(res[k]) <= 1e-6 * a, (k, res[k])
        else:
            e = oracle.rel_err(float(res[k]), ex)
            assert e <= BOUND, (k, res[k], ex.value, e)


PLANS = [dict(), dict(variant=2, wg=256, ipt=1, grid=7), dict(variant=2, wg=512, ipt=8, grid=1),
         dict(variant=2, wg=64, ipt=2, grid=300), dict(variant=3, wg=256, ipt=4, grid=64),
         dict(variant=2, wg=512, ipt=4, grid=0, flags=2), dict(variant=1, wg=256, ipt=2, grid=50),
         dict(variant=1, wg=512, ipt=8, grid=3, flags=2)]


@pytest.mark.parametrize("plan", range(len(PLANS)))
def test_small_batches(lib, plan):
    p = PLANS[plan]
    r = np.random.default_rng(100 + plan)
    lens = np.concatenate([r.integers(0, 3, 40), r.integers(0, 5000, 40), [0, 0, 70001, 0, 1, 1]])
    r.shuffle(lens)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.mixed_f32(int(off[-1]), sub=9)
    check(run(lib, x, off, **p), x, off)


@pytest.mark.parametrize("plan", range(len(PLANS)))
def test_long_segment_batches(lib, plan):
    """Mean segment length above 16384 values: workgroup slices (the
    short-segment batches above take wavefront slices), with short and empty
    segments between long ones."""
    r = np.random.default_rng(300 + plan)
    lens = np.concatenate([r.integers(20000, 300000, 12), [0, 1, 3, 0, 5, 2, 1000, 0, 64, 65]])
    r.shuffle(lens)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    assert off[-1] >= 16384 * (off.size - 1)
    x = inputs.mixed_f32(int(off[-1]), sub=13)
    check(run(lib, x, off, **PLANS[plan]), x, off)


FORM_PLANS = [dict(variant=2, wg=512, ipt=4, grid=0), dict(variant=2, wg=256, ipt=4, grid=7),
              dict(variant=2, wg=64, ipt=1, grid=300), dict(variant=2, wg=128, ipt=2, grid=33),
              dict(variant=3, wg=256, ipt=2, grid=64), dict(variant=1, wg=512, ipt=4, grid=0),
              dict(variant=1, wg=64, ipt=1, grid=1000)]


def form_layouts():
    """Short-segment batches: uniform lengths around the lane run (4 to 16
    values) and the tile (256 to 1024), runs of empty segments, leading and
    trailing empties, and mixtures that make some tiles fall back to the
    per-piece walk."""
    r = np.random.default_rng(500)
    out = []
    for L in (1, 3, 4, 5, 6, 8, 10, 15, 16, 17, 24, 31, 63, 64, 65, 100, 1000, 1500):
        out.append(("uniform%d" % L, np.full(max(1, 200000 // L), L, dtype=np.int64)))
    out.append(("short0to40", r.integers(0, 41, 20000)))
    out.append(("empties", r.choice([0, 0, 0, 50], 20000)))
    out.append(("mixed", r.choice([0, 1, 5, 64, 300, 2000], 3000)))
    lens = r.integers(10, 200, 5000)
    lens[::97] = 0
    out.append(("sprinkled_empties", np.concatenate([[0] * 300, lens, [0] * 7])))
    out.append(("long_then_short", np.concatenate([[300000], r.integers(1, 30, 10000), [0, 70000]])))
    return out


FORMS = {"workgroup": 32, "pieces": 64, "runs": 128, "auto": 0}
_EXPECTED = {}


def expected(name, x, off):
    """Per segment: the exact sum rounded to binary64 and the allowed error
    (BOUND relative, or 1e-6 of the sum of magnitudes when the exact sum is
    0), computed once per batch."""
    if name not in _EXPECTED:
        sums = oracle.segmented_sums(x, off)
        val = np.array([e.value for e in sums], dtype=np.float64)
        tol = np.abs(val) * BOUND
        for k in np.nonzero([e.fraction == 0 for e in sums])[0]:
            tol[k] = 1e-6 * float(oracle.exact_abs_sum(x[off[k]:off[k + 1]], "f32").fraction)
        _EXPECTED[name] = (val, tol)
    return _EXPECTED[name]


def check_fast(res, val, tol, what):
    bad = np.nonzero(~(np.abs(res - val) <= tol))[0]
    assert bad.size == 0, (what, int(bad[0]), res[bad[0]], val[bad[0]], bad.size)


@pytest.mark.parametrize("form", list(FORMS))
def test_forms_short_segments(lib, form):
    """Every way of cutting and walking the slices, forced through the form
    flags, on the same short-segment batches, against the oracle."""
    for name, lens in form_layouts():
        off = inputs.offsets_from_lengths(lens.astype(np.int64))
        x = inputs.mixed_f32(int(off[-1]), sub=15)
        val, tol = expected(name, x, off)
        for i, p in enumerate(FORM_PLANS):
            say("form", form, name, "plan", i, "nseg", off.size - 1, "values", int(off[-1]))
            check_fast(run(lib, x, off, flags=FORMS[form], **p), val, tol, (form, name, i))


@pytest.mark.parametrize("shift", [1, 3])
def test_runs_form_misaligned(lib, shift):
    """The reduce-by-key form on values 4 or 12 bytes past a 16-byte
    boundary: the first and last tiles of every slice mask values that are
    not the slice's own."""
    r = np.random.default_rng(600 + shift)
    lens = np.concatenate([r.integers(1, 70, 30000), [0, 5000, 0]])
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.mixed_f32(int(off[-1]), sub=16)
    base = torch.zeros(x.size + 8, dtype=torch.float32, device="cuda")
    base[shift:shift + x.size] = torch.from_numpy(x).to("cuda")
    xt = base[shift:shift + x.size]
    ot = torch.from_numpy(off).to("cuda")
    nseg = off.size - 1
    for p in FORM_PLANS:
        out = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
        lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), lib.current_stream(),
                                 lib.make_opts(flags=lib.FLAG_SEG_RUNS, **p))
        torch.cuda.synchronize()
        check(out.cpu().numpy(), x, off)


def test_runs_form_repeat_bit_identical(lib):
    lens = np.random.default_rng(700).integers(0, 100, 100000)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.normal_f32(int(off[-1]), sub=17)
    first = None
    for i in range(3):
        got = run(lib, x, off, flags=lib.FLAG_SEG_RUNS)
        if first is None:
            check(got, x, off)
            first = got
        assert np.array_equal(got, first), i


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_fixups_agree_bit_for_bit(lib, variant):
    """Segments cut by many slice boundaries (768-value segments over 4096
    wavefront slices, and one segment across every slice): the relaunch,
    ticket and barrier fix-ups sum the pieces in the same order, so they
    give the same bits; all match the oracle."""
    for name, lens in (("uniform768", np.full(3000, 768, dtype=np.int64)),
                       ("one_long", np.array([0, 2000003, 0], dtype=np.int64)),
                       ("drawn", inputs.segment_lengths(300, max_len=1 << 15))):
        off = inputs.offsets_from_lengths(lens.astype(np.int64))
        x = inputs.mixed_f32(int(off[-1]), sub=18)
        val, tol = expected(name, x, off)
        grid = 64 if variant == 3 else 512
        got = run(lib, x, off, variant=variant, wg=512, ipt=4, grid=grid)
        check_fast(got, val, tol, (name, variant))
        ref = run(lib, x, off, variant=1, wg=512, ipt=4, grid=grid)
        assert np.array_equal(got, ref), name


@pytest.mark.parametrize("ipt,wg", [(2, 512), (4, 512), (8, 256)])
def test_barrier_fixup_at_the_coresident_limit(lib, ipt, wg):
    """The grid-barrier fix-up runs at exactly the co-resident grid the
    library reports for the segmented kernel and refuses one workgroup
    more."""
    g = lib.red_max_coresident_segmented(ipt, wg)
    assert g >= 256
    lens = np.random.default_rng(900 + ipt).integers(0, 3000, 2000)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.mixed_f32(int(off[-1]), sub=20)
    check(run(lib, x, off, variant=3, wg=wg, ipt=ipt, grid=g), x, off)
    with pytest.raises(lib.RedError):
        run(lib, x, off, variant=3, wg=wg, ipt=ipt, grid=g + 1)


def test_segmented_autotune_installs_a_working_plan(lib):
    """A budgeted search on a small batch installs a plan for its nseg
    bucket; the graph path then uses it and stays exact.  The default plan
    is put back afterwards."""
    from paper_2004_05371_amd import autotune
    lens = np.random.default_rng(950).integers(0, 600, 3000)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.mixed_f32(int(off[-1]), sub=21)
    xt = torch.from_numpy(x).to("cuda")
    ot = torch.from_numpy(off).to("cuda")
    out = torch.empty(3000, dtype=torch.float64, device="cuda")
    before = lib.red_get_segmented_plan(3000)
    try:
        e = autotune.tune_segmented(xt, ot, out, budget=12)
        p = lib.red_get_segmented_plan(3000)
        assert p.as_dict() == e["plan"]
        assert e["plan"]["variant"] in ("relaunch", "atomic") and e["us"] > 0
        res = run(lib, x, off)
        check(res, x, off)
    finally:
        lib.red_set_segmented_plan(3000, before)


def test_runs_form_rejects_eight_loads(lib):
    off = np.array([0, 4], dtype=np.int64)
    x = np.ones(4, dtype=np.float32)
    with pytest.raises(lib.RedError):
        run(lib, x, off, variant=2, wg=256, ipt=8, flags=lib.FLAG_SEG_RUNS)


def test_edge_batches(lib):
    # empty total, leading / trailing empties, a single segment, all length-1
    for lens in ([0], [0, 0, 0], [0, 5, 0], [1], [12345], [3, 0, 0], [1] * 3000, [0] * 10 + [100] + [0] * 10):
        off = inputs.offsets_from_lengths(np.array(lens, dtype=np.int64))
        x = inputs.normal_f32(int(off[-1]), sub=10)
        for p in PLANS:
            check(run(lib, x, off, **p), x, off)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_misaligned_values(lib, shift):
    """Values that start 4, 8 or 12 bytes past a 16-byte boundary: the slices
    are streamed as vectors of the aligned base with the outside elements
    masked."""
    r = np.random.default_rng(200 + shift)
    lens = np.concatenate([r.integers(0, 9, 30), r.integers(0, 3000, 30), [0, 65536 + shift, 1]])
    r.shuffle(lens)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.mixed_f32(int(off[-1]), sub=12)
    base = torch.zeros(x.size + 8, dtype=torch.float32, device="cuda")
    base[shift:shift + x.size] = torch.from_numpy(x).to("cuda")
    xt = base[shift:shift + x.size]
    assert xt.data_ptr() % 16 == 4 * shift
    ot = torch.from_numpy(off).to("cuda")
    nseg = off.size - 1
    for p in PLANS:
        out = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
        lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), lib.current_stream(),
                                 lib.make_opts(**p))
        torch.cuda.synchronize()
        check(out.cpu().numpy(), x, off)


def test_single_segment_equals_red_sum(lib):
    x = inputs.normal_f32(3000017, sub=11)
    off = np.array([0, x.size], dtype=np.int64)
    seg = run(lib, x, off)
    xt = torch.from_numpy(x).to("cuda")
    tot = lib.sum(xt).item()
    ex = oracle.exact_sum(x, "f32")
    assert oracle.rel_err(float(seg[0]), ex) <= BOUND
    assert oracle.rel_err(tot, ex) <= BOUND


def test_length_one_segments_return_values(lib):
    x = inputs.mixed_f32(10007, sub=12)
    off = np.arange(x.size + 1, dtype=np.int64)
    res = run(lib, x, off)
    assert np.array_equal(res, x.astype(np.float64))


def test_repeat_bit_identical_and_graph_replay(lib):
    lens = inputs.segment_lengths(500, max_len=1 << 14)
    off = inputs.offsets_from_lengths(lens)
    x = inputs.normal_f32(int(off[-1]), sub=13)
    xt = torch.from_numpy(x).to("cuda")
    ot = torch.from_numpy(off).to("cuda")
    out = torch.empty(500, dtype=torch.float64, device="cuda")
    first = None
    for i in range(5):  # first call captures a graph, later calls replay it
        out.fill_(float("nan"))
        lib.red_sum_segmented(xt.data_ptr(), ot.data_ptr(), 500, out.data_ptr(), lib.current_stream())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        if first is None:
            first = got.copy()
            check(got, x, off)
        assert np.array_equal(got, first), i


def test_loop_baseline_matches(lib):
    lens = inputs.segment_lengths(200, max_len=1 << 12)
    off = inputs.offsets_from_lengths(lens)
    x = inputs.normal_f32(int(off[-1]), sub=14)
    xt = torch.from_numpy(x).to("cuda")
    out = torch.empty(200, dtype=torch.float64, device="cuda")
    lib.red_sum_segmented_loop(xt.data_ptr(), off, 200, out.data_ptr(), lib.current_stream())
    torch.cuda.synchronize()
    check(out.cpu().numpy(), x, off)


def test_full_batch_config(lib):
    """10,000 log-uniform segments in [1, 2^20] (about 7.4e8 values): the
    default plan, the cached plan the bench line times (ticket fix-up,
    256 x 4, grid 768, nontemporal, graph replay), the relaunch fix-up and
    the barrier fix-up."""
    x, off = inputs.segments(10000)
    say("segments total", int(off[-1]))
    sums = oracle.segmented_sums(x, off)
    for p in (dict(), dict(variant=2, wg=256, ipt=4, grid=768, flags=1), dict(variant=1, wg=256, ipt=4, grid=1024, flags=1),
              dict(variant=3, wg=512, ipt=4, grid=256)):
        say("plan", p)
        res = run(lib, x, off, **p)
        check(res, x, off, sums)


@pytest.mark.parametrize("L", [3, 4, 5, 8, 64, 768])
def test_full_size_uniform_segments(lib, L):
    """2^28 N(0,1) values in segments of 3 to 8 values (reduce-by-key form
    with quarter-tile parts and the per-piece walk; up to 89M segments), of
    64 values (reduce-by-key form, 4M segments) and of 768 values (a segment
    cut at every slice edge), default plan through the graph path: 3000
    sampled segments against the oracle's exact sums, every segment within
    1e-12 of its sum of magnitudes of a binary64 row sum, and the other
    fix-up (relaunch for the default ticket, else the ticket) on the same
    slices bit-identical."""
    n = (1 << 28) // L * L
    x = inputs.normal_f32(1 << 28, sub=19)[:n]
    nseg = n // L
    xt = torch.from_numpy(x).to("cuda")
    ot = torch.arange(0, n + 1, L, dtype=torch.int64, device="cuda")
    out = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
    say("full-size uniform segments", L, nseg)
    lib.red_sum_segmented(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), lib.current_stream())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    rows = x.reshape(nseg, L)
    approx = rows.astype(np.float64).sum(axis=1)
    mag = np.abs(rows).astype(np.float64).sum(axis=1)
    bad = np.nonzero(~(np.abs(got - approx) <= 1e-12 * mag))[0]
    assert bad.size == 0, (int(bad[0]), got[bad[0]], approx[bad[0]])
    pick = np.random.default_rng(800 + L).choice(nseg, 3000, replace=False)
    for k in pick:
        ex = oracle.exact_sum(rows[k], "f32")
        assert oracle.rel_err(float(got[k]), ex) <= BOUND, (k, got[k], ex.value)
    p = lib.red_get_segmented_plan(nseg)
    other = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
    lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, other.data_ptr(), lib.current_stream(),
                             lib.make_opts(variant=1 if p.variant == 2 else 2, wg=p.wg, ipt=p.ipt, grid=p.grid,
                                           flags=p.flags))
    torch.cuda.synchronize()
    assert np.array_equal(other.cpu().numpy(), got)
    del xt, ot, out, other
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L,shift", [(7, 1), (16, 3), (33, 2)])
def test_full_size_misaligned_reduce_by_key(lib, L, shift):
    """Close to 2^28 values at a base 4 to 12 bytes past a 16-byte boundary,
    in segments of 7, 16 and 33 values (reduce-by-key parts of 1, 2 and 4
    rows), the total not a whole number of tiles: the direct-to-LDS tile
    loads start before the first value and clamp at each slice's last
    vector.  Every segment within 1e-12 of its sum of magnitudes of a
    binary64 row sum, 1000 sampled against the oracle's exact sums."""
    nseg = ((1 << 28) - 5) // L
    n = nseg * L
    x = inputs.normal_f32(n, sub=21)
    buf = torch.zeros(n + 8, dtype=torch.float32, device="cuda")
    xt = buf[shift:shift + n]
    xt.copy_(torch.from_numpy(x))
    ot = torch.arange(0, n + 1, L, dtype=torch.int64, device="cuda")
    out = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
    say("full-size misaligned segments", L, shift, nseg)
    lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), lib.current_stream(),
                             lib.make_opts(flags=lib.FLAG_NONTEMPORAL | lib.FLAG_SEG_RUNS))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    rows = x.reshape(nseg, L)
    approx = rows.astype(np.float64).sum(axis=1)
    mag = np.abs(rows).astype(np.float64).sum(axis=1)
    bad = np.nonzero(~(np.abs(got - approx) <= 1e-12 * mag))[0]
    assert bad.size == 0, (int(bad[0]), got[bad[0]], approx[bad[0]])
    for k in np.random.default_rng(900 + L).choice(nseg, 1000, replace=False):
        ex = oracle.exact_sum(rows[k], "f32")
        assert oracle.rel_err(float(got[k]), ex) <= BOUND, (k, got[k], ex.value)
    del buf, xt, ot, out
    torch.cuda.empty_cache()


def test_graph_cache_eviction(lib):
    """More distinct batches than the graph cache holds (64): the oldest
    graphs are evicted (after their stream drains) and rebuilt on reuse;
    every result stays exact and bit-identical."""
    r = np.random.default_rng(400)
    lens = r.integers(0, 3000, 50)
    off = inputs.offsets_from_lengths(lens.astype(np.int64))
    x = inputs.normal_f32(int(off[-1]), sub=14)
    xt = torch.from_numpy(x).to("cuda")
    ot = torch.from_numpy(off).to("cuda")
    nseg = off.size - 1
    st = torch.cuda.Stream()
    outs = torch.full((80, nseg), float("nan"), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(st):
        for rep in range(2):  # the second pass finds the first graphs evicted
            for i in range(80):
                lib.red_sum_segmented(xt.data_ptr(), ot.data_ptr(), nseg, outs[i].data_ptr(), st.cuda_stream)
    st.synchronize()
    res = outs.cpu().numpy()
    assert (res == res[0]).all()
    check(res[0], x, off)


def test_persistent_batch_replays_from_a_graph(lib):
    """The grid-barrier fix-up as one persistent kernel, launched as an
    ordinary occupancy-capped grid: captured into the library's graph on the
    first call and replayed after, every replay bit-identical to the
    two-kernel relaunch graph of the same shape (the fix-ups sum the pieces
    in the same order) and to the oracle; no watchdog fired."""
    lens = inputs.segment_lengths(400, max_len=1 << 16)
    off = inputs.offsets_from_lengths(lens)
    x = inputs.mixed_f32(int(off[-1]), sub=23)
    xt = torch.from_numpy(x).to("cuda")
    ot = torch.from_numpy(off).to("cuda")
    nseg = off.size - 1
    g = min(512, lib.red_max_coresident_segmented(4, 512))
    pers = lib.make_opts(variant=3, wg=512, ipt=4, grid=g, flags=lib.FLAG_PLAIN_LAUNCH | lib.FLAG_NONTEMPORAL)
    rel = lib.make_opts(variant=1, wg=512, ipt=4, grid=g, flags=lib.FLAG_NONTEMPORAL)
    s = lib.current_stream()
    ref = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
    lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, ref.data_ptr(), s, rel)
    torch.cuda.synchronize()
    want = ref.cpu().numpy()
    check(want, x, off)
    out = torch.empty(nseg, dtype=torch.float64, device="cuda")
    for i in range(4):  # capture, then three replays
        out.fill_(float("nan"))
        lib.red_sum_segmented_ex(xt.data_ptr(), ot.data_ptr(), nseg, out.data_ptr(), s, pers)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), i
    assert lib.red_check_error(s) == lib.RED_OK
