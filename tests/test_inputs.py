"""Seeded synthetic inputs (no GPU): identical draws for identical seeds,
independent streams, the value ranges and distributions the workloads
specify, and well-formed CSR offsets."""
import numpy as np

from paper_2004_05371_amd import inputs


def test_same_seed_same_bits_and_streams_differ():
    a = inputs.normal_f32(1 << 16)
    b = inputs.normal_f32(1 << 16)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    c = inputs.normal_f32(1 << 16, sub=1)
    assert not np.array_equal(a, c)
    assert not np.array_equal(inputs.uniform_i32(1000), inputs.uniform_i32(1000, sub=1))


def test_value_ranges():
    i = inputs.uniform_i32(1 << 20)
    assert i.dtype == np.int32 and i.min() == -1000 and i.max() == 1000  # both ends drawn
    u = inputs.uniform_f32(1 << 20)
    assert u.dtype == np.float32 and u.min() >= -1.0 and u.max() <= 1.0
    m = inputs.mixed_f32(1 << 20)
    mag = np.abs(m.astype(np.float64))
    assert mag.min() >= 1e-8 * (1 - 1e-6) and mag.max() <= 1e8 * (1 + 1e-6)
    frac_neg = np.mean(m < 0)
    assert 0.49 < frac_neg < 0.51
    # log10 of the magnitude is uniform on (-8, 8)
    lg = np.log10(mag)
    assert abs(lg.mean()) < 0.05 and abs(lg.std() - 16 / np.sqrt(12)) < 0.05


def test_normal_moments_and_half_rounding():
    x = inputs.normal_f32(1 << 20)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
    for kind in ("bf16", "f16"):
        bits = inputs.normal_half_bits(1 << 16, kind)
        assert bits.dtype == np.uint16
        if kind == "f16":
            v = bits.view(np.float16).astype(np.float64)
        else:
            v = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        assert abs(v.mean()) < 0.02 and abs(v.std() - 1) < 0.02


def test_segment_lengths_and_offsets():
    lens = inputs.segment_lengths(10000)
    assert lens.dtype == np.int64 and lens.min() >= 1 and lens.max() <= 1 << 20
    # log-uniform on [1, 2^20]: ln(L) is uniform on [0, ln 2^20)
    ll = np.log(lens.astype(np.float64))
    assert abs(ll.mean() - np.log(1 << 20) / 2) < 0.2
    off = inputs.offsets_from_lengths(lens)
    assert off[0] == 0 and off[-1] == lens.sum() and np.all(np.diff(off) == lens)
    assert int(off[-1]) == 742_706_513  # the drawn batch's total, as reported
    x, o = inputs.segments(50, max_len=1 << 10)
    assert x.dtype == np.float32 and x.size == o[-1] and o.size == 51
    scaled = inputs.segment_lengths(10000, total=1 << 28)
    assert scaled.min() >= 1 and abs(int(scaled.sum()) - (1 << 28)) < 10000
