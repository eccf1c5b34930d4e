// Lane-level CPU emulation of the reduce-by-key form of the segmented batch
// (seg_wave_runs in paper_2004_05371_amd/csrc/segmented.hip) and of the
// relaunch fix-up kernel (k_seg_fixup), with a bounds check on every access.
//
// Test infrastructure only: nothing of the library is linked or included.
// The emulation restates the kernel's steps for one wavefront at a time,
// with every per-lane value held as an array of 64 and every cross-lane
// operation (ballot, readlane, the DPP wave and row shifts and row
// broadcasts of the segmented scan) written out, and the tile buffer that
// direct-to-LDS loads fill row by row modelled with the rows in flight.  It
// checks:
//   * every global access: the 16-byte vectors of the values (each must
//     overlap the array), offsets[i] (0 <= i <= nseg), out[s] (s < nseg),
//     carry_in / carry_out slots (< the wavefront count and the slot
//     capacity), and readlane indexes (< 64);
//   * every LDS access: offsets-ring positions (< 384), the ring entry read
//     is the one the walk asks for (a shadow of each slot's index), the
//     start slots (< 64), the tile buffer (< 64 x loads per lane vectors),
//     each tile position read holds the vector the read expects, no row is
//     read or loaded again while its load is in flight;
//   * the kernel's own invariants: the valid lanes of a window form a
//     prefix, each start lies in the part, masked ranges are not inverted,
//     the piece walk reads only parts taken from the tile, each carry slot
//     read by the fix-up was written by this launch;
//   * the results: every segment written exactly once, equal to the exact
//     integer sum of its values (the values are small integers, so every
//     partial is exact and the sums are compared for equality).
// A failed check prints the access that failed and exits with status 1.
//
// Built with -DMUTATION=k (k = 1..8) the emulation carries one planted
// mistake of a kind the checks must catch (the test builds each one and
// expects a failure): 1 the next segment's end read from the wrong lane,
// 2 a prefetched ring block written one block off, 3 no check for two
// starts in one run, 4 a part with as many starts as visible ring entries
// taken by the reduce-by-key walk, 5 a cut segment's piece count one short,
// 6 no mask for the values outside the slice, 7 tile vectors fetched in row
// order instead of the order the run reads expect, 8 the piece walk not
// reading the tile's remaining parts first.
//
// Usage: seg_runs_emu E L layout grid wg ipt shift seed
//   E        values in the batch
//   L        segment length (layout 0: uniform L; layout 1: lengths drawn
//            uniformly from [0, 2L], empty segments included)
//   grid wg ipt  the launch shape (ipt = loads of 16 bytes per lane per
//            tile, at most 4 in this form)
//   shift    misalignment of the values' base, in elements (0..3)
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#ifndef MUTATION
#define MUTATION 0
#endif

namespace {

constexpr int kWave = 64;
constexpr int kRing = 384;
constexpr int64_t kMaxChunks = 65536;
constexpr int64_t kRunsMeanLen = 1024;
constexpr int64_t kNone = INT64_MAX;

[[noreturn]] void fail(const char* what, long long a, long long b = 0, long long c = 0) {
  printf("{\"ok\": false, \"violation\": \"%s\", \"a\": %lld, \"b\": %lld, \"c\": %lld}\n", what, a, b, c);
  fflush(stdout);
  exit(1);
}

// ------------------------------------------------------------------ batch
struct Batch {
  int64_t E = 0, nseg = 0;
  int shift = 0;
  std::vector<int64_t> off;       // nseg + 1
  std::vector<int64_t> out;       // per segment, as written
  std::vector<uint8_t> writes;    // writes per segment
  // values are a function of the element index (small integers)
  static int64_t value(int64_t i) {
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    return (int64_t)(h % 15) - 7;
  }
};

struct Carry {
  int64_t seg = 0, val = 0, np = 0;
  uint32_t epoch = 0;  // launch that wrote it
};

struct Machine {
  Batch& b;
  int grid, wg, ipt;
  int64_t W;
  std::vector<Carry> carry_in, carry_out;
  uint32_t epoch = 1;
  long long vec_loads = 0, offset_reads = 0, parts_runs = 0, parts_pieces = 0;

  Machine(Batch& bb, int g, int w, int i) : b(bb), grid(g), wg(w), ipt(i) {
    W = (int64_t)grid * (wg / kWave);
    carry_in.resize(kMaxChunks);
    carry_out.resize(kMaxChunks);
  }

  int64_t offset(int64_t i) {
    if (i < 0 || i > b.nseg) fail("offsets read out of bounds", i, b.nseg);
    ++offset_reads;
    return b.off[i];
  }
  void write_out(int64_t s, int64_t v) {
    if (s < 0 || s >= b.nseg) fail("out write out of bounds", s, b.nseg);
    b.out[s] = v;
    if (b.writes[s] < 255) ++b.writes[s];
  }
  Carry& slot(std::vector<Carry>& c, int64_t w, const char* name) {
    if (w < 0 || w >= W || w >= kMaxChunks) fail(name, w, W);
    return c[w];
  }
  // One 16-byte vector of the aligned base (4 values); element e of the
  // batch is value 4 v - shift + j.  Values outside [0, E) are not the
  // batch's: they read as a large poison value, so a result that uses one
  // is wrong.
  void load_vec(int64_t v, int64_t* dst) {
    const int64_t e = 4 * v - b.shift;
    if (e + 3 < 0 || e >= b.E) fail("vector load out of bounds", v, e, b.E);
    ++vec_loads;
    for (int j = 0; j < 4; ++j) {
      const int64_t i = e + j;
      dst[j] = (i >= 0 && i < b.E) ? Batch::value(i) : (int64_t)1 << 40;
    }
  }
};

// Lane arrays
template <class T>
using Lanes = T[kWave];

int64_t lane_read(const int64_t* v, int lane) {
  if (lane < 0 || lane >= kWave) fail("readlane index out of range", lane);
  return v[lane];
}

// ------------------------------------------------------------------ one wavefront
// Finish the piece [max(sa, lo), min(sb, hi)) of segment s (relaunch
// fix-up): whole segments are written, pieces of cut segments go to the
// wavefront's carry slot.
void finish_piece(Machine& M, int64_t s, int64_t sa, int64_t sb, int64_t v, int64_t lo, int64_t hi, int64_t w,
                  int64_t chunk) {
  if (sb < sa) fail("segment bounds inverted", s, sa, sb);
  if (sa >= lo && sb <= hi) {
    M.write_out(s, v);
    return;
  }
  const int64_t o = sa / chunk;
  const int64_t np = (sb - 1) / chunk - o + 1 - (MUTATION == 5 ? 1 : 0);
  if (np < 1 || o + np > M.W) fail("cut segment's slice range out of the grid", s, o, np);
  Carry c{s, v, np, M.epoch};
  if (sa < lo)
    M.slot(M.carry_in, w, "carry_in write out of bounds") = c;
  else
    M.slot(M.carry_out, w, "carry_out write out of bounds") = c;
}

bool seek_segment(Machine& M, int64_t& s, int64_t hi, int64_t E, bool end_slice, int64_t& sa, int64_t& sb) {
  for (; s < M.b.nseg; ++s) {
    sa = M.offset(s);
    sb = M.offset(s + 1);
    if (sa >= hi && !(end_slice && sa == E)) return false;
    if (sa != sb) return true;
    M.write_out(s, 0);
  }
  return false;
}

int64_t first_segment(Machine& M, int64_t lo) {
  int64_t L = 0, R = M.b.nseg;
  while (L < R) {
    const int64_t mid = (L + R) >> 1;
    if (M.offset(mid) >= lo)
      R = mid;
    else
      L = mid + 1;
  }
  return (L > 0 && M.offset(L) > lo) ? L - 1 : L;
}

int run_swz(int i, int rs) { return i ^ ((i >> 4) & (rs - 1)); }

void wave_runs(Machine& M, int64_t w) {
  Batch& B = M.b;
  const int IPT = M.ipt;
  const int64_t nseg = B.nseg;
  const int64_t E = M.offset(nseg);
  const int64_t Wn = M.W;
  const int64_t chunk = std::max<int64_t>(64, (((E + Wn - 1) / Wn) + 63) & ~(int64_t)63);
  const int64_t lo = std::min(w * chunk, E);
  const int64_t hi = std::min(lo + chunk, E);
  const bool end_slice = E > 0 ? (lo < E && hi == E) : (w == 0);
  M.slot(M.carry_out, w, "carry_out clear out of bounds") = Carry{-1, 0, 0, M.epoch};

  int64_t s = first_segment(M, lo);
  int64_t sa = 0, sb = 0;
  bool have = seek_segment(M, s, hi, E, end_slice, sa, sb);
  int64_t C = 0;

  const int shift = B.shift;
  const int64_t vlo = (lo + shift) >> 2;
  const int64_t vhi = (hi + shift + 3) >> 2;
  const int64_t T = (int64_t)kWave * IPT;
  const int64_t ntiles = lo < hi ? (vhi - vlo + T - 1) / T : 0;

  // offsets ring (LDS) and its shadow: which offsets index each slot holds
  int64_t ring[kRing], ring_idx[kRing];
  for (int i = 0; i < kRing; ++i) ring_idx[i] = -1;
  int64_t fill = 0;
  int npend = 0;
  Lanes<int64_t> pend[3];
  auto off_entry = [&](int64_t i) -> int64_t { return i <= nseg ? M.offset(i) : kNone; };
  auto ring_pos = [&](int64_t base, int lane) {
    if (base < 0) fail("ring base negative", base);
    const int h = (int)(base % kRing) + lane;
    const int p = h >= kRing ? h - kRing : h;
    if (p < 0 || p >= kRing) fail("ring position out of bounds", p);
    return p;
  };
  auto put_block = [&](const int64_t* v, int64_t base) {
    for (int l = 0; l < kWave; ++l) {
      const int p = ring_pos(base, l);
      ring[p] = v[l];
      ring_idx[p] = base + l;
    }
  };
  auto refill = [&]() {
    for (int k = 0; k < npend; ++k) put_block(pend[k], fill + (int64_t)(k + (MUTATION == 2 ? 1 : 0)) * kWave);
    fill += (int64_t)npend * kWave;
    npend = 0;
    if (fill - (s + 1) < kWave) {
      fill = s + 1;
      for (int k = 0; k < 3; ++k) {
        Lanes<int64_t> blk;
        for (int l = 0; l < kWave; ++l) blk[l] = off_entry(fill + (int64_t)k * kWave + l);
        put_block(blk, fill + (int64_t)k * kWave);
      }
      fill += 3 * kWave;
    }
    if (fill - (s + 1) > kRing) fail("ring holds more than its capacity ahead of the walk", fill, s);
    npend = (int)std::min<int64_t>(3, (kRing - (fill - (s + 1))) / kWave);
    for (int k = 0; k < npend; ++k)
      for (int l = 0; l < kWave; ++l) pend[k][l] = off_entry(fill + (int64_t)k * kWave + l);
  };
  const int nparts = (IPT >= 4 && E < 12 * nseg) ? 4 : (IPT >= 2 && E < 32 * nseg) ? 2 : 1;

  // The tile buffer (LDS): direct-to-LDS load instruction u writes lane l's
  // vector at position 64 u + l (row u); lane l fetches tile vector
  // run_swz(64 u + l) of the tile, clamped to the slice's last vector.
  // tile_vec shadows which vector of the batch each position holds.  A row's
  // load stays in flight until the wait at the top of the next tile;
  // reading a row with a load in flight, or issuing a load over one, fails.
  const int rows = IPT / nparts;
  std::vector<int64_t> tile((size_t)kWave * 4 * 4, 0), pend_tile((size_t)kWave * 4 * 4, 0);
  std::vector<int64_t> tile_vec((size_t)kWave * 4, -1), pend_vec((size_t)kWave * 4, -1);
  bool row_pending[4] = {false, false, false, false};
  auto issue_rows = [&](int64_t t, int u0, int n) {
    const int64_t vb = vlo + t * T;
    for (int u = u0; u < u0 + n; ++u) {
      if (u < 0 || u >= IPT) fail("tile row out of bounds", u);
      if (row_pending[u]) fail("tile row load issued over one in flight", t, u);
      for (int l = 0; l < kWave; ++l) {
        const int pos = u * kWave + l;
        const int swz = MUTATION == 7 ? pos : run_swz(pos, rows);
        const int64_t g = std::min(vb + swz, vhi - 1);
        M.load_vec(g, &pend_tile[(size_t)pos * 4]);
        pend_vec[pos] = g;
      }
      row_pending[u] = true;
    }
  };
  auto wait_all = [&]() {
    for (int u = 0; u < 4; ++u)
      if (row_pending[u]) {
        for (int l = 0; l < kWave; ++l) {
          const size_t pos = (size_t)u * kWave + l;
          for (int j = 0; j < 4; ++j) tile[pos * 4 + j] = pend_tile[pos * 4 + j];
          tile_vec[pos] = pend_vec[pos];
        }
        row_pending[u] = false;
      }
  };

  if (ntiles > 0) issue_rows(0, 0, IPT);
  for (int64_t t = 0; t < ntiles; ++t) {
    wait_all();
    if (!have) break;
    refill();
    const int64_t e0 = 4 * (vlo + t * T) - shift;
    const int64_t e1 = 4 * (vlo + (t + 1) * T) - shift;
    const int RSw = rows, NP = IPT / rows, RLw = 4 * rows;
    // xr[l][q RL + i]: value i of lane l's run in part q.  take(q) reads
    // part q at run_swz(q 64 RS + RS l + jj), each position holding the
    // tile vector the read expects (or the slice's last vector, past it),
    // then puts the same rows of the next tile in flight.
    std::vector<int64_t> xr((size_t)kWave * 4 * IPT, 0);
    bool taken[4] = {false, false, false, false};
    auto take = [&](int q) {
      if (q < 0 || q >= NP || taken[q]) fail("part read twice or out of range", q);
      taken[q] = true;
      for (int l = 0; l < kWave; ++l)
        for (int jj = 0; jj < RSw; ++jj) {
          const int want = q * kWave * RSw + l * RSw + jj;
          const int pos = run_swz(want, RSw);
          if (pos < 0 || pos >= kWave * IPT) fail("tile read out of bounds", pos);
          if (row_pending[pos / kWave]) fail("tile read of a row with a load in flight", t, pos);
          const int64_t expect = std::min(vlo + t * T + want, vhi - 1);
          if (tile_vec[pos] != expect) fail("tile position holds another vector", pos, tile_vec[pos], expect);
          for (int j = 0; j < 4; ++j) xr[(size_t)l * 4 * IPT + q * RLw + 4 * jj + j] = tile[(size_t)pos * 4 + j];
        }
      if (t + 1 < ntiles) issue_rows(t + 1, q * RSw, RSw);
    };

    auto try_runs = [&](int RS, int Q) -> bool {
      const int RL = 4 * RS;
      const int64_t f0 = e0 + (int64_t)kWave * RL * Q;
      const int64_t f1 = f0 + (int64_t)kWave * RL;
      const int vis = (int)std::min<int64_t>(kWave, fill - (s + 1));
      if (vis <= 0) return false;
      Lanes<int64_t> O;
      Lanes<bool> valid;
      int m = 0;
      for (int l = 0; l < kWave; ++l) {
        if (l < vis) {
          const int p = ring_pos(s + 1, l);
          if (ring_idx[p] != s + 1 + l) fail("stale offsets-ring entry", s + 1 + l, ring_idx[p]);
          O[l] = ring[p];
        } else {
          O[l] = kNone;
        }
        valid[l] = O[l] < std::min(f1, hi);
        m += valid[l];
      }
      for (int l = 0; l < kWave; ++l)
        if (valid[l] != (l < m)) fail("valid lanes are not a prefix", l, m);
      if (MUTATION == 4 ? m > vis || (m == vis && vis < kWave) : m >= vis) return false;
      Lanes<int> rel, r;
      for (int l = 0; l < kWave; ++l) {
        if (valid[l] && (O[l] < f0 || O[l] >= f1)) fail("start outside its part", O[l], f0, f1);
        rel[l] = valid[l] ? (int)(O[l] - f0) : 0;
        r[l] = rel[l] / RL;
      }
      for (int l = 0; l < kWave; ++l) {
        const int rn = r[(l + 1) & (kWave - 1)];  // DPP wave shift: lane + 1 (lane 63 unused)
        if (MUTATION != 3 && valid[l] && l + 1 < m && rn == r[l]) return false;
      }
      // start slots (LDS)
      unsigned slot[kWave];
      for (int l = 0; l < kWave; ++l) slot[l] = 0u;
      for (int l = 0; l < kWave; ++l)
        if (valid[l]) {
          if (r[l] < 0 || r[l] >= kWave) fail("start slot out of bounds", r[l]);
          slot[r[l]] = ((unsigned)(l + 1) << 16) | (unsigned)rel[l];
        }
      Lanes<unsigned> word;
      for (int l = 0; l < kWave; ++l) word[l] = slot[l];
      // lane l's run of this part
      std::vector<int64_t> xv((size_t)kWave * RL);
      for (int l = 0; l < kWave; ++l)
        for (int i = 0; i < RL; ++i) xv[(size_t)l * RL + i] = xr[(size_t)l * 4 * IPT + Q * RL + i];
      if (MUTATION != 6 && (f0 < lo || f1 > hi))
        for (int l = 0; l < kWave; ++l) {
          const int64_t p = f0 + (int64_t)RL * l;
          for (int i = 0; i < RL; ++i)
            if (!(p + i >= lo && p + i < hi)) xv[(size_t)l * RL + i] = 0;
        }
      Lanes<int64_t> v, head;
      Lanes<int> f;
      for (int l = 0; l < kWave; ++l) {
        const bool has = word[l] != 0u;
        const int bpos = has ? (int)(word[l] & 0xFFFFu) - RL * l : RL;
        if (has && (bpos < 0 || bpos >= RL)) fail("start outside its lane's run", l, bpos);
        int64_t run = 0, hd = 0;
        for (int i = 0; i < RL; ++i) {
          if (i > 0 && i == bpos) {
            hd = run;
            run = 0;
          }
          run += xv[(size_t)l * RL + i];
        }
        v[l] = run;
        head[l] = hd;
        f[l] = has ? 1 : 0;
      }
      // segmented inclusive scan: row shifts 1, 2, 4, 8 inside 16-lane
      // rows, then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31
      // into rows 2 and 3; an invalid source reads (0, 0)
      auto step = [&](auto src_of) {
        Lanes<int64_t> pv;
        Lanes<int> pf;
        for (int l = 0; l < kWave; ++l) {
          const int sl = src_of(l);
          pv[l] = sl >= 0 ? v[sl] : 0;
          pf[l] = sl >= 0 ? f[sl] : 0;
        }
        for (int l = 0; l < kWave; ++l) {
          v[l] = f[l] ? v[l] : pv[l] + v[l];
          f[l] = f[l] | pf[l];
        }
      };
      for (int k : {1, 2, 4, 8}) step([k](int l) { return (l % 16) >= k ? l - k : -1; });
      step([](int l) { return ((l / 16) & 1) ? (l / 16) * 16 - 1 : -1; });
      step([](int l) { return (l / 16) >= 2 ? 31 : -1; });
      for (int l = 0; l < kWave; ++l)
        if (!f[l]) v[l] = C + v[l];
      Lanes<int64_t> total;
      for (int l = 0; l < kWave; ++l) {
        const int64_t left = v[(l - 1) & (kWave - 1)];  // DPP wave shift: lane - 1 (lane 0 unused)
        total[l] = (l == 0 ? C : left) + head[l];
      }
      for (int l = 0; l < kWave; ++l) {
        const bool has = word[l] != 0u;
        const int k = (int)(word[l] >> 16) - 1;
        if (has && k > 0 && k < m) M.write_out(s + k, total[l]);
      }
      const int64_t c_next = lane_read(v, kWave - 1);
      if (m > 0) {
        const int r0 = r[0];
        const int64_t o0 = lane_read(O, 0);
        finish_piece(M, s, sa, o0, lane_read(total, r0), lo, hi, w, chunk);
        sa = lane_read(O, m - 1);
        sb = lane_read(O, MUTATION == 1 ? m - 1 : m);
        s += m;
      }
      C = c_next;
      ++M.parts_runs;
      return true;
    };

    // per-piece walk over the runs: the value xr[l][q RL + i] lies at tile
    // position q 64 RL + RL l + i
    auto masked_sum = [&](int ra, int rb) -> int64_t {
      if (ra > rb) fail("masked range inverted", ra, rb);
      if (ra < 0 || rb > 4 * T) fail("masked range outside the tile", ra, rb);
      int64_t sum = 0;
      for (int q = 0; q < NP; ++q)
        for (int l = 0; l < kWave; ++l)
          for (int i = 0; i < RLw; ++i) {
            const int k = q * kWave * RLw + RLw * l + i;
            if (k < ra || k >= rb) continue;
            if (!taken[q]) fail("piece walk reads a part not read from the tile", q, k);
            sum += xr[(size_t)l * 4 * IPT + q * RLw + i];
          }
      return sum;
    };
    auto pieces_from = [&](int q0) {
      ++M.parts_pieces;
      for (int q = q0 + 1; q < NP && MUTATION != 8; ++q) take(q);
      const int64_t p0 = e0 + (int64_t)q0 * kWave * RLw;
      auto relp = [&](int64_t e) { return (int)std::min(std::max(e - e0, (int64_t)0), 4 * T); };
      int64_t A = std::max(std::max(sa, lo), p0), Bb = std::min(sb, hi);
      while (have && Bb <= e1) {
        finish_piece(M, s, sa, sb, C + masked_sum(relp(A), relp(Bb)), lo, hi, w, chunk);
        C = 0;
        ++s;
        have = seek_segment(M, s, hi, E, end_slice, sa, sb);
        A = std::max(sa, lo);
        Bb = std::min(sb, hi);
      }
      if (have) C += masked_sum(relp(A), relp(Bb));
    };

    {
      for (int q = 0; q < NP; ++q) {
        take(q);
        if (!try_runs(RSw, q)) {
          pieces_from(q);
          break;
        }
      }
    }
  }
  if (have) {
    finish_piece(M, s, sa, sb, C, lo, hi, w, chunk);
    ++s;
    seek_segment(M, s, hi, E, end_slice, sa, sb);
  }
}

// k_seg_fixup: wavefront w sums the pieces of the cut segment that starts
// in slice w, in slice order.
void fixup(Machine& M) {
  for (int64_t w = 0; w < M.W; ++w) {
    const Carry c = M.slot(M.carry_out, w, "fix-up carry_out read out of bounds");
    if (c.epoch != M.epoch) fail("fix-up read a carry_out slot not written by this launch", w);
    if (c.seg < 0) continue;
    if (c.np < 1) fail("fix-up piece count below one", w, c.np);
    int64_t sum = c.val;
    for (int64_t k = w + 1; k < w + c.np; ++k) {
      const Carry& p = M.slot(M.carry_in, k, "fix-up carry_in read out of bounds");
      if (p.epoch != M.epoch) fail("fix-up read a carry_in slot not written by this launch", k);
      if (p.seg != c.seg) fail("fix-up read another segment's piece", k, p.seg, c.seg);
      sum += p.val;
    }
    M.write_out(c.seg, sum);
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s E L layout grid wg ipt shift seed\n", argv[0]);
    return 2;
  }
  Batch b;
  b.E = atoll(argv[1]);
  const int64_t L = atoll(argv[2]);
  const int layout = atoi(argv[3]);
  const int grid = atoi(argv[4]), wg = atoi(argv[5]), ipt = atoi(argv[6]);
  b.shift = atoi(argv[7]);
  const uint64_t seed = strtoull(argv[8], nullptr, 10);
  if (b.E < 0 || L < 1 || grid < 1 || wg < 64 || wg % 64 || wg > 512 || (ipt != 1 && ipt != 2 && ipt != 4) ||
      b.shift < 0 || b.shift > 3) {
    fprintf(stderr, "bad arguments\n");
    return 2;
  }
  // layout
  b.off.push_back(0);
  if (layout == 0) {
    for (int64_t e = 0; e < b.E;) {
      e = std::min(b.E, e + L);
      b.off.push_back(e);
    }
  } else {
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 12345;
    auto rnd = [&]() {
      st ^= st << 13;
      st ^= st >> 7;
      st ^= st << 17;
      return st;
    };
    for (int64_t e = 0; e < b.E;) {
      e = std::min(b.E, e + (int64_t)(rnd() % (uint64_t)(2 * L + 1)));
      b.off.push_back(e);
    }
  }
  b.nseg = (int64_t)b.off.size() - 1;
  b.out.assign(b.nseg, 0);
  b.writes.assign(b.nseg, 0);
  if (b.nseg < 1) {
    printf("{\"ok\": true, \"segments\": 0}\n");
    return 0;
  }
  // the reduce-by-key form is the one the device picks only under a mean
  // of kRunsMeanLen values; the emulation runs it regardless (forced form)
  Machine M(b, grid, wg, ipt);
  if (M.W > kMaxChunks) fail("grid has more wavefronts than carry slots", M.W);
  for (int64_t w = 0; w < M.W; ++w) wave_runs(M, w);
  fixup(M);
  // results
  int64_t e = 0;
  for (int64_t s = 0; s < b.nseg; ++s) {
    int64_t want = 0;
    for (; e < b.off[s + 1]; ++e) want += Batch::value(e);
    if (b.writes[s] != 1) fail("segment not written exactly once", s, b.writes[s]);
    if (b.out[s] != want) fail("wrong segment sum", s, b.out[s], want);
  }
  printf("{\"ok\": true, \"segments\": %lld, \"values\": %lld, \"wavefronts\": %lld, \"vector_loads\": %lld, "
         "\"offset_reads\": %lld, \"parts_reduce_by_key\": %lld, \"parts_piece_walk\": %lld, "
         "\"auto_form_is_runs\": %s}\n",
         (long long)b.nseg, (long long)b.E, (long long)M.W, M.vec_loads, M.offset_reads, M.parts_runs,
         M.parts_pieces, (b.E < kRunsMeanLen * b.nseg) ? "true" : "false");
  return 0;
}
