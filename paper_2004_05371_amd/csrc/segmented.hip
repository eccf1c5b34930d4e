// Batched segmented sum reduction in one persistent launch (gfx950).
//
// The paper's persistent-kernel reduction (Section VII-C, explicit
// synchronization) keeps one grid of blocks alive for the whole job.  Here a
// fixed grid handles a whole CSR batch of uneven segments:
//
//   * the concatenated values are cut into equal slices (chunk = ceil(E / S)
//     rounded up to 64 values), one per workgroup or, when the batch's mean
//     segment is short, one per wavefront, so every slice streams the same
//     number of bytes whatever the segment lengths;
//   * a slice finds its first segment by binary search in the offsets
//     (read through the scalar cache), then streams its values as one
//     sequence of tiles of 16-byte vectors (the next tile in flight while
//     the current one is added into fp32 TwoSum-compensated accumulators);
//   * a piece of a segment that ends in a tile is finished while the next
//     tile is in flight: by a DPP wavefront combine (wavefront slices), or
//     by a wavefront combine per wave whose results are completed in
//     batches of 64 pieces after one workgroup barrier (workgroup slices);
//   * a segment that lies inside the slice is written directly (binary64);
//     a piece of a segment that crosses a slice boundary goes to a carry
//     slot, and the pieces of that segment are summed in slice order in
//     binary64, either by the wavefront that publishes the last piece
//     (atomic ticket per owning slice; no co-residency needed,
//     graph-capturable) or, in the cooperative form, by the owning slice
//     after a grid barrier.
//
// Workgroup slices keep few concurrent streams (better DRAM locality) and
// suit long segments; wavefront slices let every wave walk its own pieces
// without barriers and suit short ones.  Empty segments write 0.  The
// result is deterministic for a given grid and workgroup size.
#include <algorithm>

#include "device_prims.h"
#include "internal.h"

namespace redsum {

struct SegArgs {
  const float* x;
  const int64_t* offsets;
  int64_t nseg;
  double* out;
  SegCarry* carry_in;   // piece of a segment that started before the slice
  SegCarry* carry_out;  // piece of a segment that starts in the slice and continues
  unsigned* tickets;    // per owning slice: pieces published so far
  BarrierWords* words;
  unsigned spin_limit;
  unsigned bar_groups;
};

// offsets[i] through the scalar data cache (the offsets are read-only for
// the whole launch), so the segment walk waits on scalar loads only and
// never on the vector loads of the stream in flight.
__device__ __forceinline__ int64_t offset_at(const int64_t* offsets, int64_t i) {
  return ((const __attribute__((address_space(4))) int64_t*)offsets)[i];
}

// Sum of the np pieces of a cut segment (owning slice o: carry_out[o], then
// carry_in[o+1 .. o+np-1]) by one wavefront: lane l adds pieces o+l,
// o+l+64, ... in order, then the fixed binary64 wavefront combine
// (returned to every lane).
__device__ __forceinline__ double combine_pieces(const SegArgs& a, int64_t o, int64_t np) {
  double v = 0.0;
  for (int64_t k = o + __lane_id(); k < o + np; k += kWave) v += k == o ? a.carry_out[o].val : a.carry_in[k].val;
  return wave_reduce_dpp<OpF64>(v);
}

// Completes, by one wavefront, the piece [max(sa, lo), min(sb, hi)) of
// segment s whose total is v: a whole segment is written; a piece of a cut
// segment is published in its carry slot (slice w), and the wavefront that
// completes the segment's ticket sums all of its pieces (ticket form), or
// the owning wavefront does so after the grid barrier (barrier form:
// *own_fix records the segment).
template <bool BARRIER>
__device__ __forceinline__ void finish_piece(const SegArgs& a, int64_t s, int64_t sa, int64_t sb, double v,
                                             int64_t lo, int64_t hi, int64_t w, int64_t chunk, int64_t* own_fix) {
  const int lane = __lane_id();
  if (sa >= lo && sb <= hi) {
    if (lane == 0) a.out[s] = v;
    return;
  }
  const int64_t o = sa / chunk;
  const int64_t np = (sb - 1) / chunk - o + 1;
  if constexpr (BARRIER) {
    if (lane == 0) {
      if (sa < lo)
        a.carry_in[w] = SegCarry{s, v};
      else
        a.carry_out[w] = SegCarry{s, v};
    }
    if (sa >= lo) *own_fix = s;
  } else {
    int last = 0;
    if (lane == 0) {
      if (sa < lo)
        a.carry_in[w] = SegCarry{s, v};
      else
        a.carry_out[w] = SegCarry{s, v};
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned tk = __hip_atomic_fetch_add(&a.tickets[o], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = tk == (unsigned)(np - 1);
    }
    if (__builtin_amdgcn_readfirstlane(last)) {  // this wave published the last piece
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const double t = combine_pieces(a, o, np);
      if (lane == 0) {
        a.out[s] = t;
        __hip_atomic_store(&a.tickets[o], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Moves the segment cursor s to the next non-empty segment that starts
// before hi, writing 0 (if `writer`) for the empty segments passed on the
// way (those at positions in [lo, hi), and, for the slice that ends at E,
// those at E).  Returns false when the slice holds no further segment.
__device__ __forceinline__ bool seek_segment(const SegArgs& a, int64_t& s, int64_t hi, int64_t E, bool end_slice,
                                             int64_t& sa, int64_t& sb, bool writer) {
  for (; s < a.nseg; ++s) {
    sa = offset_at(a.offsets, s);
    sb = offset_at(a.offsets, s + 1);
    if (sa >= hi && !(end_slice && sa == E)) return false;
    if (sa != sb) return true;
    if (writer) a.out[s] = 0.0;
  }
  return false;
}

// Adds to acc the elements of the thread's IPT vectors of one tile that lie
// in the tile-relative range [ra, rb) (0 <= ra <= rb <= 4 T): vector u of
// thread idx (0 <= idx < bs) starts at element 4 (u bs + idx) of the tile.
// A wave whose 256 elements of row u miss the range skips that row (the
// test is wave-uniform).  32-bit unsigned range test: r in [ra, rb) iff
// r - ra < rb - ra.
template <int IPT>
__device__ __forceinline__ void add_masked(CompF32* acc, const v4f* v, int bs, int idx, int ra, int rb) {
  const unsigned w = (unsigned)(rb - ra);
  const int wave0 = __builtin_amdgcn_readfirstlane(idx & ~(kWave - 1));
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int wb = 4 * (u * bs + wave0);  // first element of this wave's part of row u
    if (wb >= rb || wb + 4 * kWave <= ra) continue;
    const unsigned r = (unsigned)(4 * (u * bs + idx) - ra);
    v4f x = v[u];
    x.x = r < w ? x.x : 0.0f;
    x.y = r + 1u < w ? x.y : 0.0f;
    x.z = r + 2u < w ? x.z : 0.0f;
    x.w = r + 3u < w ? x.w : 0.0f;
    ModeF32Comp::add_vec(acc[u], x);
  }
}

// Whether any of the calling wave's rows of a workgroup tile meets [ra, rb).
template <int IPT>
__device__ __forceinline__ bool wave_touches(int bs, int ra, int rb) {
  const int wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~(kWave - 1));
  bool t = false;
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int wb = 4 * (u * bs + wave0);
    t = t || (wb < rb && wb + 4 * kWave > ra);
  }
  return t;
}

// Pieces whose workgroup combine is finished together, after one barrier.
constexpr int kBatch = 64;

struct PieceInfo {
  int64_t s, sa, sb;  // segment id and its bounds
};

// At most 512 threads per workgroup: a thread keeps two tiles of IPT
// 16-byte vectors and IPT compensated accumulators in registers, which for
// IPT = 8 needs more than the 128 VGPRs a 1024-thread workgroup allows.
constexpr int kSegMaxWG = 512;

// Batches whose mean segment holds fewer values than this take wavefront
// slices, the others workgroup slices (measured on MI355X: 64- to
// 4096-value segments run 2 to 8 times faster on wavefront slices, long
// ones about 10 to 30 % faster on workgroup slices).
constexpr int64_t kWaveSliceMeanLen = 16384;

// Wavefront-granular slices (short segments: every wave walks its own
// pieces, with no workgroup barrier): wavefront w of the grid owns slice
// w and streams it as tiles of 64 x IPT vectors.
template <int IPT, bool NT, bool BARRIER>
__device__ __forceinline__ void seg_wave_slices(const SegArgs& a) {
  using M = ModeF32Comp;
  const int nwaves = blockDim.x / kWave;
  const int lane = __lane_id();
  const int64_t w = (int64_t)blockIdx.x * nwaves + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t W = (int64_t)gridDim.x * nwaves;
  const int64_t nseg = a.nseg;
  const int64_t E = offset_at(a.offsets, nseg);
  const int64_t chunk = std::max<int64_t>(64, (((E + W - 1) / W) + 63) & ~(int64_t)63);
  const int64_t lo = std::min(w * chunk, E);
  const int64_t hi = std::min(lo + chunk, E);
  // The slice that ends at E also writes the empty segments that sit at
  // position E (for E == 0: slice 0).
  const bool end_slice = E > 0 ? (lo < E && hi == E) : (w == 0);

  // First s in [0, nseg] with offsets[s] >= lo (offsets[nseg] = E >= lo).
  int64_t L = 0, R = nseg;
  while (L < R) {
    const int64_t mid = (L + R) >> 1;
    if (offset_at(a.offsets, mid) >= lo)
      R = mid;
    else
      L = mid + 1;
  }
  // Segment L-1 crosses lo if it ends after lo.
  int64_t s = (L > 0 && offset_at(a.offsets, L) > lo) ? L - 1 : L;
  int64_t sa = 0, sb = 0;
  bool have = seek_segment(a, s, hi, E, end_slice, sa, sb, lane == 0);
  int64_t A = std::max(sa, lo), B = std::min(sb, hi);  // current piece

  // The slice is streamed as one sequence of tiles (64 x IPT 16-byte
  // vectors of the 16-byte-aligned base, the next tile's loads issued
  // before the current tile is added), whatever the segment boundaries.
  const int shift = (int)((reinterpret_cast<uintptr_t>(a.x) & 15) >> 2);
  const v4f* xa = reinterpret_cast<const v4f*>(a.x - shift);
  const int64_t vlo = (lo + shift) >> 2;
  const int64_t vhi = (hi + shift + 3) >> 2;  // vectors [vlo, vhi) hold the slice
  constexpr int64_t T = kWave * IPT;
  const int64_t ntiles = lo < hi ? (vhi - vlo + T - 1) / T : 0;

  CompF32 acc[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) acc[u] = M::zero();
  v4f cur[IPT], nxt[IPT];
  auto load_tile = [&](v4f* v, int64_t t) {
    const int64_t v0 = vlo + t * T + lane;
    if (vlo + (t + 1) * T <= vhi) {
#pragma unroll
      for (int u = 0; u < IPT; ++u) v[u] = load_vec<NT>(xa + v0 + u * kWave);
    } else {
#pragma unroll
      for (int u = 0; u < IPT; ++u)
        v[u] = v0 + u * kWave < vhi ? load_vec<NT>(xa + v0 + u * kWave) : v4f{0, 0, 0, 0};
    }
  };

  int64_t own_fix = -1;  // barrier form: the cut segment this slice owns
  if (ntiles > 0) load_tile(cur, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    // The current tile is complete before the next one is requested, so
    // nothing below waits on the loads in flight (on this target a wait
    // with stores and loads both pending would drain every load).
    __builtin_amdgcn_s_waitcnt(0);
    if (t + 1 < ntiles) load_tile(nxt, t + 1);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t e0 = 4 * (vlo + t * T) - shift;        // first element of the tile
    const int64_t e1 = 4 * (vlo + (t + 1) * T) - shift;  // one past its last
    auto rel = [&](int64_t e) { return (int)std::min(std::max(e - e0, (int64_t)0), 4 * T); };
    // Pieces that end in this tile.
    while (have && B <= e1) {
      add_masked<IPT>(acc, cur, kWave, lane, rel(A), rel(B));
      CompF32 tot = acc[0];
#pragma unroll
      for (int u = 1; u < IPT; ++u) tot = OpComp::add(tot, acc[u]);
#pragma unroll
      for (int u = 0; u < IPT; ++u) acc[u] = M::zero();
      tot = wave_reduce_dpp<OpComp>(tot);
      finish_piece<BARRIER>(a, s, sa, sb, comp_to_double(tot), lo, hi, w, chunk, &own_fix);
      ++s;
      have = seek_segment(a, s, hi, E, end_slice, sa, sb, lane == 0);
      A = std::max(sa, lo);
      B = std::min(sb, hi);
    }
    // The piece that continues past this tile.
    if (have) {
      if (A <= e0 && vlo + (t + 1) * T <= vhi) {
#pragma unroll
        for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], cur[u]);
      } else {
        add_masked<IPT>(acc, cur, kWave, lane, rel(A), rel(B));
      }
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) cur[u] = nxt[u];
  }
  if constexpr (BARRIER) {
    grid_barrier(a.words, gridDim.x, a.bar_groups, a.spin_limit);
    if (own_fix >= 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int64_t o = offset_at(a.offsets, own_fix) / chunk;
      const int64_t np = (offset_at(a.offsets, own_fix + 1) - 1) / chunk - o + 1;
      const double v = combine_pieces(a, o, np);
      if (lane == 0) a.out[own_fix] = v;
    }
  }
}

// Workgroup-granular slices (long segments: few streams, little per-piece
// work): workgroup g owns slice g, streams it as tiles of blockDim x IPT
// vectors, and finishes the pieces that end in a tile in batches of
// kBatch after one workgroup barrier, wave w finishing pieces w,
// w + nwaves, ...
template <int IPT, bool NT, bool BARRIER>
__device__ __forceinline__ void seg_workgroup_slices(const SegArgs& a) {
  using M = ModeF32Comp;
  // Per-wave partials of up to kBatch finished pieces, completed together
  // after one barrier.  Two buffers used alternately: a wave writes a
  // buffer again only after the next batch's barrier, which every wave
  // reaches after its reads of that buffer.
  __shared__ CompF32 part[2][kBatch][kMaxWavesPerWG];
  __shared__ PieceInfo info[2][kBatch];
  __shared__ int64_t own_fix;  // barrier form: cut segment this workgroup owns
  int buf = 0, nb = 0;
  const int64_t nseg = a.nseg;
  const int64_t E = offset_at(a.offsets, nseg);
  const int64_t G = gridDim.x;
  const int64_t g = blockIdx.x;
  const int64_t chunk = std::max<int64_t>(64, (((E + G - 1) / G) + 63) & ~(int64_t)63);
  const int64_t lo = std::min(g * chunk, E);
  const int64_t hi = std::min(lo + chunk, E);
  // The workgroup whose slice ends at E also writes the empty segments that
  // sit at position E (for E == 0: workgroup 0).
  const bool end_wg = E > 0 ? (lo < E && hi == E) : (g == 0);

  // First s in [0, nseg] with offsets[s] >= lo (offsets[nseg] = E >= lo).
  int64_t L = 0, R = nseg;
  while (L < R) {
    const int64_t mid = (L + R) >> 1;
    if (offset_at(a.offsets, mid) >= lo)
      R = mid;
    else
      L = mid + 1;
  }
  // Segment L-1 crosses lo if it ends after lo.
  int64_t s = (L > 0 && offset_at(a.offsets, L) > lo) ? L - 1 : L;
  int64_t sa = 0, sb = 0;
  bool have = seek_segment(a, s, hi, E, end_wg, sa, sb, threadIdx.x == 0);
  int64_t A = std::max(sa, lo), B = std::min(sb, hi);  // current piece

  // The slice is streamed as one sequence of tiles (blockDim x IPT 16-byte
  // vectors of the 16-byte-aligned base, the next tile's loads issued
  // before the current tile is added), whatever the segment boundaries: a
  // piece that ends inside a tile is finished (workgroup combine and
  // publication) while the next tile is in flight.
  const int shift = (int)((reinterpret_cast<uintptr_t>(a.x) & 15) >> 2);
  const v4f* xa = reinterpret_cast<const v4f*>(a.x - shift);
  const int64_t vlo = (lo + shift) >> 2;
  const int64_t vhi = (hi + shift + 3) >> 2;  // vectors [vlo, vhi) hold the slice
  const int64_t bs = blockDim.x;
  const int64_t T = bs * IPT;
  const int64_t ntiles = lo < hi ? (vhi - vlo + T - 1) / T : 0;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int nwaves = (int)bs / kWave;
  if (tid == 0) own_fix = -1;

  // Completes the batched pieces: wave w finishes pieces w, w + nwaves, ...
  auto flush = [&]() {
    __syncthreads();
    for (int j = wave; j < nb; j += nwaves) {
      CompF32 v = lane < nwaves ? part[buf][j][lane] : OpComp::zero();
      v = wave_reduce_dpp<OpComp>(v);
      const PieceInfo& pi = info[buf][j];
      finish_piece<BARRIER>(a, pi.s, pi.sa, pi.sb, comp_to_double(v), lo, hi, g, chunk, &own_fix);
    }
    buf ^= 1;
    nb = 0;
  };

  CompF32 acc[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) acc[u] = M::zero();
  v4f cur[IPT], nxt[IPT];
  auto load_tile = [&](v4f* v, int64_t t) {
    const int64_t v0 = vlo + t * T + tid;
    if (vlo + (t + 1) * T <= vhi) {
#pragma unroll
      for (int u = 0; u < IPT; ++u) v[u] = load_vec<NT>(xa + v0 + u * bs);
    } else {
#pragma unroll
      for (int u = 0; u < IPT; ++u) v[u] = v0 + u * bs < vhi ? load_vec<NT>(xa + v0 + u * bs) : v4f{0, 0, 0, 0};
    }
  };

  if (ntiles > 0) load_tile(cur, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    // The current tile is complete before the next one is requested, so
    // nothing below waits on the loads in flight (on this target a wait
    // with stores and loads both pending would drain every load).
    __builtin_amdgcn_s_waitcnt(0);
    if (t + 1 < ntiles) load_tile(nxt, t + 1);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t e0 = 4 * (vlo + t * T) - shift;        // first element of the tile
    const int64_t e1 = 4 * (vlo + (t + 1) * T) - shift;  // one past its last
    const int64_t span = e1 - e0;  // 4 T elements
    auto rel = [&](int64_t e) { return (int)std::min(std::max(e - e0, (int64_t)0), span); };
    // Pieces that end in this tile: each wave's share goes to the batch.
    while (have && B <= e1) {
      const int ra = rel(A), rb = rel(B);
      add_masked<IPT>(acc, cur, (int)bs, tid, ra, rb);
      CompF32 tot = acc[0];
#pragma unroll
      for (int u = 1; u < IPT; ++u) tot = OpComp::add(tot, acc[u]);
#pragma unroll
      for (int u = 0; u < IPT; ++u) acc[u] = M::zero();
      // A piece that started in this tile has nothing in the waves whose
      // rows miss it: they skip the wavefront combine.
      if (A < e0 || wave_touches<IPT>((int)bs, ra, rb)) tot = wave_reduce_dpp<OpComp>(tot);
      else tot = OpComp::zero();
      if (lane == 0) part[buf][nb][wave] = tot;
      if (tid == 0) info[buf][nb] = PieceInfo{s, sa, sb};
      if (++nb == kBatch) flush();
      ++s;
      have = seek_segment(a, s, hi, E, end_wg, sa, sb, threadIdx.x == 0);
      A = std::max(sa, lo);
      B = std::min(sb, hi);
    }
    // The piece that continues past this tile.
    if (have) {
      if (A <= e0 && vlo + (t + 1) * T <= vhi) {
#pragma unroll
        for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], cur[u]);
      } else {
        add_masked<IPT>(acc, cur, (int)bs, tid, rel(A), rel(B));
      }
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) cur[u] = nxt[u];
  }
  if (nb > 0) flush();
  if constexpr (BARRIER) {
    grid_barrier(a.words, gridDim.x, a.bar_groups, a.spin_limit);  // also a workgroup barrier
    const int64_t os = own_fix;
    if (os >= 0 && wave == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int64_t o = offset_at(a.offsets, os) / chunk;
      const int64_t np = (offset_at(a.offsets, os + 1) - 1) / chunk - o + 1;
      const double v = combine_pieces(a, o, np);
      if (lane == 0) a.out[os] = v;
    }
  }
}

template <int IPT, bool NT, bool BARRIER>
__global__ __launch_bounds__(kSegMaxWG) void k_segmented(SegArgs a) {
  const int64_t E = offset_at(a.offsets, a.nseg);
  if (E < kWaveSliceMeanLen * a.nseg)  // the same decision in every workgroup
    seg_wave_slices<IPT, NT, BARRIER>(a);
  else
    seg_workgroup_slices<IPT, NT, BARRIER>(a);
}

namespace {

int ipt_index(int ipt) { return ipt == 1 ? 0 : ipt == 2 ? 1 : ipt == 4 ? 2 : ipt == 8 ? 3 : -1; }

struct SegTable {
  const void* k[2][2][4];  // barrier, nontemporal, ipt index
  template <bool B, bool NT>
  void fill() {
    k[B][NT][0] = reinterpret_cast<const void*>(&k_segmented<1, NT, B>);
    k[B][NT][1] = reinterpret_cast<const void*>(&k_segmented<2, NT, B>);
    k[B][NT][2] = reinterpret_cast<const void*>(&k_segmented<4, NT, B>);
    k[B][NT][3] = reinterpret_cast<const void*>(&k_segmented<8, NT, B>);
  }
  SegTable() {
    fill<false, false>();
    fill<false, true>();
    fill<true, false>();
    fill<true, true>();
  }
};

const SegTable& seg_table() {
  static const SegTable t;
  return t;
}

}  // namespace

// Default (measured on MI355X for 10,000 log-uniform segments): one
// 512-thread workgroup per CU, 4 loads of 16 bytes per thread per tile.
red_plan default_seg_plan(int64_t nseg, const DeviceInfo& dev) {
  (void)nseg;
  red_plan p;
  p.variant = RED_VARIANT_ATOMIC;
  p.wg = 512;
  p.ipt = 4;
  p.grid = dev.cus;
  p.flags = RED_FLAG_NONTEMPORAL;
  return p;
}

int seg_max_coresident(int ipt, int wg, const DeviceInfo& dev, int* n_wg) {
  const int ii = ipt_index(ipt);
  if (ii < 0) return set_error(RED_EINVAL, "bad ipt %d", ipt);
  int per_cu = 0;
  RED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, seg_table().k[1][0][ii], wg, 0));
  *n_wg = per_cu * dev.cus;
  return RED_OK;
}

int seg_launch(const SegLaunch& sl, const float* x, const int64_t* offsets, int64_t nseg, double* out,
               Workspace* ws, hipStream_t s, const DeviceInfo& dev) {
  const red_plan& p = sl.plan;
  const int ii = ipt_index(p.ipt);
  if (ii < 0) return set_error(RED_EINVAL, "bad ipt %d", p.ipt);
  if (p.wg > kSegMaxWG) return set_error(RED_EINVAL, "segmented: at most %d threads per workgroup", kSegMaxWG);
  const bool barrier = p.variant == RED_VARIANT_PERSISTENT;
  if (!barrier && p.variant != RED_VARIANT_ATOMIC)
    return set_error(RED_EINVAL, "segmented: variant must be ATOMIC (ticket) or PERSISTENT (barrier)");
  int grid = p.grid > 0 ? p.grid : 4 * dev.cus;
  grid = std::max(1, std::min(grid, RED_MAX_GRID));
  // One carry slot and one ticket per wavefront slice.
  grid = std::min<int>(grid, (int)(kMaxChunks / (p.wg / kWave)));
  if (barrier) {
    int maxg = 0;
    int rc = seg_max_coresident(p.ipt, p.wg, dev, &maxg);
    if (rc) return rc;
    if (grid > maxg)
      return set_error(RED_EINVAL, "segmented persistent: grid %d exceeds %d co-resident workgroups",
                       grid, maxg);
  }
  SegArgs a;
  a.x = x;
  a.offsets = offsets;
  a.nseg = nseg;
  a.out = out;
  a.carry_in = ws->carry_in;
  a.carry_out = ws->carry_out;
  a.tickets = ws->seg_tickets;
  a.words = ws->words;
  a.spin_limit = watchdog_spins();
  a.bar_groups = ((p.flags & RED_FLAG_XCD) && dev.nxcc > 1) ? (kBarrierXcd | (unsigned)dev.nxcc)
                                                            : barrier_groups(grid);
  void* args[] = {&a};
  const bool nt = (p.flags & RED_FLAG_NONTEMPORAL) != 0;
  const bool coop = barrier && (p.flags & RED_FLAG_PLAIN_LAUNCH) == 0;
  const int slot = timer_begin(s);
  int rc = launch(seg_table().k[barrier ? 1 : 0][nt ? 1 : 0][ii], grid, p.wg, args, s, coop);
  timer_end(s, slot);
  return rc;
}

}  // namespace redsum
