// Batched segmented sum reduction in one persistent launch (gfx950).
//
// The paper's persistent-kernel reduction (Section VII-C, explicit
// synchronization) keeps one grid of blocks alive for the whole job.  Here a
// fixed grid of G workgroups handles a whole CSR batch of uneven segments:
//
//   * workgroup g owns the element slice [g*chunk, (g+1)*chunk) of the
//     concatenated values (chunk = ceil(E / G) rounded up to 64 elements),
//     so every workgroup streams the same number of bytes whatever the
//     segment lengths;
//   * it finds the first segment meeting its slice by binary search in the
//     offsets, then streams its slice as one sequence of tiles of 16-byte
//     vectors (the next tile in flight while the current one is added into
//     fp32 TwoSum-compensated accumulators); each piece of a segment is
//     finished by a wavefront + LDS combine as soon as its last tile is in,
//     so segment boundaries never drain the load pipeline;
//   * a segment that lies inside the slice is written directly (binary64);
//     a piece of a segment that crosses a slice boundary goes to a carry
//     slot, and the pieces of that segment are summed in slice order in
//     binary64, either by the last contributing workgroup (atomic ticket per
//     owning slice; no co-residency needed, graph-capturable) or, in the
//     cooperative form, by the owning workgroup after a grid barrier.
//
// Empty segments write 0.  The result is deterministic for a given grid.
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

// Pieces whose workgroup combine is finished together, after one barrier.
constexpr int kBatch = 64;

struct PieceInfo {
  int64_t s, sa, sb;  // segment id and its bounds
};

// Sum of the np pieces of a cut segment (owning slice o: carry_out[o], then
// carry_in[o+1 .. o+np-1]) by one wavefront: lane l adds pieces o+l,
// o+l+64, ... in order, then the fixed binary64 wavefront combine
// (returned to every lane).
__device__ __forceinline__ double combine_pieces(const SegArgs& a, int64_t o, int64_t np) {
  double v = 0.0;
  for (int64_t k = o + __lane_id(); k < o + np; k += kWave) v += k == o ? a.carry_out[o].val : a.carry_in[k].val;
  return wave_reduce_dpp<OpF64>(v);
}

// Completes one piece whose workgroup total is v, by one wavefront: a whole
// segment is written; a piece of a cut segment is published in its carry
// slot, and the piece that completes the segment's ticket sums all pieces
// (ticket form), or the owning workgroup does so after the grid barrier
// (barrier form: *own_fix records the segment).
template <bool BARRIER>
__device__ __forceinline__ void finish_piece(const SegArgs& a, const PieceInfo& p, double v, int64_t lo, int64_t hi,
                                             int64_t g, int64_t chunk, int64_t* own_fix) {
  const int lane = __lane_id();
  if (p.sa >= lo && p.sb <= hi) {
    if (lane == 0) a.out[p.s] = v;
    return;
  }
  const int64_t o = p.sa / chunk;
  const int64_t np = (p.sb - 1) / chunk - o + 1;
  int last = 0;
  if (lane == 0) {
    const SegCarry c{p.s, v};
    if (p.sa < lo)
      a.carry_in[g] = c;
    else
      a.carry_out[g] = c;
    if constexpr (BARRIER) {
      if (p.sa >= lo) *own_fix = p.s;
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned tk = __hip_atomic_fetch_add(&a.tickets[o], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = tk == (unsigned)(np - 1);
    }
  }
  if constexpr (!BARRIER) {
    if (__builtin_amdgcn_readfirstlane(last)) {  // this wave published the last piece
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const double w = combine_pieces(a, o, np);
      if (lane == 0) {
        a.out[p.s] = w;
        __hip_atomic_store(&a.tickets[o], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Moves the segment cursor s to the next non-empty segment that starts
// before hi, writing 0 for the empty segments passed on the way (those at
// positions in [lo, hi), and, for the workgroup whose slice ends at E, those
// at E).  Returns false when the slice holds no further segment.
__device__ __forceinline__ bool seek_segment(const SegArgs& a, int64_t& s, int64_t hi, int64_t E, bool end_wg,
                                             int64_t& sa, int64_t& sb) {
  for (; s < a.nseg; ++s) {
    sa = offset_at(a.offsets, s);
    sb = offset_at(a.offsets, s + 1);
    if (sa >= hi && !(end_wg && sa == E)) return false;
    if (sa != sb) return true;
    if (threadIdx.x == 0) a.out[s] = 0.0;
  }
  return false;
}

// The elements of the thread's IPT vectors of one tile that lie in the
// tile-relative range [ra, rb) (0 <= ra <= rb <= 4 T): vector u of thread
// tid starts at element 4 (u blockDim + tid) of the tile.  32-bit unsigned
// range test: r in [ra, rb) iff r - ra < rb - ra.
// A wave whose 256 elements of row u miss the range skips that row (the
// test is wave-uniform), so a short piece costs little beyond its combine.
template <int IPT>
__device__ __forceinline__ void add_masked(CompF32* acc, const v4f* v, int bs, int ra, int rb) {
  const unsigned w = (unsigned)(rb - ra);
  const int wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~(kWave - 1));
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int wb = 4 * (u * bs + wave0);  // first element of this wave's part of row u
    if (wb >= rb || wb + 4 * kWave <= ra) continue;
    const unsigned r = (unsigned)(4 * (u * bs + (int)threadIdx.x) - ra);
    v4f x = v[u];
    x.x = r < w ? x.x : 0.0f;
    x.y = r + 1u < w ? x.y : 0.0f;
    x.z = r + 2u < w ? x.z : 0.0f;
    x.w = r + 3u < w ? x.w : 0.0f;
    ModeF32Comp::add_vec(acc[u], x);
  }
}

// Whether any of the calling wave's rows of the tile meets [ra, rb).
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

template <int IPT, bool NT, bool BARRIER>
__global__ __launch_bounds__(1024) void k_segmented(SegArgs a) {
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
  bool have = seek_segment(a, s, hi, E, end_wg, sa, sb);
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
      finish_piece<BARRIER>(a, info[buf][j], comp_to_double(v), lo, hi, g, chunk, &own_fix);
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
      add_masked<IPT>(acc, cur, (int)bs, ra, rb);
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
      have = seek_segment(a, s, hi, E, end_wg, sa, sb);
      A = std::max(sa, lo);
      B = std::min(sb, hi);
    }
    // The piece that continues past this tile.
    if (have) {
      if (A <= e0 && vlo + (t + 1) * T <= vhi) {
#pragma unroll
        for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], cur[u]);
      } else {
        add_masked<IPT>(acc, cur, (int)bs, rel(A), rel(B));
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
  const bool barrier = p.variant == RED_VARIANT_PERSISTENT;
  if (!barrier && p.variant != RED_VARIANT_ATOMIC)
    return set_error(RED_EINVAL, "segmented: variant must be ATOMIC (ticket) or PERSISTENT (barrier)");
  int grid = p.grid > 0 ? p.grid : 4 * dev.cus;
  grid = std::max(1, std::min(grid, RED_MAX_GRID));
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
