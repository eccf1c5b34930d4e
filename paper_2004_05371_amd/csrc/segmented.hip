// Batched segmented sum reduction over a fixed grid (gfx950).
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
//     the current one is added into fp32 TwoSum-compensated accumulators,
//     or, in the reduce-by-key form, into binary64 per-lane runs);
//   * the segments are finished in one of three forms, chosen on the device
//     from the mean segment length: a piece that ends in a tile is finished
//     by a wavefront combine per wave, completed in batches of 64 pieces
//     after one workgroup barrier (workgroup slices); by one DPP wavefront
//     combine (wavefront slices); or, for very short segments, the wavefront
//     reduces by key over per-lane runs of consecutive values with a
//     segmented scan across its lanes (seg_wave_runs);
//   * a segment that lies inside the slice is written directly (binary64);
//     a piece of a segment that crosses a slice boundary goes to a carry
//     slot, and the pieces of that segment are summed in slice order in
//     binary64 by one wavefront: by the wavefront that publishes the last
//     piece (atomic ticket per owning slice, the default), in a second
//     kernel after the launch boundary (relaunch fix-up), or by the owning
//     slice after a grid barrier (co-resident grid); within one launch the
//     pieces are published with device-scope atomic stores, so neither the
//     ticket nor the barrier needs an L2 write-back or invalidation.
//
// Workgroup slices keep few concurrent streams (better DRAM locality) and
// suit long segments; wavefront slices let every wave walk its own pieces
// without barriers and suit short ones.  Empty segments write 0.  The
// result is deterministic for a given grid and workgroup size, and the
// three fix-ups give the same bits.
#include <algorithm>
#include <type_traits>

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
  int form;  // SegForm: automatic, or one form forced
  int grid;  // workgroups of the slice kernel
  int wg;    // threads per workgroup of the slice kernel
};

// How the pieces of a segment cut by slice boundaries are summed.
enum SegFix : int {
  kFixTicket = 0,    // the wavefront that publishes the last piece (atomic ticket)
  kFixBarrier = 1,   // the owning slice, after a grid barrier (co-resident grid)
  kFixRelaunch = 2,  // a second kernel, after the implicit barrier between launches
};

// How the slices are cut and walked.
enum SegForm : int {
  kSegAuto = 0,        // chosen on the device from the mean segment length
  kSegWorkgroup = 1,   // workgroup slices
  kSegWavePieces = 2,  // wavefront slices, one combine per piece
  kSegWaveRuns = 3,    // wavefront slices, reduce-by-key over lane runs
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
// (returned to every lane).  The pieces are read with device-scope atomic
// loads: the ticket and grid-barrier fix-ups read them in the launch that
// published them, with no acquire.
__device__ __forceinline__ double combine_pieces(const SegArgs& a, int64_t o, int64_t np) {
  double v = 0.0;
  for (int64_t k = o + __lane_id(); k < o + np; k += kWave)
    v += load_published(k == o ? &a.carry_out[o].val : &a.carry_in[k].val);
  return wave_reduce_dpp<OpF64>(v);
}

// A carry slot published to the other workgroups of the same launch.
__device__ __forceinline__ void publish_carry(SegCarry* slot, int64_t s, double v, int64_t np) {
  publish(&slot->seg, (long long)s);
  publish(&slot->val, v);
  publish(&slot->np, (long long)np);
}

// Completes, by one wavefront, the piece [max(sa, lo), min(sb, hi)) of
// segment s whose total is v: a whole segment is written; a piece of a cut
// segment is published in its carry slot (slice w), and the wavefront that
// completes the segment's ticket sums all of its pieces (ticket fix-up), or
// the owning wavefront does so after the grid barrier (barrier fix-up:
// *own_fix records the segment), or the fix-up kernel that follows does
// (relaunch fix-up: the slot is an ordinary store, made visible by the
// kernel boundary).  Within one launch the slots are published with
// device-scope atomic stores, waited for before the ticket or the barrier,
// so no workgroup writes back its L2 or invalidates it.
template <int FIX>
__device__ __forceinline__ void finish_piece(const SegArgs& a, int64_t s, int64_t sa, int64_t sb, double v,
                                             int64_t lo, int64_t hi, int64_t w, int64_t chunk, int64_t* own_fix) {
  const int lane = __lane_id();
  if (sa >= lo && sb <= hi) {
    if (lane == 0) a.out[s] = v;
    return;
  }
  const int64_t o = sa / chunk;
  const int64_t np = (sb - 1) / chunk - o + 1;
  if constexpr (FIX == kFixRelaunch) {
    if (lane == 0) {
      if (sa < lo)
        a.carry_in[w] = SegCarry{s, v, np};
      else
        a.carry_out[w] = SegCarry{s, v, np};
    }
  } else if constexpr (FIX == kFixBarrier) {
    if (lane == 0) publish_carry(sa < lo ? &a.carry_in[w] : &a.carry_out[w], s, v, np);
    if (sa >= lo) *own_fix = s;
  } else {
    int last = 0;
    if (lane == 0) {
      publish_carry(sa < lo ? &a.carry_in[w] : &a.carry_out[w], s, v, np);
      drain_stores();
      const unsigned tk = __hip_atomic_fetch_add(&a.tickets[o], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = tk == (unsigned)(np - 1);
    }
    if (__builtin_amdgcn_readfirstlane(last)) {  // this wave published the last piece
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
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

// The segment that holds element lo of a non-empty slice, or for an empty
// slice the first one that starts at or after lo: the first s in
// [0, nseg] with offsets[s] >= lo by binary search (offsets[nseg] = E >= lo),
// stepped back by one when segment s-1 crosses lo.
__device__ __forceinline__ int64_t first_segment(const SegArgs& a, int64_t lo) {
  int64_t L = 0, R = a.nseg;
  while (L < R) {
    const int64_t mid = (L + R) >> 1;
    if (offset_at(a.offsets, mid) >= lo)
      R = mid;
    else
      L = mid + 1;
  }
  return (L > 0 && offset_at(a.offsets, L) > lo) ? L - 1 : L;
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

// Batches whose mean segment holds fewer values than this take the
// reduce-by-key form of the wavefront slices (plans of at most 4 loads per
// thread).  Measured on MI355X with 2^28 values, 512 x 4, two workgroups
// per CU: 4.7 TB/s against 0.9 per piece at 64 values, 5.7 against 5.0 at
// 512, even at 1024.
constexpr int64_t kRunsMeanLen = 1024;

// Wavefront-granular slices (short segments: every wave walks its own
// pieces, with no workgroup barrier): wavefront w of the grid owns slice
// w and streams it as tiles of 64 x IPT vectors.
template <int IPT, bool NT, int FIX>
__device__ __forceinline__ void seg_wave_slices(const SegArgs& a) {
  // Barrier fix-up: thread 0 holds the barrier generation of this launch.
  unsigned gen = FIX == kFixBarrier ? grid_barrier_gen(a.words) : 0u;
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
  // Relaunch fix-up: the slot says "no cut segment starts here" unless a
  // later store by the same lane replaces it.
  if constexpr (FIX == kFixRelaunch)
    if (lane == 0) a.carry_out[w] = SegCarry{-1, 0.0, 0};

  int64_t s = first_segment(a, lo);
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
      finish_piece<FIX>(a, s, sa, sb, comp_to_double(tot), lo, hi, w, chunk, &own_fix);
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
  if constexpr (FIX == kFixBarrier) {
    grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);
    if (own_fix >= 0) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the pieces are loaded as published
      const int64_t o = offset_at(a.offsets, own_fix) / chunk;
      const int64_t np = (offset_at(a.offsets, own_fix + 1) - 1) / chunk - o + 1;
      const double v = combine_pieces(a, o, np);
      if (lane == 0) a.out[own_fix] = v;
    }
  }
}

// f(integral_constant<B>), ..., f(integral_constant<E - 1>); the _while
// form stops after the first call that returns false.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for_while(F&& f) {
  if constexpr (B < E) {
    if (f(std::integral_constant<int, B>{})) static_for_while<B + 1, E>(f);
  }
}

// Reduce-by-key form of the wavefront slices, for very short segments.
//
// Each tile of 64 x IPT 16-byte vectors (256 IPT contiguous values) is
// walked in parts of RS rows (fewer rows when the mean segment is short),
// and in each part lane l holds the run of RL = 4 RS consecutive values
// that starts at value RL l of the part.  The tile comes into LDS by
// direct-to-LDS loads, each lane fetching the vector that the run reads
// expect at its position, so the loads hold no registers while in flight;
// a part's rows are loaded for the next tile as soon as the part has been
// read.  The starts of the segments that follow the open one come from a
// ring of the offsets held in LDS (kRing entries ahead of the walk,
// refilled a tile ahead).  When fewer than 64 segments start in a part and
// no run holds two starts:
//   * each lane sums its run in binary64, cut at the start it holds (if
//     any) into a head, the end of the segment open on its left, and a
//     tail;
//   * a segmented inclusive scan of the tails in binary64 across the lanes,
//     seeded with the slice's partial of the open segment, gives every lane
//     the partial of the segment open at its right end;
//   * a lane that holds a start completes the segment that ends there (its
//     head plus the scan of the lane on its left): it writes the sum when
//     the segment began in the part, and the first start of the part
//     closes the segment that was open, which may have begun before the
//     slice and goes through finish_piece.
// Other parts (an empty segment, two starts in one run, 64 starts or more)
// and the rest of their tile are finished piece by piece as in
// seg_wave_slices, the open partial carried in binary64 between the two.
constexpr int kRing = 384;        // offsets entries held in LDS per wavefront
constexpr int kCpolNT = 2;        // the nontemporal bit of a load's cache policy
constexpr int kWaitLds = 0xC07F;  // s_waitcnt lgkmcnt(0): LDS reads returned, other counters free
constexpr int kWaveShl1 = 0x130;  // DPP wave_shl:1: lane l receives lane l + 1 (lane 63 receives 0)
constexpr int kWaveShr1 = 0x138;  // DPP wave_shr:1: lane l receives lane l - 1 (lane 0 receives 0)

struct RunLds {
  v4f tile[kWave * 4];   // one tile of up to 4 rows, swizzled
  unsigned slot[kWave];  // per lane run: (k + 1) << 16 | tile position of start k, or 0
  int64_t ring[kRing];   // offsets[i] at i mod kRing, for i in [fill - kRing, fill)
};

// LDS words written by one lane and read by another inside a wavefront.
// The wavefront's LDS instructions execute in program order, so ordinary
// LDS loads and stores suffice; the accesses are relaxed atomics on
// LDS-space pointers (no compiler may forward a lane's own store to its
// load, as it could for plain data) behind compiler-only fences (keeping
// program order).  A volatile access through a generic pointer would be
// compiled as a flat access with a wait for every outstanding global load.
template <class T>
using LdsPtr = __attribute__((address_space(3))) T*;

template <class T>
__device__ __forceinline__ LdsPtr<T> lds_ptr(T* p) {
  return (LdsPtr<T>)p;
}

template <class T>
__device__ __forceinline__ void lds_put(LdsPtr<T> p, int i, T v) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __atomic_store_n(p + i, v, __ATOMIC_RELAXED);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <class T>
__device__ __forceinline__ T lds_get(LdsPtr<T> p, int i) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const T v = __atomic_load_n(p + i, __ATOMIC_RELAXED);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return v;
}

// The same accesses while a direct-to-LDS load fills another LDS region.
// The compiler cannot tell the regions apart, so before any LDS access it
// would wait for every load in flight.  Written as inline assembly, which
// its wait insertion does not treat as a memory access, each access waits
// only for itself (lgkmcnt(0) in the same block, so no register is read or
// reused before the LDS has answered).
template <class T>
__device__ __forceinline__ unsigned lds_addr(LdsPtr<T> p, int i) {
  return (unsigned)(uintptr_t)(p + i);
}

__device__ __forceinline__ void lds_put_u32_now(LdsPtr<unsigned> p, int i, unsigned v) {
  asm volatile("ds_write_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : : "v"(lds_addr(p, i)), "v"(v) : "memory");
}

__device__ __forceinline__ unsigned lds_get_u32_now(LdsPtr<unsigned> p, int i) {
  unsigned v;
  asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(lds_addr(p, i)) : "memory");
  return v;
}

__device__ __forceinline__ int64_t lds_get_i64_now(LdsPtr<int64_t> p, int i) {
  int64_t v;
  asm volatile("ds_read_b64 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(lds_addr(p, i)) : "memory");
  return v;
}

// Position in the tile buffer of the part's vector i (parts of RS rows):
// within each group of 16 vectors the low bits are XOR-ed so that the run
// reads (lane l, vector RS l + j) of 16 consecutive lanes fall in distinct
// 16-byte bank groups.  The map is its own inverse and keeps each vector in
// its row, so the load that fills position 64 u + l fetches vector
// run_swz(64 u + l) and each load instruction still reads one contiguous
// KB.
template <int RS>
__device__ __forceinline__ int run_swz(int i) {
  return i ^ ((i >> 4) & (RS - 1));
}

// The values and the wavefront's three LDS regions come in as distinct
// restrict pointers: the compiler then knows that the ring and slot
// accesses cannot touch the tile that a direct-to-LDS load is filling, and
// does not wait for that load before them.
template <int IPT, bool NT, int FIX>
__device__ static void seg_wave_runs_in(const SegArgs& a, const float* __restrict__ x,
                                        const LdsPtr<v4f> __restrict__ tile,
                                                 const LdsPtr<unsigned> __restrict__ slot,
                                                 const LdsPtr<int64_t> __restrict__ ring) {
  // Barrier fix-up: thread 0 holds the barrier generation of this launch.
  unsigned gen = FIX == kFixBarrier ? grid_barrier_gen(a.words) : 0u;
  static_assert(IPT <= 4, "runs of at most 16 values");
  const int nwaves = blockDim.x / kWave;
  const int lane = __lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t w = (int64_t)blockIdx.x * nwaves + wv;
  const int64_t W = (int64_t)gridDim.x * nwaves;
  const int64_t nseg = a.nseg;
  const int64_t E = offset_at(a.offsets, nseg);
  const int64_t chunk = std::max<int64_t>(64, (((E + W - 1) / W) + 63) & ~(int64_t)63);
  const int64_t lo = std::min(w * chunk, E);
  const int64_t hi = std::min(lo + chunk, E);
  const bool end_slice = E > 0 ? (lo < E && hi == E) : (w == 0);
  // Relaunch fix-up: the slot says "no cut segment starts here" unless a
  // later store by the same lane replaces it.
  if constexpr (FIX == kFixRelaunch)
    if (lane == 0) a.carry_out[w] = SegCarry{-1, 0.0, 0};

  int64_t s = first_segment(a, lo);
  int64_t sa = 0, sb = 0;
  bool have = seek_segment(a, s, hi, E, end_slice, sa, sb, lane == 0);
  double C = 0.0;  // partial of segment s over [max(sa, lo), current position)

  const int shift = (int)((reinterpret_cast<uintptr_t>(x) & 15) >> 2);
  const v4f* xa = reinterpret_cast<const v4f*>(x - shift);
  const int64_t vlo = (lo + shift) >> 2;
  const int64_t vhi = (hi + shift + 3) >> 2;
  constexpr int64_t T = kWave * IPT;
  const int64_t ntiles = lo < hi ? (vhi - vlo + T - 1) / T : 0;

  // Offsets ring in LDS: entry i mod kRing holds offsets[i] (INT64_MAX
  // past nseg) for i in [fill - kRing, fill).  At the top of a tile, when
  // every load has completed, the blocks of 64 entries loaded at the top of
  // the previous tile are written, and up to three more are requested, as
  // many as fit without overwriting entries from s + 1 on.  A (sub-)tile
  // reads entries s + 1 .. s + 64, those that are in the ring.
  auto off_entry = [&](int64_t i) -> int64_t { return i <= nseg ? a.offsets[i] : INT64_MAX; };
  int64_t fill = 0;
  int npend = 0;
  int64_t pend0 = 0, pend1 = 0, pend2 = 0;
  // (base + lane) mod kRing; base is wave-uniform and below 2^31 + 4 kRing
  // (nseg < 2^31), so the modulo is a 32-bit one.
  auto ring_pos = [&](int64_t base) {
    const int h = (int)((unsigned)__builtin_amdgcn_readfirstlane((int)base) % (unsigned)kRing) + lane;
    return h >= kRing ? h - kRing : h;
  };
  auto put = [&](int64_t v, int64_t base) { lds_put(ring, ring_pos(base), v); };
  auto refill = [&]() {
    if (npend > 0) put(pend0, fill);
    if (npend > 1) put(pend1, fill + kWave);
    if (npend > 2) put(pend2, fill + 2 * kWave);
    fill += (int64_t)npend * kWave;
    npend = 0;
    if (fill - (s + 1) < kWave) {  // first tile, or after a long stretch walked piece by piece
      fill = s + 1;
      put(off_entry(fill + lane), fill);
      put(off_entry(fill + kWave + lane), fill + kWave);
      put(off_entry(fill + 2 * kWave + lane), fill + 2 * kWave);
      fill += 3 * kWave;
    }
    npend = (int)std::min<int64_t>(3, (kRing - (fill - (s + 1))) / kWave);
    if (npend > 0) pend0 = off_entry(fill + lane);
    if (npend > 1) pend1 = off_entry(fill + kWave + lane);
    if (npend > 2) pend2 = off_entry(fill + 2 * kWave + lane);
  };
  // Batches whose mean segment is short walk each tile in parts of fewer
  // rows, so that a part holds fewer than 64 starts: halves under a mean of
  // 32 values, quarters (4 loads per thread) under 12.
  const int nparts = (IPT >= 4 && E < 12 * nseg) ? 4 : (IPT >= 2 && E < 32 * nseg) ? 2 : 1;

  // Tiles arrive by direct-to-LDS loads, so no registers are held while a
  // tile is in flight.  Load instruction u writes lane i's vector at tile
  // position 64 u + i, and lane i fetches the tile vector that the run
  // reads expect there (run_swz is its own inverse, and it permutes within
  // groups of 16 vectors, so each instruction still reads 1 KB in one
  // piece).  Positions past the slice's last vector fetch that vector
  // again; the values they hold lie at or past hi and are masked out.
  const int rows = IPT / nparts;  // rows per part
  auto issue_rows = [&](int64_t t, int u0, int nrows) {
    const int64_t vb = vlo + t * T;
#pragma unroll
    for (int u = u0; u < u0 + nrows; ++u) {
      const int pos = u * kWave + lane;
      const int64_t g = std::min<int64_t>(vb + (pos ^ ((pos >> 4) & (rows - 1))), vhi - 1);  // run_swz<rows>(pos)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(xa + g),
                                       (LdsPtr<void>)(tile + u * kWave), 16, 0,
                                       NT ? kCpolNT : 0);
    }
  };

  int64_t own_fix = -1;
  if (ntiles > 0) issue_rows(0, 0, IPT);
  // The tiles walked in parts of RS rows: part q's values are
  // [e0 + 256 RS q, e0 + 256 RS (q + 1)), and lane l holds their run
  // [256 RS q + 4 RS l, + 4 RS) as xr[4 RS q .. 4 RS q + 4 RS).  The loop
  // over the tiles is instantiated per part size, so that the registers
  // one layout keeps across the loop are not added to another's.
  auto walk = [&](auto rs_tag) {
    constexpr int RS = decltype(rs_tag)::value;
    constexpr int NP = IPT / RS;
    constexpr int RL = 4 * RS;  // values per lane run
    constexpr int64_t P = (int64_t)kWave * RL;
    for (int64_t t = 0; t < ntiles; ++t) {
      // Tile t is in LDS and every offsets load has completed here.
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (!have) break;  // the slice is finished, and no load is in flight
      refill();
      const int64_t e0 = 4 * (vlo + t * T) - shift;
      const int64_t e1 = 4 * (vlo + (t + 1) * T) - shift;
      float xr[4 * IPT];
      // Reads part Q's runs.  Its rows then hold nothing else that is still
      // to be read, so the same rows of the next tile go in flight: a part
      // holds only its own runs in registers while it is walked.
      auto take = [&](auto q_tag) {
        constexpr int Q = decltype(q_tag)::value;
#pragma unroll
        for (int jj = 0; jj < RS; ++jj) {
          const v4f y = tile[run_swz<RS>(Q * kWave * RS + lane * RS + jj)];
          xr[Q * RL + 4 * jj] = y.x;
          xr[Q * RL + 4 * jj + 1] = y.y;
          xr[Q * RL + 4 * jj + 2] = y.z;
          xr[Q * RL + 4 * jj + 3] = y.w;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(kWaitLds);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (t + 1 < ntiles) issue_rows(t + 1, Q * RS, RS);
      };

      // Reduce-by-key walk over part Q (values [f0, f1)); returns false,
      // having changed nothing, when the part needs the per-piece walk.
      auto try_runs = [&](auto q_tag) -> bool {
        constexpr int Q = decltype(q_tag)::value;
        const int64_t f0 = e0 + (int64_t)kWave * RL * Q;
        const int64_t f1 = f0 + (int64_t)kWave * RL;
        // Entries s + 1 .. s + vis are in the ring; a view of fewer than 64
        // must end past the part to show every start in it.
        const int vis = (int)std::min<int64_t>(kWave, fill - (s + 1));
        if (vis <= 0) return false;
        // O: the start of segment s + 1 + lane
        const int64_t O = lane < vis ? lds_get_i64_now(ring, ring_pos(s + 1)) : INT64_MAX;
        const bool valid = O < std::min(f1, hi);
        const int m = __popcll(__ballot(valid));  // the valid lanes are 0 .. m-1
        if (m >= vis) return false;
        const int rel = valid ? (int)(O - f0) : 0;
        const int r = rel / RL;  // lane whose run holds start `lane`
        const int rn = dpp_move<kWaveShl1, 0xF, 0xF>(r);  // lane + 1's run (lane 63: unused)
        const bool clash = valid && lane + 1 < m && rn == r;
        if (__ballot(clash) != 0) return false;
        // Start k (lane k) tells lane r_k where it lies.
        lds_put_u32_now(slot, lane, 0u);
        if (valid) lds_put_u32_now(slot, r, ((unsigned)(lane + 1) << 16) | (unsigned)rel);
        const unsigned word = lds_get_u32_now(slot, lane);
        float xv[RL];
#pragma unroll
        for (int i = 0; i < RL; ++i) xv[i] = xr[Q * RL + i];
        if (f0 < lo || f1 > hi) {  // values outside the slice are not its own
          const int64_t p = f0 + (int64_t)RL * lane;
#pragma unroll
          for (int i = 0; i < RL; ++i) xv[i] = (p + i >= lo && p + i < hi) ? xv[i] : 0.0f;
        }
        const bool has = word != 0u;
        const int b = has ? (int)(word & 0xFFFFu) - RL * lane : RL;  // the start's place in the run
        // The run's head and tail in binary64: an fp32 value widens exactly,
        // and each of the at most RL - 1 additions rounds once, at 2^-53.
        double run = 0.0, head = 0.0;
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          if (i > 0) {
            const bool at = i == b;
            head = at ? run : head;
            run = at ? 0.0 : run;
          }
          run += (double)xv[i];
        }
        double v = run;
        int f = has ? 1 : 0;
        wave_segscan(v, f);
        if (!f) v = C + v;  // lanes 0 .. l hold no start: the open segment continues
        const double left = dpp_move<kWaveShr1, 0xF, 0xF>(v);  // lane - 1's scan (lane 0: unused)
        const double total = (lane == 0 ? C : left) + head;
        const int k = (int)(word >> 16) - 1;
        if (has && k > 0 && k < m) a.out[s + k] = total;  // segment s + k lies in the part
        const double c_next = read_lane(v, kWave - 1);
        if (m > 0) {
          const int r0 = __builtin_amdgcn_readfirstlane(r);
          const int64_t o0 = read_lane(O, 0);
          finish_piece<FIX>(a, s, sa, o0, read_lane(total, r0), lo, hi, w, chunk, &own_fix);
          sa = read_lane(O, m - 1);
          sb = read_lane(O, m);
          s += m;
        }
        C = c_next;
        return true;
      };

      // Piece by piece, as in seg_wave_slices, over the tile's values from
      // part Q0 on, with the open partial C: each lane adds its values of a
      // piece (tile positions [ra, rb)) by compensated fp32 adds, then the
      // wavefront combine.  Parts Q0 + 1 .. NP - 1 are read first.
      auto pieces_from = [&](auto q_tag) {
        constexpr int Q0 = decltype(q_tag)::value;
        static_for<Q0 + 1, NP>(take);
        auto relp = [&](int64_t e) { return (int)std::min(std::max(e - e0, (int64_t)0), 4 * T); };
        auto piece_sum = [&](int ra, int rb) {
          const unsigned wd = (unsigned)(rb - ra);
          CompF32 acc = ModeF32Comp::zero();
#pragma unroll
          for (int q = Q0; q < NP; ++q) {
            if (q * kWave * RL >= rb || (q + 1) * kWave * RL <= ra) continue;
            const unsigned r = (unsigned)(q * kWave * RL + RL * lane - ra);
#pragma unroll
            for (int i = 0; i < RL; ++i) ModeF32Comp::add_elem(acc, r + i < wd ? xr[q * RL + i] : 0.0f);
          }
          return comp_to_double(wave_reduce_dpp<OpComp>(acc));
        };
        int64_t A = std::max(std::max(sa, lo), e0 + Q0 * P), B = std::min(sb, hi);
        while (have && B <= e1) {
          finish_piece<FIX>(a, s, sa, sb, C + piece_sum(relp(A), relp(B)), lo, hi, w, chunk, &own_fix);
          C = 0.0;
          ++s;
          have = seek_segment(a, s, hi, E, end_slice, sa, sb, lane == 0);
          A = std::max(sa, lo);
          B = std::min(sb, hi);
        }
        if (have) C += piece_sum(relp(A), relp(B));
      };

      // Parts in order; the first part that cannot take the reduce-by-key
      // walk, and the rest of the tile, go piece by piece.
      static_for_while<0, NP>([&](auto q_tag) -> bool {
        take(q_tag);
        if (try_runs(q_tag)) return true;
        pieces_from(q_tag);
        return false;
      });
    }
  };
  if constexpr (IPT == 4) {
    if (nparts == 4)
      walk(std::integral_constant<int, 1>{});
    else if (nparts == 2)
      walk(std::integral_constant<int, 2>{});
    else
      walk(std::integral_constant<int, 4>{});
  } else if constexpr (IPT == 2) {
    if (nparts == 2)
      walk(std::integral_constant<int, 1>{});
    else
      walk(std::integral_constant<int, 2>{});
  } else {
    walk(std::integral_constant<int, 1>{});
  }
  if (have) {  // the segment open at the slice's end ends at or after hi
    finish_piece<FIX>(a, s, sa, sb, C, lo, hi, w, chunk, &own_fix);
    ++s;
    seek_segment(a, s, hi, E, end_slice, sa, sb, lane == 0);  // empty segments at E
  }
  if constexpr (FIX == kFixBarrier) {
    grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);
    if (own_fix >= 0) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the pieces are loaded as published
      const int64_t o = offset_at(a.offsets, own_fix) / chunk;
      const int64_t np = (offset_at(a.offsets, own_fix + 1) - 1) / chunk - o + 1;
      const double v = combine_pieces(a, o, np);
      if (lane == 0) a.out[own_fix] = v;
    }
  }
}

template <int IPT, bool NT, int FIX>
__device__ __forceinline__ void seg_wave_runs(const SegArgs& a, RunLds* lds_all) {
  RunLds& L = lds_all[__builtin_amdgcn_readfirstlane(threadIdx.x / kWave)];
  seg_wave_runs_in<IPT, NT, FIX>(a, a.x, lds_ptr(L.tile), lds_ptr(L.slot), lds_ptr(L.ring));
}

// Workgroup-granular slices (long segments: few streams, little per-piece
// work): workgroup g owns slice g, streams it as tiles of blockDim x IPT
// vectors, and finishes the pieces that end in a tile in batches of
// kBatch after one workgroup barrier, wave w finishing pieces w,
// w + nwaves, ...
// Per-wave partials of up to kBatch finished pieces, completed together
// after one barrier.  Two buffers used alternately: a wave writes a buffer
// again only after the next batch's barrier, which every wave reaches after
// its reads of that buffer.
struct WorkgroupLds {
  CompF32 part[2][kBatch][kMaxWavesPerWG];
  PieceInfo info[2][kBatch];
  int64_t own_fix;  // barrier form: cut segment this workgroup owns
};

template <int IPT, bool NT, int FIX>
__device__ __forceinline__ void seg_workgroup_slices(const SegArgs& a, WorkgroupLds& lds) {
  // Barrier fix-up: thread 0 holds the barrier generation of this launch.
  unsigned gen = FIX == kFixBarrier ? grid_barrier_gen(a.words) : 0u;
  using M = ModeF32Comp;
  auto& part = lds.part;
  auto& info = lds.info;
  int64_t& own_fix = lds.own_fix;
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

  int64_t s = first_segment(a, lo);
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
  // Relaunch fix-up: "no cut segment starts here" unless a store after the
  // first batch barrier replaces it.  The fix-up kernel looks at one slot
  // per wavefront of the grid, so the other waves also clear the slots
  // [G, G * nwaves) that workgroup slices do not use.
  if constexpr (FIX == kFixRelaunch) {
    if (tid == 0) a.carry_out[g] = SegCarry{-1, 0.0, 0};
    if (wave > 0 && lane == 0) a.carry_out[G + g * (nwaves - 1) + (wave - 1)] = SegCarry{-1, 0.0, 0};
  }

  // Completes the batched pieces: wave w finishes pieces w, w + nwaves, ...
  auto flush = [&]() {
    __syncthreads();
    for (int j = wave; j < nb; j += nwaves) {
      CompF32 v = lane < nwaves ? part[buf][j][lane] : OpComp::zero();
      v = wave_reduce_dpp<OpComp>(v);
      const PieceInfo& pi = info[buf][j];
      finish_piece<FIX>(a, pi.s, pi.sa, pi.sb, comp_to_double(v), lo, hi, g, chunk, &own_fix);
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
  if constexpr (FIX == kFixBarrier) {
    grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);  // also a workgroup barrier
    const int64_t os = own_fix;
    if (os >= 0 && wave == 0) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the pieces are loaded as published
      const int64_t o = offset_at(a.offsets, os) / chunk;
      const int64_t np = (offset_at(a.offsets, os + 1) - 1) / chunk - o + 1;
      const double v = combine_pieces(a, o, np);
      if (lane == 0) a.out[os] = v;
    }
  }
}

// One form runs per launch, so the forms share the workgroup's LDS, which
// is dynamic: the reduce-by-key form needs one RunLds per wavefront, so a
// small workgroup does not reserve the space of a 512-thread one.
union SegLds {
  WorkgroupLds wg;
  RunLds runs[kSegMaxWG / kWave];
};

size_t seg_lds_bytes(int wg) {
  return std::max(sizeof(WorkgroupLds), (size_t)(wg / kWave) * sizeof(RunLds));
}

// The form of a launch: forced, or from the batch's mean segment length
// (the same decision in every workgroup, and in the fix-up kernel).
template <int IPT>
__device__ __forceinline__ int seg_form(const SegArgs& a) {
  if (a.form != kSegAuto) return a.form;
  const int64_t E = offset_at(a.offsets, a.nseg);
  return E >= kWaveSliceMeanLen * a.nseg ? kSegWorkgroup
         : (IPT <= 4 && E < kRunsMeanLen * a.nseg) ? kSegWaveRuns
                                                 : kSegWavePieces;
}

template <int IPT, bool NT, int FIX>
__global__ __launch_bounds__(kSegMaxWG) void k_segmented(SegArgs a) {
  extern __shared__ __align__(16) unsigned char seg_lds[];
  SegLds& lds = *reinterpret_cast<SegLds*>(seg_lds);
  const int form = seg_form<IPT>(a);
  if (form == kSegWorkgroup) {
    seg_workgroup_slices<IPT, NT, FIX>(a, lds.wg);
  } else if (form == kSegWaveRuns) {
    if constexpr (IPT <= 4) seg_wave_runs<IPT, NT, FIX>(a, lds.runs);
  } else {
    seg_wave_slices<IPT, NT, FIX>(a);
  }
}

// Relaunch fix-up: wavefront w of this grid looks at carry slot w, which
// the slice kernel wrote for every w below its grid's wavefront count
// (slice w's slot in the wavefront forms; in the workgroup form, the slots
// past the grid say "none"); if a cut segment starts in slice w, it sums
// the segment's pieces in slice order (the same combine as the ticket and
// barrier fix-ups) and writes it.  The slot holds the segment and its
// piece count, so the fix-up reads no offsets.
constexpr int kFixupWG = 256;

__global__ __launch_bounds__(kFixupWG) void k_seg_fixup(SegArgs a) {
  const int64_t w = (int64_t)blockIdx.x * (kFixupWG / kWave) + threadIdx.x / kWave;
  if (w >= (int64_t)a.grid * (a.wg / kWave)) return;
  const SegCarry c = a.carry_out[w];
  if (c.seg < 0) return;
  const double v = combine_pieces(a, w, c.np);
  if (__lane_id() == 0) a.out[c.seg] = v;
}

namespace {

int ipt_index(int ipt) { return ipt == 1 ? 0 : ipt == 2 ? 1 : ipt == 4 ? 2 : ipt == 8 ? 3 : -1; }

struct SegTable {
  const void* k[3][2][4];  // SegFix, nontemporal, ipt index
  template <int F, bool NT>
  void fill() {
    k[F][NT][0] = reinterpret_cast<const void*>(&k_segmented<1, NT, F>);
    k[F][NT][1] = reinterpret_cast<const void*>(&k_segmented<2, NT, F>);
    k[F][NT][2] = reinterpret_cast<const void*>(&k_segmented<4, NT, F>);
    k[F][NT][3] = reinterpret_cast<const void*>(&k_segmented<8, NT, F>);
  }
  SegTable() {
    fill<kFixTicket, false>();
    fill<kFixTicket, true>();
    fill<kFixBarrier, false>();
    fill<kFixBarrier, true>();
    fill<kFixRelaunch, false>();
    fill<kFixRelaunch, true>();
  }
};

const SegTable& seg_table() {
  static const SegTable t;
  return t;
}

}  // namespace

// Default (measured on MI355X over uniform segment lengths and 10,000
// log-uniform ones): the atomic-ticket fix-up.  With the cut pieces
// published by device-scope atomic stores it is one kernel and 1 to 4 %
// faster than the relaunch fix-up's two (768-value segments, every slice
// boundary a cut: 188 against 196 us; with a release fence per cut piece
// it had taken 405 us).  Four 256-thread workgroups per CU: 16 wavefronts,
// the most the reduce-by-key form keeps resident, which beat two 512-thread
// workgroups by up to 8 % on 16-value segments and 2 to 4 % at 512 values
// and on the drawn batch; 4 loads of 16 bytes per thread per tile.
red_plan default_seg_plan(int64_t nseg, const DeviceInfo& dev) {
  (void)nseg;
  red_plan p;
  p.variant = RED_VARIANT_ATOMIC;
  p.wg = 256;
  p.ipt = 4;
  p.grid = 4 * dev.cus;
  p.flags = RED_FLAG_NONTEMPORAL;
  return p;
}

int seg_max_coresident(int ipt, int wg, const DeviceInfo& dev, int* n_wg) {
  const int ii = ipt_index(ipt);
  if (ii < 0) return set_error(RED_EINVAL, "bad ipt %d", ipt);
  int per_cu = 0;
  RED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, seg_table().k[kFixBarrier][0][ii], wg,
                                                         seg_lds_bytes(wg)));
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
  const int fix = barrier ? kFixBarrier : p.variant == RED_VARIANT_RELAUNCH ? kFixRelaunch : kFixTicket;
  if (!barrier && p.variant != RED_VARIANT_ATOMIC && p.variant != RED_VARIANT_RELAUNCH)
    return set_error(RED_EINVAL, "segmented: variant must be RELAUNCH, ATOMIC (ticket) or PERSISTENT (barrier)");
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
  a.bar_groups = ((p.flags & RED_FLAG_XCD) && xcd_tree_fits(dev.nxcc)) ? (kBarrierXcd | (unsigned)dev.nxcc)
                                                            : barrier_groups(grid);
  a.form = (p.flags & RED_FLAG_SEG_WORKGROUP) ? kSegWorkgroup
           : (p.flags & RED_FLAG_SEG_PIECES)  ? kSegWavePieces
           : (p.flags & RED_FLAG_SEG_RUNS)    ? kSegWaveRuns
                                              : kSegAuto;
  if (a.form == kSegWaveRuns && p.ipt > 4)
    return set_error(RED_EINVAL, "segmented: the reduce-by-key form takes at most 4 loads per thread");
  a.grid = grid;
  a.wg = p.wg;
  void* args[] = {&a};
  const bool nt = (p.flags & RED_FLAG_NONTEMPORAL) != 0;
  const bool coop = barrier && (p.flags & RED_FLAG_PLAIN_LAUNCH) == 0;
  const int slot = timer_begin(s);
  int rc = launch(seg_table().k[fix][nt ? 1 : 0][ii], grid, p.wg, args, s, coop, seg_lds_bytes(p.wg));
  if (rc == RED_OK && fix == kFixRelaunch) {
    // One wavefront per possible slice (the wavefront-slice count bounds the
    // workgroup-slice count).
    const int64_t waves = (int64_t)grid * (p.wg / kWave);
    const int fix_grid = (int)((waves + kFixupWG / kWave - 1) / (kFixupWG / kWave));
    rc = launch(reinterpret_cast<const void*>(&k_seg_fixup), fix_grid, kFixupWG, args, s, false);
  }
  timer_end(s, slot);
  return rc;
}

}  // namespace redsum
