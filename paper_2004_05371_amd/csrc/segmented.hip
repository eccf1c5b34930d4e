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
//     offsets and walks the segments of its slice in order, reducing each
//     piece with the whole workgroup (16-byte loads, fp32 TwoSum-compensated
//     accumulators, wavefront + LDS combine);
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

// Per-thread compensated sum of x[a, b) with the whole workgroup: scalar
// head up to a 16-byte boundary, then tiles of blockDim.x * IPT vectors,
// then the scalar tail.
template <int IPT, bool NT>
__device__ __forceinline__ CompF32 thread_sum_range(const float* x, int64_t a, int64_t b) {
  using M = ModeF32Comp;
  const uintptr_t addr = reinterpret_cast<uintptr_t>(x + a);
  const int64_t len = b - a;
  const int64_t head = std::min<int64_t>((int64_t)(((16 - (addr & 15)) & 15) >> 2), len);
  const int64_t nvec = (len - head) >> 2;
  const int64_t tail = len - head - (nvec << 2);
  const v4f* xv = reinterpret_cast<const v4f*>(x + a + head);
  const int64_t bs = blockDim.x;
  const int64_t tile = bs * IPT;
  const int64_t ntiles = nvec / tile;
  const int tid = threadIdx.x;

  CompF32 acc[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) acc[u] = M::zero();
  for (int64_t t = 0; t < ntiles; ++t) {
    const v4f* p = xv + t * tile + tid;
    v4f v[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) v[u] = load_vec<NT>(p + u * bs);
    __builtin_amdgcn_sched_barrier(0);  // all IPT loads in flight before use
#pragma unroll
    for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], v[u]);
  }
  for (int64_t i = ntiles * tile + tid; i < nvec; i += bs) M::add_vec(acc[0], load_vec<NT>(xv + i));
  if (tid < head)
    M::add_elem(acc[0], x[a + tid]);
  else if (tid < head + tail)
    M::add_elem(acc[0], x[a + head + (nvec << 2) + (tid - head)]);
#pragma unroll
  for (int u = 1; u < IPT; ++u) acc[0] = OpComp::add(acc[0], acc[u]);
  return acc[0];
}

// Sum the pieces of segment s (owning slice o, np pieces) in slice order.
__device__ __forceinline__ double combine_pieces(const SegArgs& a, int64_t o, int64_t np) {
  double v = a.carry_out[o].val;
  for (int64_t k = o + 1; k < o + np; ++k) v += a.carry_in[k].val;
  return v;
}

template <int IPT, bool NT, bool BARRIER>
__global__ __launch_bounds__(1024) void k_segmented(SegArgs a) {
  __shared__ CompF32 lds[kMaxWavesPerWG];
  const int64_t nseg = a.nseg;
  const int64_t E = a.offsets[nseg];
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
    if (a.offsets[mid] >= lo)
      R = mid;
    else
      L = mid + 1;
  }
  // Segment L-1 crosses lo if it ends after lo.
  int64_t s = (L > 0 && a.offsets[L] > lo) ? L - 1 : L;

  int64_t own_seg = -1;  // segment that starts in this slice and continues
  for (; s < nseg; ++s) {
    const int64_t sa = a.offsets[s];
    const int64_t sb = a.offsets[s + 1];
    if (sa >= hi && !(end_wg && sa == E)) break;
    if (sa == sb) {
      if (threadIdx.x == 0) a.out[s] = 0.0;
      continue;
    }
    const int64_t pa = std::max(sa, lo);
    const int64_t pb = std::min(sb, hi);
    CompF32 acc = thread_sum_range<IPT, NT>(a.x, pa, pb);
    CompF32 tot = block_reduce<OpComp>(acc, lds);
    if (threadIdx.x == 0) {
      const double v = comp_to_double(tot);
      if (sa >= lo && sb <= hi) {
        a.out[s] = v;
      } else {
        const SegCarry c{s, v};
        if (sa < lo)
          a.carry_in[g] = c;
        else
          a.carry_out[g] = c;
        const int64_t o = sa / chunk;
        const int64_t np = (sb - 1) / chunk - o + 1;
        if constexpr (!BARRIER) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          const unsigned tk =
              __hip_atomic_fetch_add(&a.tickets[o], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (tk == (unsigned)(np - 1)) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            a.out[s] = combine_pieces(a, o, np);
            __hip_atomic_store(&a.tickets[o], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        } else {
          if (sa >= lo) own_seg = s;
        }
      }
    }
    __syncthreads();  // lds is reused by the next piece
  }
  if constexpr (BARRIER) {
    grid_barrier(a.words, gridDim.x, a.bar_groups, a.spin_limit);
    if (threadIdx.x == 0 && own_seg >= 0) {
      const int64_t sa = a.offsets[own_seg];
      const int64_t sb = a.offsets[own_seg + 1];
      const int64_t o = sa / chunk;
      const int64_t np = (sb - 1) / chunk - o + 1;
      a.out[own_seg] = combine_pieces(a, o, np);
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

red_plan default_seg_plan(int64_t nseg, const DeviceInfo& dev) {
  (void)nseg;
  red_plan p;
  p.variant = RED_VARIANT_ATOMIC;
  p.wg = 256;
  p.ipt = 8;
  p.grid = 3 * dev.cus;
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
