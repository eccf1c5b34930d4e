// Iterative 1D Jacobi stencil: the time loop inside one persistent kernel
// versus one kernel launch per step (gfx950).
//
// Section VII-B of Zhang et al. points out a benefit of grid barriers that
// the reduction does not show: a persistent kernel that holds the time loop
// of an iterative stencil keeps its data in on-chip memory across the
// barriers, where one launch per step (the implicit barrier) must stream
// the whole array through HBM or the caches every step.
//
// The step is u'[i] = u[i] + r ((u[i-1] + u[i+1]) - 2 u[i]) for
// 1 <= i <= n-2, with u[0] and u[n-1] fixed, each operation one binary32
// operation in that order (no contraction), so both forms reproduce the
// step-by-step definition bit for bit.
//
//   * relaunch:   k_jacobi_step per step, ping-pong between u and the
//                 caller's scratch array;
//   * persistent: workgroup g owns the block [g m, (g+1) m) and holds it,
//                 with a halo of K values on each side, in its threads'
//                 registers.  It runs K steps on the shrinking valid range
//                 (redundantly recomputing the halo, so neighbours need no
//                 exchange inside the K steps), then publishes its first and
//                 last K values (device-scope atomic stores), meets the other
//                 workgroups at a grid barrier that neither writes back nor
//                 invalidates an L2, and reads its neighbours' values into
//                 its halo (device-scope atomic loads).  One barrier per K
//                 steps; HBM is touched only at the start, at the end and for
//                 the 2 K boundary values per workgroup and barrier.
#include <algorithm>

#include "device_prims.h"
#include "internal.h"

namespace redsum {

// One step at an interior point, in the method's operation order.
__device__ __forceinline__ float jacobi_point(float left, float centre, float right, float r) {
#pragma clang fp contract(off)
  const float neighbours = left + right;
  const float twice = 2.0f * centre;
  return centre + r * (neighbours - twice);
}

__global__ __launch_bounds__(1024) void k_jacobi_step(const float* __restrict__ u, float* __restrict__ v, int64_t n,
                                                      float r) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float c = u[i];
    v[i] = (i == 0 || i == n - 1) ? c : jacobi_point(u[i - 1], c, u[i + 1], r);
  }
}

__global__ __launch_bounds__(1024) void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

struct StencilArgs {
  float* u;        // values, in and out
  float* scratch;  // n values: boundary publication, alternating with u
  int64_t n;
  int64_t m;       // block length per workgroup
  int steps;
  int k;           // steps per grid barrier = halo width, 1 <= k <= m
  float r;
  BarrierWords* words;
  unsigned spin_limit;
  unsigned bar_groups;
};

// The window of a workgroup (its block and k-wide halos, at most
// kWindowMax values) is held in registers: thread t owns the VPT
// consecutive window values from VPT t on.  A step reads the two values
// beside a thread's run from its neighbours, through LDS: each thread
// stores its first and last value to one of two edge buffers (alternating
// by step), meets the others at the step's only workgroup barrier, and
// reads the neighbours' edges.  A buffer is written again two steps later,
// after the next barrier, which every thread reaches after its reads.  The
// kernel is built for VPT = 2, 4, 8, 16 and 32.
constexpr int kWindowMax = 16384;

// Widest halo (steps per grid barrier) the library picks by itself.
constexpr int64_t kAutoHalo = 128;

template <int VPT>
__global__ __launch_bounds__(1024) void k_jacobi_persistent(StencilArgs a) {
  static_assert(VPT >= 2, "a run has a first and a last value");
  unsigned gen = grid_barrier_gen(a.words);  // thread 0: the barrier generation of this launch
  extern __shared__ float edge[];            // [2 buffers][first, last][blockDim.x]
  const int64_t n = a.n;
  const int k = a.k;
  const int64_t lo = (int64_t)blockIdx.x * a.m;
  const int64_t hi = std::min(lo + a.m, n);
  const int blen = (int)(hi - lo);
  const int len = blen + 2 * k;
  const int64_t base = lo - k;  // window value j is element base + j
  const int tid = threadIdx.x;
  const int bs = blockDim.x;
  const int j0 = VPT * tid;     // this thread's window values j0 .. j0 + VPT - 1

  float x[VPT];
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int64_t e = base + j0 + i;
    x[i] = (j0 + i < len && e >= 0 && e < n) ? a.u[e] : 0.0f;
  }

  // Window positions of the array's end points, which never change (-1 or
  // len when the window does not hold them).
  const int jz = (int)std::max<int64_t>(std::min<int64_t>(-base, len), -1);
  const int jn = (int)std::max<int64_t>(std::min<int64_t>(n - 1 - base, len), -1);
  const bool holds_end = (jz >= j0 && jz < j0 + VPT) || (jn >= j0 && jn < j0 + VPT);

  int sync = 0, buf = 0;
  for (int step = 0; step < a.steps;) {
    const int kk = std::min(k, a.steps - step);
    for (int s = 1; s <= kk; ++s) {
      // After step s only the window values of the elements
      // [lo - k + s, hi + k - s) are valid: the range shrinks by one value
      // on each side per step, so no valid value depends on one outside it.
      // The values outside (the halo being used up, and positions past the
      // array's ends) are updated too and never read for a valid one; the
      // halo is reloaded at the next exchange.  Only the array's end points
      // keep their value.
      float* eb = edge + 2 * bs * buf;
      eb[tid] = x[0];
      eb[bs + tid] = x[VPT - 1];
      __syncthreads();
      // Window value j0 - 1 is the left neighbour's last, j0 + VPT the right
      // neighbour's first (thread 0 and the last thread read a value that
      // only feeds positions outside the valid range).
      const float left = tid > 0 ? eb[bs + tid - 1] : 0.0f;
      const float right = tid + 1 < bs ? eb[tid + 1] : 0.0f;
      float y[VPT];
      y[0] = jacobi_point(left, x[0], x[1], a.r);
#pragma unroll
      for (int i = 1; i < VPT - 1; ++i) y[i] = jacobi_point(x[i - 1], x[i], x[i + 1], a.r);
      y[VPT - 1] = jacobi_point(x[VPT - 2], x[VPT - 1], right, a.r);
      if (!holds_end) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) x[i] = y[i];
      } else {  // the run that holds element 0 or n - 1
#pragma unroll
        for (int i = 0; i < VPT; ++i) x[i] = (j0 + i == jz || j0 + i == jn) ? x[i] : y[i];
      }
      buf ^= 1;
    }
    step += kk;
    if (step < a.steps) {
      // Publish the first and last k values of the block (time `step`) to
      // the buffer of this barrier's parity, meet, read the neighbours'.
      // The first publication goes to scratch: u is still being read for
      // the initial halos.  The edges cross the barrier as device-scope
      // atomic stores and loads, so the barrier neither writes back nor
      // invalidates an L2.
      float* pub = (sync & 1) ? a.u : a.scratch;
      const int w = std::min(k, blen);
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int j = j0 + i;
        if ((j >= k && j < k + w) || (j >= k + blen - w && j < k + blen)) publish(&pub[base + j], x[i]);
      }
      grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int j = j0 + i;
        const int64_t e = base + j;
        // left halo: the left neighbour's last k values; right halo: the
        // right neighbour's first k values
        if ((j < k && e >= 0) || (j >= k + blen && j < len && e < n)) x[i] = load_published(&pub[e]);
      }
      ++sync;
    }
  }
  // Neighbours read u for their initial halos and, at odd exchanges, as the
  // publication buffer: the block is written back only once every
  // workgroup is past its last read of u (each workgroup's loads complete
  // before it arrives; no data crosses this barrier).
  grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int j = j0 + i;
    if (j >= k && j < k + blen) a.u[base + j] = x[i];
  }
}

namespace {

const void* persistent_kernel(int vpt) {
  switch (vpt) {
    case 2: return reinterpret_cast<const void*>(&k_jacobi_persistent<2>);
    case 4: return reinterpret_cast<const void*>(&k_jacobi_persistent<4>);
    case 8: return reinterpret_cast<const void*>(&k_jacobi_persistent<8>);
    case 16: return reinterpret_cast<const void*>(&k_jacobi_persistent<16>);
    default: return reinterpret_cast<const void*>(&k_jacobi_persistent<32>);
  }
}

// LDS of the two edge buffers of a workgroup of wg threads.
size_t edge_bytes(int wg) { return (size_t)4 * wg * sizeof(float); }

// Workgroups of the kernel for `vpt` values per thread that all CUs hold at
// once with wg threads each.
int stencil_coresident(int vpt, int wg, const DeviceInfo& dev, int* n_wg) {
  int per_cu = 0;
  RED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel(vpt), wg, edge_bytes(wg)));
  *n_wg = per_cu * dev.cus;
  return RED_OK;
}

}  // namespace

int stencil_launch(float* u, float* scratch, int64_t n, int steps, float r, int steps_per_sync, const red_plan& p,
                   Workspace* ws, hipStream_t s, const DeviceInfo& dev) {
  if (n < 3 || steps == 0) return RED_OK;
  int variant = p.variant;
  // The geometry (workgroups, block length) is set for the caller's halo,
  // or for a halo of 8 when the library chooses it.
  const int k_req = steps_per_sync > 0 ? steps_per_sync : 8;
  // Window capacity: kWindowMax values, or 32 per thread of the caller's
  // workgroup size.
  const int64_t wmax = p.wg > 0 ? std::min<int64_t>(kWindowMax, (int64_t)32 * p.wg) : kWindowMax;

  // Persistent geometry: one workgroup per CU unless the array needs more
  // windows, then a whole number of workgroups per CU, so that no CU holds
  // one block more than the others (4 M values in windows of 16 K would
  // need 259: 512 of half the size keep every CU equally loaded); at least
  // 64 values per workgroup.
  int grid = 0, wg = p.wg > 0 ? p.wg : 512, vpt = 0;
  int64_t m = 0;
  int k = 0;
  if (variant != RED_VARIANT_RELAUNCH) {
    const int64_t cap = std::max<int64_t>(1, wmax - 2 * (int64_t)k_req);  // block values per window
    const int64_t need = (n + cap - 1) / cap;
    int64_t g = p.grid > 0 ? p.grid
                           : need <= dev.cus ? (int64_t)dev.cus : (need + dev.cus - 1) / dev.cus * dev.cus;
    g = std::max<int64_t>(1, std::min<int64_t>(g, (n + 63) / 64));
    m = (n + g - 1) / g;
    grid = (int)((n + m - 1) / m);
    // Halo width: the caller's steps per barrier, else the widest halo up to
    // kAutoHalo that the window holds beside the block.  The halo values are
    // recomputed redundantly, so a wider one trades a little arithmetic for
    // fewer grid barriers.
    k = steps_per_sync > 0 ? (int)std::min<int64_t>(k_req, m)
                           : (int)std::max<int64_t>(1, std::min<int64_t>({kAutoHalo, m, (wmax - m) / 2}));
    const int64_t len = m + 2 * (int64_t)k;
    // Values per thread and threads per workgroup: the caller's workgroup
    // size with the fewest values per thread that cover the window; else
    // the fewest values per thread (2 to 32) whose workgroup, rounded to
    // whole wavefronts, stays within 1024 threads and is co-resident with
    // the grid (small windows spread over more wavefronts: 0.28 against
    // 0.37 us per step with 8 values per thread at 64 K values).
    int g_max = 0;
    if (len <= wmax) {
      if (p.wg > 0) {
        for (int v = 4; v <= 32 && !vpt; v *= 2)
          if ((int64_t)v * wg >= len) vpt = v;
        int rc = stencil_coresident(vpt, wg, dev, &g_max);
        if (rc) return rc;
      } else {
        for (int v = 2; v <= 32 && !vpt; v *= 2) {
          const int t = (int)((len + v - 1) / v + kWave - 1) / kWave * kWave;
          if (t > 1024) continue;
          int gm = 0;
          int rc = stencil_coresident(v, t, dev, &gm);
          if (rc) return rc;
          if (gm >= grid) {
            vpt = v;
            wg = t;
            g_max = gm;
          }
        }
      }
    }
    if (!vpt || g_max < grid) {
      if (variant == RED_VARIANT_PERSISTENT)
        return set_error(RED_EINVAL,
                         "persistent stencil: %d workgroups of %lld values with halos do not fit the co-resident "
                         "workgroups' registers (at most %lld values per workgroup; %d co-resident)",
                         grid, (long long)len, (long long)wmax, g_max);
      variant = RED_VARIANT_RELAUNCH;  // AUTO: the array does not fit on chip
    } else {
      variant = RED_VARIANT_PERSISTENT;
    }
  }

  if (variant == RED_VARIANT_RELAUNCH) {
    int gridr = p.grid > 0 ? p.grid : 4 * dev.cus;
    gridr = (int)std::max<int64_t>(1, std::min<int64_t>(gridr, (n + wg - 1) / wg));
    float* src = u;
    float* dst = scratch;
    for (int t = 0; t < steps; ++t) {
      void* args[] = {&src, &dst, &n, &r};
      int rc = launch(reinterpret_cast<const void*>(&k_jacobi_step), gridr, wg, args, s, false);
      if (rc) return rc;
      std::swap(src, dst);
    }
    if (src != u) {
      void* args[] = {&src, &u, &n};
      return launch(reinterpret_cast<const void*>(&k_copy_f32), gridr, wg, args, s, false);
    }
    return RED_OK;
  }

  StencilArgs a;
  a.u = u;
  a.scratch = scratch;
  a.n = n;
  a.m = m;
  a.steps = steps;
  a.k = k;
  a.r = r;
  a.words = ws->words;
  a.spin_limit = watchdog_spins();
  a.bar_groups = ((p.flags & RED_FLAG_XCD) && xcd_tree_fits(dev.nxcc)) ? (kBarrierXcd | (unsigned)dev.nxcc)
                                                            : barrier_groups(grid);
  void* args[] = {&a};
  const bool coop = (p.flags & RED_FLAG_PLAIN_LAUNCH) == 0;
  const int slot = timer_begin(s);
  int rc = launch(persistent_kernel(vpt), grid, wg, args, s, coop, edge_bytes(wg));
  timer_end(s, slot);
  return rc;
}

}  // namespace redsum
