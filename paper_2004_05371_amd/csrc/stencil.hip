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
//   * persistent: workgroup g owns the block [g m, (g+1) m) and holds it in
//                 LDS with a halo of K values on each side.  It runs K steps
//                 on the shrinking valid range (redundantly recomputing the
//                 halo, so neighbours need no exchange inside the K steps),
//                 then publishes its first and last K values (device-scope
//                 atomic stores), meets the other workgroups at a grid
//                 barrier that neither writes back nor invalidates an L2,
//                 and reads its neighbours' values into its halo (device-
//                 scope atomic loads).  One barrier per K steps;
//                 HBM is touched only at the start, at the end and for the
//                 2 K boundary values per workgroup and barrier.
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

// Per step each thread updates 4 consecutive window values per row of
// 4 x blockDim values (one 128-bit LDS read, two neighbour reads); the LDS
// window of a workgroup is at most 4 x kStencilRows x blockDim values.  The
// kernel is built for ROWS = 1, 2, 4, kStencilRows and launched with the
// smallest that holds the window, so a small window costs few instructions.
constexpr int kStencilRows = 8;

// Widest halo (steps per grid barrier) the library picks by itself.
constexpr int64_t kAutoHalo = 128;

// The window is padded to whole 4-value groups plus one group, so the last
// group's 128-bit read and its right neighbour stay inside the allocation.
__host__ __device__ inline int stencil_window_alloc(int len) { return ((len + 3) & ~3) + 4; }

template <int ROWS>
__global__ __launch_bounds__(1024) void k_jacobi_persistent(StencilArgs a) {
  unsigned gen = grid_barrier_gen(a.words);  // thread 0: the barrier generation of this launch
  extern __shared__ v4f win4[];  // 16-byte aligned window
  float* win = reinterpret_cast<float*>(win4);  // win[j] = element lo - k + j, j in [0, len)
  const int64_t n = a.n;
  const int k = a.k;
  const int64_t lo = (int64_t)blockIdx.x * a.m;
  const int64_t hi = std::min(lo + a.m, n);
  const int blen = (int)(hi - lo);
  const int len = blen + 2 * k;
  const int64_t base = lo - k;
  const int tid = threadIdx.x;
  const int bs = blockDim.x;
  const int qn = (len + 4 * bs - 1) / (4 * bs);  // rows of 4 bs values in the window

  for (int j = tid; j < len; j += bs) {
    const int64_t e = base + j;
    win[j] = (e >= 0 && e < n) ? a.u[e] : 0.0f;
  }
  __syncthreads();

  int sync = 0;
  for (int step = 0; step < a.steps;) {
    const int kk = std::min(k, a.steps - step);
    for (int s = 1; s <= kk; ++s) {
      // Window indices still valid after this step: elements
      // [lo - k + s, hi + k - s); the end points of the array never change.
      const int jlo = (int)(std::max<int64_t>(base + s, 1) - base);
      const int jhi = (int)(std::min<int64_t>(hi + k - s, n - 1) - base);
      // Group q of this thread: window values j0 .. j0+3, j0 = 4 (q bs + tid).
      // A value outside [jlo, jhi) keeps its old value, so whole groups are
      // written back (each group belongs to one thread).
      v4f nv[ROWS];
      bool any[ROWS];
#pragma unroll
      for (int q = 0; q < ROWS; ++q) {
        any[q] = false;
        if (q < qn) {  // workgroup-uniform: only the rows of the window
          const int j0 = 4 * (q * bs + tid);
          any[q] = j0 < jhi && j0 + 4 > jlo;
          if (any[q]) {
            const v4f c = win4[j0 >> 2];
            const float left = j0 > 0 ? win[j0 - 1] : 0.0f;  // value 0 is never updated (jlo >= 1)
            const float right = win[j0 + 4];
            v4f v;
            v.x = jacobi_point(left, c.x, c.y, a.r);
            v.y = jacobi_point(c.x, c.y, c.z, a.r);
            v.z = jacobi_point(c.y, c.z, c.w, a.r);
            v.w = jacobi_point(c.z, c.w, right, a.r);
            if (j0 < jlo || j0 + 4 > jhi) {  // a group at an edge of the valid range
              v.x = (j0 >= jlo && j0 < jhi) ? v.x : c.x;
              v.y = (j0 + 1 >= jlo && j0 + 1 < jhi) ? v.y : c.y;
              v.z = (j0 + 2 >= jlo && j0 + 2 < jhi) ? v.z : c.z;
              v.w = (j0 + 3 >= jlo && j0 + 3 < jhi) ? v.w : c.w;
            }
            nv[q] = v;
          }
        }
      }
      __syncthreads();  // every read of the old values precedes the writes
#pragma unroll
      for (int q = 0; q < ROWS; ++q)
        if (q < qn && any[q]) win4[(4 * (q * bs + tid)) >> 2] = nv[q];
      __syncthreads();
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
      for (int j = tid; j < w; j += bs) {
        publish(&pub[lo + j], win[k + j]);
        publish(&pub[hi - 1 - j], win[k + blen - 1 - j]);
      }
      grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);
      for (int j = tid; j < k; j += bs) {
        const int64_t el = lo - k + j;  // left halo: the left neighbour's last k values
        if (el >= 0) win[j] = load_published(&pub[el]);
        const int64_t er = hi + j;      // right halo: the right neighbour's first k values
        if (er < n) win[k + blen + j] = load_published(&pub[er]);
      }
      __syncthreads();
      ++sync;
    }
  }
  // Neighbours read u for their initial halos and, at odd exchanges, as the
  // publication buffer: the block is written back only once every
  // workgroup is past its last read of u (each workgroup's loads complete
  // before it arrives; no data crosses this barrier).
  grid_barrier_published(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen);
  for (int j = tid; j < blen; j += bs) a.u[lo + j] = win[k + j];
}

namespace {

const void* persistent_kernel(int rows) {
  switch (rows) {
    case 1: return reinterpret_cast<const void*>(&k_jacobi_persistent<1>);
    case 2: return reinterpret_cast<const void*>(&k_jacobi_persistent<2>);
    case 4: return reinterpret_cast<const void*>(&k_jacobi_persistent<4>);
    default: return reinterpret_cast<const void*>(&k_jacobi_persistent<kStencilRows>);
  }
}

int stencil_coresident(int wg, size_t lds_bytes, const DeviceInfo& dev, int* n_wg) {
  int per_cu = 0;
  RED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel(kStencilRows), wg, lds_bytes));
  *n_wg = per_cu * dev.cus;
  if (*n_wg < 1) return set_error(RED_EINVAL, "persistent stencil: a %d-thread workgroup with %zu bytes of LDS "
                                              "cannot be resident", wg, lds_bytes);
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
  // LDS window: the 64 KB a workgroup gets without opting in to more, less
  // a margin for the barrier's static LDS.
  auto window_floats = [&](int threads) {
    return std::min<int64_t>((std::min<int64_t>(dev.lds_per_wg, 65536) - 256) / 4 - 8,
                             (int64_t)4 * kStencilRows * threads);
  };
  // Threads per workgroup when the caller leaves them open: 16 wavefronts
  // per CU either way, as one 1024-thread workgroup when one window per CU
  // holds the array with at least 4 values per thread (measured on MI355X:
  // 0.87 against 1.11 us per step at 1 M values, k = 32), else 512-thread
  // workgroups, two per CU when the array needs more windows than CUs.
  int wg = p.wg;
  if (wg == 0) {
    const int64_t cap1024 = std::max<int64_t>(1, window_floats(1024) - 2 * (int64_t)k_req);
    wg = (variant != RED_VARIANT_RELAUNCH && n >= (int64_t)4 * 1024 * dev.cus &&
          (n + cap1024 - 1) / cap1024 <= dev.cus)
             ? 1024
             : 512;
  }
  const int64_t lds_floats = window_floats(wg);

  // Persistent geometry: one workgroup per CU unless the array needs more
  // LDS windows, never more than are co-resident with the largest window,
  // at least 64 values per workgroup.
  int grid = 0;
  int64_t m = 0;
  int k = 0;
  size_t lds_bytes = 0;
  if (variant != RED_VARIANT_RELAUNCH) {
    int g_max = 0;
    int rc = stencil_coresident(wg, (size_t)stencil_window_alloc((int)lds_floats) * 4, dev, &g_max);
    if (rc) return rc;
    const int64_t cap = std::max<int64_t>(1, lds_floats - 2 * (int64_t)k_req);  // block values per window
    // More windows than CUs: a whole number of workgroups per CU, so that no
    // CU holds one block more than the others (4 M values need 259 windows
    // of 64 KB: 512 of half the size keep every CU equally loaded).
    const int64_t need = (n + cap - 1) / cap;
    int64_t g = p.grid > 0 ? p.grid
                           : need <= dev.cus ? (int64_t)dev.cus : (need + dev.cus - 1) / dev.cus * dev.cus;
    g = std::max<int64_t>(1, std::min<int64_t>({g, (int64_t)g_max, (n + 63) / 64}));
    m = (n + g - 1) / g;
    grid = (int)((n + m - 1) / m);
    // Halo width: the caller's steps per barrier, else the widest halo up to
    // kAutoHalo that the window holds beside the block.  The halo values are
    // recomputed redundantly, so a wider one trades a little arithmetic for
    // fewer grid barriers (measured on MI355X, 512 steps: 1.95 us per step
    // at k = 32 and 1.72 at k = 128 on 4 M values, 0.86 and 0.66 on 1 M).
    k = steps_per_sync > 0 ? (int)std::min<int64_t>(k_req, m)
                           : (int)std::max<int64_t>(1, std::min<int64_t>({kAutoHalo, m, (lds_floats - m) / 2}));
    const int64_t len = m + 2 * (int64_t)k;
    if (len > lds_floats) {
      if (variant == RED_VARIANT_PERSISTENT)
        return set_error(RED_EINVAL,
                         "persistent stencil: %lld values per workgroup with halos exceed the %lld values of an "
                         "LDS window at this workgroup size (%d co-resident workgroups hold about %lld values)",
                         (long long)len, (long long)lds_floats, g_max, (long long)cap * g_max);
      variant = RED_VARIANT_RELAUNCH;  // AUTO: the array does not fit on chip
    } else {
      variant = RED_VARIANT_PERSISTENT;
      lds_bytes = (size_t)stencil_window_alloc((int)len) * 4;
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
  int rows = 1;
  while (rows < kStencilRows && (int64_t)4 * rows * wg < m + 2 * (int64_t)k) rows *= 2;
  int rc = launch(persistent_kernel(rows), grid, wg, args, s, coop, lds_bytes);
  timer_end(s, slot);
  return rc;
}

}  // namespace redsum
