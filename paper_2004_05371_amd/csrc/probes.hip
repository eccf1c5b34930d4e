// Synchronization latency probes (Sections IV, V and IX of Zhang et al.).
//
// * wavefront level  -- a dependent chain of cross-lane operations (DPP,
//   ds_swizzle, ds_bpermute wavefront combines, or one DPP add step), timed
//   in-kernel with the shader clock (the in-SM clock method of Section
//   IX-C) and by the host differential of Eq. 7 between chains of r1 and r2
//   operations;
// * workgroup level  -- a chain of s_barrier (__syncthreads) in n_wg
//   workgroups;
// * grid level       -- a chain of software grid barriers in one cooperative
//   kernel;
// * implicit barrier -- the launch overhead of a kernel boundary by kernel
//   fusion (Eq. 6) with kernels that wait a fixed wall-clock time per unit
//   (the paper's nanosleep null kernel, Section IV), and the total latency
//   of a null kernel by the three-timestamp formula of Section IV.
// Uncertainties follow Eq. 8.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "device_prims.h"
#include "internal.h"

namespace redsum {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Value types of the wavefront probe: wrapping integer adds (so a chain of
// doubling steps is defined), the Ops of the reduction otherwise.
struct OpU32 {
  using T = unsigned;
  __device__ static T zero() { return 0u; }
  __device__ static T add(T a, T b) { return a + b; }
};
struct OpU64 {
  using T = unsigned long long;
  __device__ static T zero() { return 0ull; }
  __device__ static T add(T a, T b) { return a + b; }
};

// Keeps a chain of combines dependent and its values bounded: the next
// input of lane l is the combined value scaled down plus a lane term.
__device__ __forceinline__ float chain_mix(float r, int lane) { return r * 0.0078125f + (float)(lane & 7) * 0.125f; }
__device__ __forceinline__ double chain_mix(double r, int lane) { return r * 0.0078125 + (double)(lane & 7) * 0.125; }
__device__ __forceinline__ unsigned chain_mix(unsigned r, int lane) { return (r >> 6) + (unsigned)(lane & 7); }
__device__ __forceinline__ unsigned long long chain_mix(unsigned long long r, int lane) {
  return (r >> 6) + (unsigned long long)(lane & 7);
}
__device__ __forceinline__ CompF32 chain_mix(CompF32 r, int lane) {
  return CompF32{r.s * 0.0078125f + (float)(lane & 7) * 0.125f, r.c * 0.0078125f};
}

template <int OP, class Op>
__global__ __launch_bounds__(1024) void k_wave_chain(int r, unsigned* sink, long long* cycles) {
  using T = typename Op::T;
  const int lane = __lane_id();
  T v = chain_mix(Op::zero(), lane);
  __builtin_amdgcn_sched_barrier(0);
  const long long t0 = __builtin_amdgcn_s_memtime();
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll 8
  for (int i = 0; i < r; ++i) {
    if constexpr (OP == RED_WAVE_DPP)
      v = chain_mix(wave_reduce_dpp<Op>(v), lane);
    else if constexpr (OP == RED_WAVE_SWIZZLE)
      v = chain_mix(wave_reduce_swizzle<Op>(v), lane);
    else if constexpr (OP == RED_WAVE_BPERMUTE)
      v = chain_mix(wave_reduce_bpermute<Op>(v), lane);
    else
      v = Op::add(v, dpp_move<kRowShr1, 0xF, 0xF>(v));
  }
  __builtin_amdgcn_sched_barrier(0);
  const long long t1 = __builtin_amdgcn_s_memtime();
  __builtin_amdgcn_sched_barrier(0);
  if (threadIdx.x == 0) cycles[blockIdx.x] = t1 - t0;
  unsigned w0;
  __builtin_memcpy(&w0, &v, 4);
  // Keeps the chain live: a value the compiler cannot bound (it would
  // remove a chain whose result provably misses a constant).
  if (w0 == (unsigned)r * 0x9E3779B9u + 0x7F7F1234u) sink[threadIdx.x] = w0;
}

// One wavefront combine of `op` on the 64 values in[0..64) (one per lane);
// lane l writes the value the combine returns to it to out[l].  The one
// DPP step returns v[l] + v[l - 1] inside each 16-lane row (0 from outside
// the row).
template <int OP, class Op>
__global__ __launch_bounds__(64) void k_wave_once(const typename Op::T* in, typename Op::T* out) {
  using T = typename Op::T;
  const int lane = __lane_id();
  T v = in[lane];
  if constexpr (OP == RED_WAVE_DPP)
    v = wave_reduce_dpp<Op>(v);
  else if constexpr (OP == RED_WAVE_SWIZZLE)
    v = wave_reduce_swizzle<Op>(v);
  else if constexpr (OP == RED_WAVE_BPERMUTE)
    v = wave_reduce_bpermute<Op>(v);
  else
    v = Op::add(v, dpp_move<kRowShr1, 0xF, 0xF>(v));
  out[lane] = v;
}

__global__ __launch_bounds__(1024) void k_block_chain(int r, long long* cycles) {
  __builtin_amdgcn_sched_barrier(0);
  const long long t0 = __builtin_amdgcn_s_memtime();
  __builtin_amdgcn_sched_barrier(0);
  for (int i = 0; i < r; ++i) __syncthreads();
  __builtin_amdgcn_sched_barrier(0);
  const long long t1 = __builtin_amdgcn_s_memtime();
  if (threadIdx.x == 0) cycles[blockIdx.x] = t1 - t0;
}

// Block-barrier throughput under load: every workgroup runs barriers
// (s_barrier) back to back for `window` ticks of the 100 MHz wall clock and
// records how many it completed and over how many ticks.  Thread 0 reads
// the clock after every 64 barriers and broadcasts the decision through
// LDS behind one more barrier, so every thread runs the same count.
__global__ __launch_bounds__(1024) void k_block_tput(long long window, long long* counts, long long* ticks) {
  __shared__ int stop;
  long long t0 = 0;
  if (threadIdx.x == 0) {
    stop = 0;
    t0 = __builtin_amdgcn_s_memrealtime();
  }
  __syncthreads();
  long long n = 0;
  for (;;) {
    for (int k = 0; k < 64; ++k) __syncthreads();
    if (threadIdx.x == 0) stop = __builtin_amdgcn_s_memrealtime() - t0 >= window;
    __syncthreads();
    n += 65;
    if (stop) break;
  }
  if (threadIdx.x == 0) {
    counts[blockIdx.x] = n;
    ticks[blockIdx.x] = __builtin_amdgcn_s_memrealtime() - t0;
  }
}

// r grid barriers back to back; PUB: the barrier for data published by
// device-scope atomics (no L2 write-back at arrival, no invalidation after).
template <bool PUB>
__global__ __launch_bounds__(1024) void k_grid_chain(int r, BarrierWords* w, unsigned groups,
                                                    unsigned spin_limit, long long* stamps) {
  unsigned gen = grid_barrier_gen(w);
  __syncthreads();
  const long long t0 = __builtin_amdgcn_s_memrealtime();
  for (int i = 0; i < r; ++i) {
    if constexpr (PUB)
      grid_barrier_published(w, gridDim.x, groups, spin_limit, gen);
    else
      grid_barrier(w, gridDim.x, groups, spin_limit, gen);
  }
  const long long t1 = __builtin_amdgcn_s_memrealtime();
  if (blockIdx.x == 0 && threadIdx.x == 0) stamps[0] = t1 - t0;
}

// Waits `ticks` of the 100 MHz wall clock (a "wait unit" kernel; the
// paper's nanosleep kernel).  The loop ends because the clock advances.
__global__ __launch_bounds__(1024) void k_spin(long long ticks) {
  if (ticks <= 0) return;
  const long long t0 = __builtin_amdgcn_s_memrealtime();
  while (__builtin_amdgcn_s_memrealtime() - t0 < ticks) __builtin_amdgcn_s_sleep(2);
}

__global__ __launch_bounds__(1024) void k_grid_order(BarrierWords* w, unsigned groups, unsigned spin_limit,
                                                    long long* before, long long* after) {
  unsigned gen = grid_barrier_gen(w);
  __syncthreads();
  if (threadIdx.x == 0) before[blockIdx.x] = __builtin_amdgcn_s_memrealtime();
  grid_barrier(w, gridDim.x, groups, spin_limit, gen);
  if (threadIdx.x == 0) after[blockIdx.x] = __builtin_amdgcn_s_memrealtime();
}

// Visibility across the grid barrier: in round r thread 0 of workgroup g
// stores r * G + g to data[g] with an ordinary store; after the barrier
// every thread reads its share of data[0 .. G) with ordinary loads (the
// same addresses every round, so a stale line in either cache level would
// show) and counts the slots that do not hold this round's value; a second
// barrier keeps round r + 1's stores after every read of round r.  PUB:
// device-scope atomic stores and loads around the barrier for published
// data.
template <bool PUB>
__global__ __launch_bounds__(1024) void k_grid_visibility(BarrierWords* w, unsigned groups, unsigned spin_limit,
                                                         long long* data, unsigned long long* errors,
                                                         int rounds) {
  const unsigned G = gridDim.x;
  unsigned long long bad = 0;
  unsigned gen = grid_barrier_gen(w);
  auto barrier = [&]() {
    if constexpr (PUB)
      return grid_barrier_published(w, G, groups, spin_limit, gen);
    else
      return grid_barrier(w, G, groups, spin_limit, gen);
  };
  for (int r = 0; r < rounds; ++r) {
    const long long mine = (long long)r * G + blockIdx.x;
    if (threadIdx.x == 0) {
      if constexpr (PUB)
        publish(&data[blockIdx.x], mine);
      else
        data[blockIdx.x] = mine;
    }
    if (!barrier()) break;
    for (unsigned i = threadIdx.x; i < G; i += blockDim.x) {
      const long long v = PUB ? load_published(&data[i]) : data[i];
      bad += v != (long long)r * G + i;
    }
    if (!barrier()) break;
  }
  if (bad) atomicAdd(errors, bad);
}

// Workgroup `skip` never arrives; the others leave through the watchdog.
__global__ __launch_bounds__(1024) void k_watchdog(BarrierWords* w, int skip, unsigned groups,
                                                  unsigned spin_limit) {
  if ((int)blockIdx.x == skip) return;
  unsigned gen = grid_barrier_gen(w);
  grid_barrier(w, gridDim.x, groups, spin_limit, gen);
}

// XCD of every workgroup (thread 0 records it).
__global__ __launch_bounds__(1024) void k_xcc_map(int* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = (int)xcc_id();
}

__global__ void k_reset_words(BarrierWords* w) {
  if (threadIdx.x == 0) {
    *tally_word(w->count) = 0;
    *tally_word(w->gen) = 0;  // generation and fall-back request
    *tally_word(w->ticket) = 0;
    w->err.v = 0;
    w->fb.v = 0;
  }
  for (int i = threadIdx.x; i < kMaxBarrierGroups; i += blockDim.x) *tally_word(w->group[i]) = 0;
  for (int i = threadIdx.x; i < kMaxTreeClasses; i += blockDim.x) *tally_word(w->cls[i]) = 0;
  for (int i = threadIdx.x; i < kMaxTreeNodes; i += blockDim.x) *tally_word(w->node[i]) = 0;
}

// Read-only bandwidth proxy (Section VII-B): grid-stride 16-byte loads, two
// adds per load.
template <int IPT, bool NT>
__global__ __launch_bounds__(1024) void k_bw_proxy(const v4u* x, int64_t nvec, unsigned* sink) {
  const int64_t bs = blockDim.x;
  const int64_t tile = bs * IPT;
  const int64_t ntiles = nvec / tile;
  unsigned acc = 0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    v4u v[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) v[u] = load_vec<NT>(x + t * tile + u * bs + threadIdx.x);
    __builtin_amdgcn_sched_barrier(0);  // all IPT loads in flight before use
#pragma unroll
    for (int u = 0; u < IPT; ++u) acc += v[u].x + v[u].y;
  }
  for (int64_t i = ntiles * tile + blockIdx.x * bs + threadIdx.x; i < nvec; i += gridDim.x * bs)
    acc += x[i].x + x[i].y;
  if (acc == 0x9E3779B9u) sink[blockIdx.x] = acc;  // keeps the loads live
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  int init() {
    RED_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
    RED_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
    return RED_OK;
  }
};

// Milliseconds between two events around `k` launches of one kernel.
int time_launches(const void* fn, int grid, int block, void** args, bool coop, int k, hipStream_t s,
                  Events& ev, double* ms) {
  RED_HIP(hipEventRecord(ev.a, s));
  for (int i = 0; i < k; ++i) {
    int rc = launch(fn, grid, block, args, s, coop);
    if (rc) return rc;
  }
  RED_HIP(hipEventRecord(ev.b, s));
  RED_HIP(hipEventSynchronize(ev.b));
  float f = 0.f;
  RED_HIP(hipEventElapsedTime(&f, ev.a, ev.b));
  *ms = f;
  return RED_OK;
}

// An executable graph of `k` launches of a one-argument wait kernel, its
// argument fixed at capture.  Captured on a private stream, so the caller's
// stream may be the null stream.
struct LaunchGraph {
  hipGraphExec_t exec = nullptr;
  ~LaunchGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
  int build(const void* fn, int grid, int block, long long ticks, int k) {
    hipStream_t cs = nullptr;
    RED_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    int rc = RED_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      void* args[] = {&ticks};
      for (int q = 0; q < k && rc == RED_OK; ++q) rc = launch(fn, grid, block, args, cs, false);
      e = hipStreamEndCapture(cs, &g);
    }
    if (rc == RED_OK && e != hipSuccess) rc = hip_fail(e, "graph capture");
    if (rc == RED_OK) {
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    return rc;
  }
};

int hip_check(hipError_t e) { return e == hipSuccess ? (int)RED_OK : hip_fail(e, "hipGraphLaunch"); }

// Milliseconds between two events around one replay of a graph.
int time_graph(const LaunchGraph& lg, hipStream_t s, Events& ev, double* ms) {
  RED_HIP(hipEventRecord(ev.a, s));
  RED_HIP(hipGraphLaunch(lg.exec, s));
  RED_HIP(hipEventRecord(ev.b, s));
  RED_HIP(hipEventSynchronize(ev.b));
  float f = 0.f;
  RED_HIP(hipEventElapsedTime(&f, ev.a, ev.b));
  *ms = f;
  return RED_OK;
}

double mean(const std::vector<double>& v) {
  double s = 0;
  for (double x : v) s += x;
  return s / v.size();
}

double median_of(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  const size_t n = v.size();
  return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

double sdev(const std::vector<double>& v) {
  const double m = mean(v);
  double s = 0;
  for (double x : v) s += (x - m) * (x - m);
  return v.size() > 1 ? std::sqrt(s / (v.size() - 1)) : 0.0;
}

// `reps` timed pairs of one launch with r1 and one with r2 repetitions:
// Eq. 7 on the mean latencies, Eq. 8 on their spreads.
template <class SetR, class ReadCycles>
int differential_pairs(const void* fn, int grid, int block, void** args, bool coop, int reps, hipStream_t s,
                       SetR set_r, ReadCycles read_cycles, int64_t r1, int64_t r2, Events& ev, double* ns,
                       double* sigma, double* per_op_counter) {
  std::vector<double> l1, l2, c1, c2;
  double ms = 0;
  int rc = RED_OK;
  for (int i = 0; i < reps; ++i) {
    set_r(r1);
    if ((rc = time_launches(fn, grid, block, args, coop, 1, s, ev, &ms))) return rc;
    l1.push_back(ms * 1e6);
    if (per_op_counter) c1.push_back(read_cycles());
    set_r(r2);
    if ((rc = time_launches(fn, grid, block, args, coop, 1, s, ev, &ms))) return rc;
    l2.push_back(ms * 1e6);
    if (per_op_counter) c2.push_back(read_cycles());
  }
  *ns = red_eq7_latency(mean(l1), mean(l2), r1, r2);
  *sigma = red_eq8_sigma(l1.data(), l2.data(), (int)l1.size(), r1, r2);
  if (per_op_counter) *per_op_counter = (mean(c1) - mean(c2)) / (double)(r1 - r2);
  return RED_OK;
}

// Runs the Eq. 7 / Eq. 8 differential between r1 and r2 repetitions.
// `set_r` rewrites the repetition argument; `read_cycles` (optional)
// returns the in-kernel counter of the last launch.
// r1 > r2 > 0 fixes the two repetition counts; r1 = r2 = 0 calibrates them.
template <class SetR, class ReadCycles>
int differential(const void* fn, int grid, int block, void** args, bool coop, int reps, hipStream_t s,
                 SetR set_r, ReadCycles read_cycles, double target_us, int64_t r_max, double* ns,
                 double* sigma, double* per_op_counter, int64_t r1_fixed = 0, int64_t r2_fixed = 0) {
  Events ev;
  int rc = ev.init();
  if (rc) return rc;
  double ms = 0;
  if (r1_fixed > 0) {
    set_r(r1_fixed);  // warm-up
    if ((rc = time_launches(fn, grid, block, args, coop, 1, s, ev, &ms))) return rc;
    return differential_pairs(fn, grid, block, args, coop, reps, s, set_r, read_cycles, r1_fixed, r2_fixed, ev,
                              ns, sigma, per_op_counter);
  }
  // Warm-up and calibration: choose r2 so that the r2 kernel runs about
  // target_us beyond its fixed cost, r1 = 8 r2 (Section IX-B: kernels must
  // be long enough to saturate the launch pipeline).
  int64_t rc_small = 16, rc_big = 16 * 64;
  set_r(rc_small);
  if ((rc = time_launches(fn, grid, block, args, coop, 1, s, ev, &ms))) return rc;
  double t_small = 0, t_big = 0;
  set_r(rc_small);
  if ((rc = time_launches(fn, grid, block, args, coop, 1, s, ev, &t_small))) return rc;
  set_r(rc_big);
  if ((rc = time_launches(fn, grid, block, args, coop, 1, s, ev, &t_big))) return rc;
  double per = std::max(1e-6, (t_big - t_small) * 1e3 / (double)(rc_big - rc_small));  // us per op
  int64_t r2 = (int64_t)std::ceil(target_us / per);
  r2 = std::max<int64_t>(4, std::min<int64_t>(r2, r_max / 8));
  const int64_t r1 = 8 * r2;
  return differential_pairs(fn, grid, block, args, coop, reps, s, set_r, read_cycles, r1, r2, ev, ns, sigma,
                            per_op_counter);
}

int read_i64(const long long* dptr, long long* h) {
  RED_HIP(hipMemcpy(h, dptr, sizeof(long long), hipMemcpyDeviceToHost));
  return RED_OK;
}

int probe_prologue(hipStream_t s, const DeviceInfo** dev, Workspace** ws) {
  int rc = ensure_device(dev);
  if (rc) return rc;
  if (stream_capturing(s)) return set_error(RED_EINVAL, "probes cannot run inside stream capture");
  return get_workspace(s, ws);
}

int reset_words(Workspace* ws, hipStream_t s) {
  void* args[] = {&ws->words};
  int rc = launch(reinterpret_cast<const void*>(&k_reset_words), 1, 64, args, s, false);
  if (rc) return rc;
  RED_HIP(hipStreamSynchronize(s));
  return RED_OK;
}

// The XCD-aggregated barrier shape of the device (flat on one XCD); with
// `skew` odd workgroups report the next XCD, which drives the barrier's
// fall-back path from the host.
unsigned xcd_groups(const DeviceInfo& dev, bool skew) {
  if (!xcd_tree_fits(dev.nxcc)) return 1u;
  return kBarrierXcd | (unsigned)dev.nxcc | (skew ? kBarrierSkew : 0u);
}

int coresident(const void* fn, int wg, const DeviceInfo& dev, int* n) {
  int per_cu = 0;
  RED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, wg, 0));
  *n = per_cu * dev.cus;
  return RED_OK;
}

}  // namespace

int bw_proxy_launch(const void* x, int64_t nbytes, int n_wg, int wg, bool nt, Workspace* ws, hipStream_t s) {
  const v4u* xv = static_cast<const v4u*>(x);
  int64_t nvec = nbytes / 16;
  unsigned* sink = ws->sink;
  void* args[] = {&xv, &nvec, &sink};
  const void* fn = nt ? reinterpret_cast<const void*>(&k_bw_proxy<4, true>)
                      : reinterpret_cast<const void*>(&k_bw_proxy<4, false>);
  return launch(fn, n_wg, wg, args, s, false);
}

// Wavefront-probe kernel of `op` on values of Op's type.
template <class Op>
const void* wave_chain_fn(int op) {
  switch (op) {
    case RED_WAVE_DPP: return reinterpret_cast<const void*>(&k_wave_chain<RED_WAVE_DPP, Op>);
    case RED_WAVE_SWIZZLE: return reinterpret_cast<const void*>(&k_wave_chain<RED_WAVE_SWIZZLE, Op>);
    case RED_WAVE_BPERMUTE: return reinterpret_cast<const void*>(&k_wave_chain<RED_WAVE_BPERMUTE, Op>);
    default: return reinterpret_cast<const void*>(&k_wave_chain<RED_WAVE_DPP_STEP, Op>);
  }
}

template <class Op>
const void* wave_once_fn(int op) {
  switch (op) {
    case RED_WAVE_DPP: return reinterpret_cast<const void*>(&k_wave_once<RED_WAVE_DPP, Op>);
    case RED_WAVE_SWIZZLE: return reinterpret_cast<const void*>(&k_wave_once<RED_WAVE_SWIZZLE, Op>);
    case RED_WAVE_BPERMUTE: return reinterpret_cast<const void*>(&k_wave_once<RED_WAVE_BPERMUTE, Op>);
    default: return reinterpret_cast<const void*>(&k_wave_once<RED_WAVE_DPP_STEP, Op>);
  }
}

}  // namespace redsum

using namespace redsum;

extern "C" {

double red_eq6_overhead(double lat_ij, double lat_ji, int i, int j) {
  return (lat_ij - lat_ji) / (double)(i - j);
}

double red_eq7_latency(double lat_k1, double lat_k2, int64_t r1, int64_t r2) {
  return (lat_k1 - lat_k2) / (double)(r1 - r2);
}

double red_eq8_sigma(const double* k1, const double* k2, int nsamp, int64_t r1, int64_t r2) {
  if (!k1 || !k2 || nsamp < 2 || r1 == r2) return NAN;
  std::vector<double> a(k1, k1 + nsamp), b(k2, k2 + nsamp);
  const double s1 = sdev(a), s2 = sdev(b);
  return std::sqrt(s1 * s1 + s2 * s2) / std::fabs((double)(r1 - r2));
}

int sync_bench_wave_ex(int op, int type, int wg_size, int reps, double* ns, double* sigma_ns, double* cycles,
                       void* stream) {
  if (op < RED_WAVE_DPP || op > RED_WAVE_DPP_STEP) return set_error(RED_EINVAL, "bad wave op %d", op);
  if (type < RED_WAVE_T_F32 || type > RED_WAVE_T_COMP) return set_error(RED_EINVAL, "bad wave type %d", type);
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (reps < 2 || !ns || !sigma_ns) return set_error(RED_EINVAL, "reps >= 2 and non-null outputs required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = type == RED_WAVE_T_F32   ? wave_chain_fn<OpF32>(op)
                   : type == RED_WAVE_T_I32 ? wave_chain_fn<OpU32>(op)
                   : type == RED_WAVE_T_F64 ? wave_chain_fn<OpF64>(op)
                   : type == RED_WAVE_T_I64 ? wave_chain_fn<OpU64>(op)
                                            : wave_chain_fn<OpComp>(op);
  int r = 0;
  unsigned* sink = ws->sink;
  long long* cyc = ws->stamps;
  void* args[] = {&r, &sink, &cyc};
  return differential(
      fn, 1, wg_size, args, false, reps, s, [&](int64_t v) { r = (int)v; },
      [&]() {
        long long h = 0;
        read_i64(cyc, &h);
        return (double)h;
      },
      20.0, 1 << 22, ns, sigma_ns, cycles);
}

int sync_bench_wave(int op, int wg_size, int reps, double* ns, double* sigma_ns, double* cycles,
                    void* stream) {
  return sync_bench_wave_ex(op, RED_WAVE_T_F32, wg_size, reps, ns, sigma_ns, cycles, stream);
}

int sync_bench_block(int wg_size, int n_wg, int reps, double* ns, double* sigma_ns, double* cycles,
                     void* stream) {
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (reps < 2 || !ns || !sigma_ns) return set_error(RED_EINVAL, "reps >= 2 and non-null outputs required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  int r = 0;
  long long* cyc = ws->stamps;
  void* args[] = {&r, &cyc};
  return differential(
      reinterpret_cast<const void*>(&k_block_chain), n_wg, wg_size, args, false, reps, s,
      [&](int64_t v) { r = (int)v; },
      [&]() {
        long long h = 0;
        read_i64(cyc, &h);
        return (double)h;
      },
      20.0, 1 << 22, ns, sigma_ns, cycles);
}

int sync_bench_grid_ex(int n_wg, int wg_size, int groups, int reps, double* ns, double* sigma_ns,
                       double* cycles, void* stream) {
  return sync_bench_grid_r(n_wg, wg_size, groups, 0, 0, reps, ns, sigma_ns, cycles, stream);
}

namespace {

int grid_probe(bool pub, int n_wg, int wg_size, int groups, int64_t r1, int64_t r2, int reps, double* ns,
               double* sigma_ns, double* cycles, void* stream) {
  if (!((r1 == 0 && r2 == 0) || (r1 > r2 && r2 > 0 && r1 <= (1 << 16))))
    return set_error(RED_EINVAL, "repetitions: r1 = r2 = 0, or r1 > r2 > 0 and r1 <= 65536");
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (groups < -2 || groups > kMaxBarrierGroups) return set_error(RED_EINVAL, "bad groups %d", groups);
  if (reps < 2 || !ns || !sigma_ns) return set_error(RED_EINVAL, "reps >= 2 and non-null outputs required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = pub ? reinterpret_cast<const void*>(&k_grid_chain<true>)
                       : reinterpret_cast<const void*>(&k_grid_chain<false>);
  int maxg = 0;
  if ((rc = coresident(fn, wg_size, *dev, &maxg))) return rc;
  if (n_wg > maxg)
    return set_error(RED_EINVAL, "grid probe: %d workgroups of %d threads are not co-resident (max %d)",
                     n_wg, wg_size, maxg);
  if ((rc = reset_words(ws, s))) return rc;
  int r = 0;
  BarrierWords* w = ws->words;
  unsigned grp = groups > 0 ? (unsigned)groups
                 : groups < 0 ? xcd_groups(*dev, groups == -2)
                              : barrier_groups(n_wg);
  unsigned spin = watchdog_spins();
  long long* st = ws->stamps;
  void* args[] = {&r, &w, &grp, &spin, &st};
  const double tick_ns = 1e6 / (double)dev->wallclock_khz;
  rc = differential(
      fn, n_wg, wg_size, args, true, reps, s, [&](int64_t v) { r = (int)v; },
      [&]() {
        long long h = 0;
        read_i64(st, &h);
        return (double)h * tick_ns;
      },
      50.0, 1 << 16, ns, sigma_ns, cycles, r1, r2);
  if (rc) return rc;
  unsigned err = 0;
  RED_HIP(hipMemcpy(&err, &ws->words->err.v, 4, hipMemcpyDeviceToHost));
  if (err) {
    reset_words(ws, s);
    return set_error(RED_ETIMEOUT, "grid probe: barrier watchdog fired");
  }
  return RED_OK;
}

}  // namespace

int sync_bench_grid_r(int n_wg, int wg_size, int groups, int64_t r1, int64_t r2, int reps, double* ns,
                      double* sigma_ns, double* cycles, void* stream) {
  return grid_probe(false, n_wg, wg_size, groups, r1, r2, reps, ns, sigma_ns, cycles, stream);
}

int sync_bench_grid_published(int n_wg, int wg_size, int groups, int64_t r1, int64_t r2, int reps, double* ns,
                              double* sigma_ns, double* cycles, void* stream) {
  return grid_probe(true, n_wg, wg_size, groups, r1, r2, reps, ns, sigma_ns, cycles, stream);
}

int sync_bench_grid(int n_wg, int wg_size, int reps, double* ns, double* sigma_ns, double* cycles,
                    void* stream) {
  return sync_bench_grid_ex(n_wg, wg_size, 0, reps, ns, sigma_ns, cycles, stream);
}

int sync_bench_relaunch(int n_wg, int wg_size, int cooperative, int reps, double* ns, double* sigma_ns,
                        double* null_kernel_ns, void* stream) {
  // (i, j) = (8, 1) with a 5 us wait unit (Section IX-B: about 5 us keeps
  // one GPU's launch pipeline saturated); 0 ticks: 5 us of this device's
  // wall clock.
  return sync_bench_relaunch_ex(n_wg, wg_size, cooperative, 8, 1, 0, reps, ns, sigma_ns, null_kernel_ns, stream);
}

int sync_bench_relaunch_ex(int n_wg, int wg_size, int cooperative, int i, int j, int64_t unit_ticks, int reps,
                           double* ns, double* sigma_ns, double* null_kernel_ns, void* stream) {
  if (i < 1 || j < 1 || i == j || i > 64 || j > 64) return set_error(RED_EINVAL, "launch counts: 1 <= i, j <= 64, i != j");
  if (unit_ticks < 0 || unit_ticks > 100000000) return set_error(RED_EINVAL, "unit_ticks out of range");
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (cooperative < 0 || cooperative > 2)
    return set_error(RED_EINVAL, "launch type %d: 0 ordinary, 1 cooperative, 2 graph", cooperative);
  if (reps < 2 || !ns || !sigma_ns) return set_error(RED_EINVAL, "reps >= 2 and non-null outputs required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (cooperative == 2 && stream_capturing(s))
    return set_error(RED_EINVAL, "graph launch probe inside a stream capture");
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = reinterpret_cast<const void*>(&k_spin);
  const bool coop = cooperative == 1;
  const bool graph = cooperative == 2;
  if (coop) {
    int maxg = 0;
    if ((rc = coresident(fn, wg_size, *dev, &maxg))) return rc;
    if (n_wg > maxg) return set_error(RED_EINVAL, "relaunch probe: cooperative grid too large (max %d)", maxg);
  }
  Events ev;
  if ((rc = ev.init())) return rc;
  long long ticks = 0;
  void* args[] = {&ticks};
  const long long unit = unit_ticks > 0 ? unit_ticks : std::max<long long>(1, dev->wallclock_khz * 5 / 1000);
  double ms = 0;
  // Graph form: i kernels of j units and j kernels of i units, each one graph.
  LaunchGraph g_ij, g_ji;
  if (graph) {
    if ((rc = g_ij.build(fn, n_wg, wg_size, unit * j, i))) return rc;
    if ((rc = g_ji.build(fn, n_wg, wg_size, unit * i, j))) return rc;
  }
  auto run_ij = [&](double* t) {
    if (graph) return time_graph(g_ij, s, ev, t);
    ticks = unit * j;
    return time_launches(fn, n_wg, wg_size, args, coop, i, s, ev, t);
  };
  auto run_ji = [&](double* t) {
    if (graph) return time_graph(g_ji, s, ev, t);
    ticks = unit * i;
    return time_launches(fn, n_wg, wg_size, args, coop, j, s, ev, t);
  };
  if ((rc = run_ij(&ms))) return rc;  // warm-up
  if ((rc = run_ji(&ms))) return rc;
  std::vector<double> lij, lji;
  for (int k = 0; k < reps; ++k) {
    if ((rc = run_ij(&ms))) return rc;
    lij.push_back(ms * 1e6);
    if ((rc = run_ji(&ms))) return rc;
    lji.push_back(ms * 1e6);
  }
  *ns = red_eq6_overhead(mean(lij), mean(lji), i, j);
  *sigma_ns = red_eq8_sigma(lij.data(), lji.data(), (int)lij.size(), i, j);
  if (null_kernel_ns && graph) {
    // One replay launches the whole graph, so the host clock around a
    // replay does not separate its kernels: the per-kernel latency of a
    // null kernel inside a graph is the Eq. 7 differential between graphs
    // of 40 and of 5 null kernels, timed with events.
    constexpr int kBig = 40, kSmall = 5;
    LaunchGraph gb, gs;
    if ((rc = gb.build(fn, n_wg, wg_size, 0, kBig))) return rc;
    if ((rc = gs.build(fn, n_wg, wg_size, 0, kSmall))) return rc;
    if ((rc = time_graph(gb, s, ev, &ms))) return rc;  // warm-up
    if ((rc = time_graph(gs, s, ev, &ms))) return rc;
    std::vector<double> lb, ls;
    for (int k = 0; k < reps; ++k) {
      if ((rc = time_graph(gb, s, ev, &ms))) return rc;
      lb.push_back(ms * 1e6);
      if ((rc = time_graph(gs, s, ev, &ms))) return rc;
      ls.push_back(ms * 1e6);
    }
    *null_kernel_ns = red_eq7_latency(mean(lb), mean(ls), kBig, kSmall);
  } else if (null_kernel_ns) {
    // Section IV: host clock around 1 launch and around 5 launches of a
    // null kernel, each followed by a device synchronization; the median
    // over the repetitions, because a host-side stall of a few us in one
    // repetition moves the mean by more than the figure itself.
    ticks = 0;
    auto one = [&]() { return launch(fn, n_wg, wg_size, args, s, coop); };
    auto five = [&]() {
      for (int q = 0; q < 5; ++q) {
        int r = launch(fn, n_wg, wg_size, args, s, coop);
        if (r) return r;
      }
      return (int)RED_OK;
    };
    std::vector<double> tot;
    for (int k = 0; k < reps; ++k) {
      auto t1 = std::chrono::steady_clock::now();
      if ((rc = one())) return rc;
      RED_HIP(hipStreamSynchronize(s));
      auto t2 = std::chrono::steady_clock::now();
      if ((rc = five())) return rc;
      RED_HIP(hipStreamSynchronize(s));
      auto t3 = std::chrono::steady_clock::now();
      const double a = std::chrono::duration<double, std::nano>(t2 - t1).count();
      const double b = std::chrono::duration<double, std::nano>(t3 - t2).count();
      tot.push_back((b - a) / 4.0);
    }
    *null_kernel_ns = median_of(tot);
  }
  return RED_OK;
}

int sync_bench_block_tput(int wg_size, int wg_per_cu, int64_t window_ticks, double* barriers_per_us_per_cu,
                          double* cycles_per_barrier, void* stream) {
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (wg_per_cu < 1 || wg_per_cu > 32) return set_error(RED_EINVAL, "bad wg_per_cu %d", wg_per_cu);
  if (window_ticks < 100 || window_ticks > 100000000) return set_error(RED_EINVAL, "window_ticks out of range");
  if (!barriers_per_us_per_cu) return set_error(RED_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = reinterpret_cast<const void*>(&k_block_tput);
  int maxg = 0;
  if ((rc = coresident(fn, wg_size, *dev, &maxg))) return rc;
  const int n_wg = wg_per_cu * dev->cus;
  if (n_wg > maxg || n_wg > RED_MAX_GRID)
    return set_error(RED_EINVAL, "%d workgroups of %d threads per CU are not co-resident", wg_per_cu, wg_size);
  long long* counts = ws->stamps;
  long long* ticks = ws->stamps + RED_MAX_GRID;
  long long window = (long long)window_ticks;
  void* args[] = {&window, &counts, &ticks};
  if ((rc = launch(fn, n_wg, wg_size, args, s, false))) return rc;  // warm-up
  if ((rc = launch(fn, n_wg, wg_size, args, s, false))) return rc;
  RED_HIP(hipStreamSynchronize(s));
  std::vector<long long> hc(n_wg), ht(n_wg);
  RED_HIP(hipMemcpy(hc.data(), counts, n_wg * sizeof(long long), hipMemcpyDeviceToHost));
  RED_HIP(hipMemcpy(ht.data(), ticks, n_wg * sizeof(long long), hipMemcpyDeviceToHost));
  const double tick_us = 1e3 / (double)dev->wallclock_khz;
  double rate = 0, per = 0;  // barriers per microsecond, summed over workgroups; microseconds per barrier
  for (int k = 0; k < n_wg; ++k) {
    const double us = (double)ht[k] * tick_us;
    if (hc[k] <= 0 || us <= 0) return set_error(RED_EHIP, "block throughput probe: empty record %d", k);
    rate += (double)hc[k] / us;
    per += us / (double)hc[k];
  }
  *barriers_per_us_per_cu = rate / dev->cus;
  if (cycles_per_barrier) *cycles_per_barrier = per / n_wg * (double)dev->clock_khz * 1e-3;
  return RED_OK;
}

int sync_bench_spin(int64_t unit_ticks, int64_t r1, int64_t r2, int reps, double* ns, double* sigma_ns,
                    void* stream) {
  if (unit_ticks < 1 || r2 < 1 || r1 <= r2 || r1 * unit_ticks > 100000000)
    return set_error(RED_EINVAL, "need unit_ticks >= 1, r1 > r2 >= 1, r1 * unit_ticks <= 1e8");
  if (reps < 2 || !ns || !sigma_ns) return set_error(RED_EINVAL, "reps >= 2 and non-null outputs required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  long long ticks = 0;
  void* args[] = {&ticks};
  return differential(
      reinterpret_cast<const void*>(&k_spin), 1, 64, args, false, reps, s,
      [&](int64_t v) { ticks = (long long)(v * unit_ticks); }, [&]() { return 0.0; }, 0.0, 0, ns, sigma_ns,
      nullptr, r1, r2);
}

int sync_check_wave(int op, int type, const void* host_in, void* host_out, void* stream) {
  if (op < RED_WAVE_DPP || op > RED_WAVE_DPP_STEP) return set_error(RED_EINVAL, "bad wave op %d", op);
  if (type < RED_WAVE_T_F32 || type > RED_WAVE_T_COMP) return set_error(RED_EINVAL, "bad wave type %d", type);
  if (!host_in || !host_out) return set_error(RED_EINVAL, "null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const size_t esz = (type == RED_WAVE_T_F32 || type == RED_WAVE_T_I32) ? 4 : 8;
  char* in = reinterpret_cast<char*>(ws->stamps);  // 64 values in, 64 out
  char* out = in + kWave * 8;
  RED_HIP(hipMemcpyAsync(in, host_in, kWave * esz, hipMemcpyHostToDevice, s));
  const void* fn = type == RED_WAVE_T_F32   ? wave_once_fn<OpF32>(op)
                   : type == RED_WAVE_T_I32 ? wave_once_fn<OpU32>(op)
                   : type == RED_WAVE_T_F64 ? wave_once_fn<OpF64>(op)
                   : type == RED_WAVE_T_I64 ? wave_once_fn<OpU64>(op)
                                            : wave_once_fn<OpComp>(op);
  void* args[] = {&in, &out};
  if ((rc = launch(fn, 1, kWave, args, s, false))) return rc;
  RED_HIP(hipMemcpyAsync(host_out, out, kWave * esz, hipMemcpyDeviceToHost, s));
  RED_HIP(hipStreamSynchronize(s));
  return RED_OK;
}

int sync_check_grid_order(int n_wg, int wg_size, int64_t* max_before, int64_t* min_after, void* stream) {
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (!max_before || !min_after) return set_error(RED_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = reinterpret_cast<const void*>(&k_grid_order);
  int maxg = 0;
  if ((rc = coresident(fn, wg_size, *dev, &maxg))) return rc;
  if (n_wg > maxg) return set_error(RED_EINVAL, "order check: grid too large (max %d)", maxg);
  if ((rc = reset_words(ws, s))) return rc;
  BarrierWords* w = ws->words;
  unsigned grp = barrier_groups(n_wg);
  unsigned spin = watchdog_spins();
  long long* before = ws->stamps;
  long long* after = ws->stamps + RED_MAX_GRID;
  void* args[] = {&w, &grp, &spin, &before, &after};
  if ((rc = launch(fn, n_wg, wg_size, args, s, true))) return rc;
  RED_HIP(hipStreamSynchronize(s));
  std::vector<long long> hb(n_wg), ha(n_wg);
  RED_HIP(hipMemcpy(hb.data(), before, n_wg * sizeof(long long), hipMemcpyDeviceToHost));
  RED_HIP(hipMemcpy(ha.data(), after, n_wg * sizeof(long long), hipMemcpyDeviceToHost));
  unsigned err = 0;
  RED_HIP(hipMemcpy(&err, &ws->words->err.v, 4, hipMemcpyDeviceToHost));
  if (err) {
    reset_words(ws, s);
    return set_error(RED_ETIMEOUT, "order check: barrier watchdog fired");
  }
  *max_before = *std::max_element(hb.begin(), hb.end());
  *min_after = *std::min_element(ha.begin(), ha.end());
  return RED_OK;
}

namespace {

int grid_visibility(bool pub, int n_wg, int wg_size, int groups, int rounds, int64_t* errors, void* stream) {
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (groups < -2 || groups > kMaxBarrierGroups) return set_error(RED_EINVAL, "bad groups %d", groups);
  if (rounds < 1 || rounds > 100000) return set_error(RED_EINVAL, "bad rounds %d", rounds);
  if (!errors) return set_error(RED_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = pub ? reinterpret_cast<const void*>(&k_grid_visibility<true>)
                       : reinterpret_cast<const void*>(&k_grid_visibility<false>);
  int maxg = 0;
  if ((rc = coresident(fn, wg_size, *dev, &maxg))) return rc;
  if (n_wg > maxg) return set_error(RED_EINVAL, "visibility check: grid too large (max %d)", maxg);
  if ((rc = reset_words(ws, s))) return rc;
  BarrierWords* w = ws->words;
  unsigned grp = groups > 0 ? (unsigned)groups
                 : groups < 0 ? xcd_groups(*dev, groups == -2)
                              : barrier_groups(n_wg);
  unsigned spin = watchdog_spins();
  long long* data = ws->stamps;  // RED_MAX_GRID slots
  unsigned long long* err_count = reinterpret_cast<unsigned long long*>(ws->stamps + RED_MAX_GRID);
  RED_HIP(hipMemsetAsync(err_count, 0, sizeof(unsigned long long), s));
  void* args[] = {&w, &grp, &spin, &data, &err_count, &rounds};
  if ((rc = launch(fn, n_wg, wg_size, args, s, true))) return rc;
  RED_HIP(hipStreamSynchronize(s));
  unsigned long long h = 0;
  RED_HIP(hipMemcpy(&h, err_count, sizeof h, hipMemcpyDeviceToHost));
  unsigned err = 0;
  RED_HIP(hipMemcpy(&err, &ws->words->err.v, 4, hipMemcpyDeviceToHost));
  if (err) {
    reset_words(ws, s);
    return set_error(err == kErrTimeout ? RED_ETIMEOUT : RED_ENOTSUP, "visibility check: barrier error %u", err);
  }
  *errors = (int64_t)h;
  return RED_OK;
}

}  // namespace

int sync_check_grid_visibility(int n_wg, int wg_size, int groups, int rounds, int64_t* errors, void* stream) {
  return grid_visibility(false, n_wg, wg_size, groups, rounds, errors, stream);
}

int sync_check_grid_visibility_published(int n_wg, int wg_size, int groups, int rounds, int64_t* errors,
                                         void* stream) {
  return grid_visibility(true, n_wg, wg_size, groups, rounds, errors, stream);
}

int sync_check_watchdog(int n_wg, int wg_size, int skip_wg, int spin_limit, void* stream) {
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 2 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (skip_wg < 0 || skip_wg >= n_wg) return set_error(RED_EINVAL, "skip_wg out of range");
  if (spin_limit < 1 || spin_limit > (1 << 24)) return set_error(RED_EINVAL, "spin_limit out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  const void* fn = reinterpret_cast<const void*>(&k_watchdog);
  int maxg = 0;
  if ((rc = coresident(fn, wg_size, *dev, &maxg))) return rc;
  if (n_wg > maxg) return set_error(RED_EINVAL, "watchdog check: grid too large (max %d)", maxg);
  if ((rc = reset_words(ws, s))) return rc;
  BarrierWords* w = ws->words;
  unsigned grp = barrier_groups(n_wg);
  unsigned spin = (unsigned)spin_limit;
  void* args[] = {&w, &skip_wg, &grp, &spin};
  if ((rc = launch(fn, n_wg, wg_size, args, s, true))) return rc;
  return red_check_error(stream);
}

int sync_xcc_map(int n_wg, int wg_size, int32_t* host_xcc, void* stream) {
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  if (!host_xcc) return set_error(RED_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  Workspace* ws;
  int rc = probe_prologue(s, &dev, &ws);
  if (rc) return rc;
  int* out = reinterpret_cast<int*>(ws->stamps);  // 2 * RED_MAX_GRID int64 slots
  void* args[] = {&out};
  if ((rc = launch(reinterpret_cast<const void*>(&k_xcc_map), n_wg, wg_size, args, s, false))) return rc;
  RED_HIP(hipStreamSynchronize(s));
  RED_HIP(hipMemcpy(host_xcc, out, (size_t)n_wg * sizeof(int32_t), hipMemcpyDeviceToHost));
  return RED_OK;
}

int red_bw_proxy(const void* x, int64_t nbytes, int n_wg, int wg_size, void* stream) {
  return red_bw_proxy_ex(x, nbytes, n_wg, wg_size, 0, stream);
}

int red_bw_proxy_ex(const void* x, int64_t nbytes, int n_wg, int wg_size, int flags, void* stream) {
  if (flags & ~RED_FLAG_NONTEMPORAL) return set_error(RED_EINVAL, "unknown flags 0x%x", flags);
  if (!x || nbytes < 0) return set_error(RED_EINVAL, "bad buffer");
  if (reinterpret_cast<uintptr_t>(x) & 15) return set_error(RED_EINVAL, "x must be 16-byte aligned");
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad wg_size %d", wg_size);
  if (n_wg < 1 || n_wg > RED_MAX_GRID) return set_error(RED_EINVAL, "bad n_wg %d", n_wg);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  Workspace* ws;
  if ((rc = get_workspace(s, &ws))) return rc;
  return bw_proxy_launch(x, nbytes, n_wg, wg_size, (flags & RED_FLAG_NONTEMPORAL) != 0, ws, s);
}

}  // extern "C"
