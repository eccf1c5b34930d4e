// Device-wide sum reduction kernels for gfx950 and their host dispatch.
//
// Section VII-C (single-GPU reduction) of Zhang et al. describes two ways of
// synchronizing the device between the per-block partial sums and the final
// combine: an implicit barrier between two kernels on one stream
// (Kernel1/Kernel2), and an explicit grid barrier inside one persistent
// cooperative kernel.  Both are built here, plus a third single-kernel form
// in which the last workgroup to arrive (atomic ticket) does the final
// combine, which needs no co-residency.
//
// Every variant shares the same per-thread accumulation (the paper's
// `summing`, a grid-stride loop, here over 16-byte vectors with IPT loads in
// flight per thread) and the same workgroup combine (the paper's
// `block_reduce`, here a DPP wavefront combine, LDS staging and a second
// wavefront combine in wave 0).  One partial per workgroup is stored (int64
// for int32 input, binary64 for floating-point input), and the final
// combine sums the partials in a fixed order, so a plan gives bit-identical
// results on every call.
#include <algorithm>

#include "device_prims.h"
#include "internal.h"

namespace redsum {

// Arguments of every reduction kernel (passed by value).
struct ReduceArgs {
  const void* x;
  int64_t head;   // scalar elements before the first 16-byte boundary
  int64_t nvec;   // full 16-byte vectors after the head
  int64_t tail;   // scalar elements after the vectors
  void* partials; // one Part per workgroup
  BarrierWords* words;
  void* out;      // one Part
  unsigned spin_limit;
  unsigned bar_groups;  // grid-barrier shape (persistent variant)
  unsigned xcd_nxcc;    // atomic variant: XCD-aggregated publication over this many XCDs (0 = off)
};

// Per-thread accumulation of this thread's grid-stride share.  The vector
// body is cut into tiles of blockDim.x * IPT vectors; workgroup g takes
// tiles g, g + G, ...; inside a tile, load u of thread t reads vector
// u * blockDim.x + t, so each wavefront load instruction reads 1 KiB of
// contiguous memory.  IPT independent accumulators keep IPT loads in flight.
// With PIPE the loads of the workgroup's next tile are issued before the
// arithmetic of the current one (two register buffers), so a wave keeps
// loads in flight while it computes.
template <int IPT, bool NT, class Vec>
__device__ __forceinline__ void load_tile(Vec (&v)[IPT], const Vec* xv, int64_t t, int64_t tile, int64_t bs) {
  const Vec* p = xv + t * tile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < IPT; ++u) v[u] = load_vec<NT>(p + u * bs);
}

template <class M, int IPT, bool NT, bool PIPE>
__device__ __forceinline__ typename M::Acc thread_accumulate(const ReduceArgs& a) {
  using In = typename M::In;
  using Vec = typename M::Vec;
  using Acc = typename M::Acc;
  const In* x = static_cast<const In*>(a.x);
  const Vec* xv = reinterpret_cast<const Vec*>(x + a.head);
  const int64_t bs = blockDim.x;
  const int64_t tile = bs * IPT;
  const int64_t ntiles = a.nvec / tile;
  const int64_t G = gridDim.x;

  Acc acc[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) acc[u] = M::zero();

  if constexpr (!PIPE) {
    for (int64_t t = blockIdx.x; t < ntiles; t += G) {
      Vec v[IPT];
      load_tile<IPT, NT>(v, xv, t, tile, bs);
      // Keep the IPT loads issued back to back before any of them is used,
      // so that they are all in flight together.
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], v[u]);
    }
  } else {
    // The loop leaves before a prefetch rather than guarding it, so the
    // loads stay in straight-line code and the compiler's wait counts only
    // wait for the older buffer.
    Vec va[IPT], vb[IPT];
    int64_t t = blockIdx.x;
    if (t < ntiles) {
      load_tile<IPT, NT>(va, xv, t, tile, bs);
      for (;;) {
        const int64_t t2 = t + G;
        if (t2 >= ntiles) {
#pragma unroll
          for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], va[u]);
          break;
        }
        load_tile<IPT, NT>(vb, xv, t2, tile, bs);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], va[u]);
        const int64_t t3 = t2 + G;
        if (t3 >= ntiles) {
#pragma unroll
          for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], vb[u]);
          break;
        }
        load_tile<IPT, NT>(va, xv, t3, tile, bs);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < IPT; ++u) M::add_vec(acc[u], vb[u]);
        t = t3;
      }
    }
  }
  // Vectors after the last full tile.
  for (int64_t i = ntiles * tile + (int64_t)blockIdx.x * bs + threadIdx.x; i < a.nvec;
       i += (int64_t)gridDim.x * bs)
    M::add_vec(acc[0], load_vec<NT>(xv + i));
  // Unaligned head and the tail: fewer than 16 bytes each, workgroup 0.
  if (blockIdx.x == 0) {
    const int64_t t = threadIdx.x;
    if (t < a.head)
      M::add_elem(acc[0], x[t]);
    else if (t < a.head + a.tail)
      M::add_elem(acc[0], x[a.head + a.nvec * M::kVE + (t - a.head)]);
  }
#pragma unroll
  for (int u = 1; u < IPT; ++u) acc[0] = M::Op::add(acc[0], acc[u]);
  return acc[0];
}

// Workgroup total of the thread accumulators, as the stored partial type
// (valid in thread 0).
template <class M, int IPT, bool NT, bool PIPE>
__device__ __forceinline__ typename M::Part workgroup_partial(const ReduceArgs& a) {
  __shared__ typename M::Op::T lds[kMaxWavesPerWG];
  typename M::Acc acc = thread_accumulate<M, IPT, NT, PIPE>(a);
  return M::to_part(block_reduce<typename M::Op>(acc, lds));
}

// Final combine of `count` partials by one workgroup: thread t sums
// partials t, t + blockDim.x, ... in order, then the workgroup combine.
// Deterministic for a fixed (count, blockDim.x).  Valid in thread 0.
template <class Part>
__device__ __forceinline__ Part combine_partials(const Part* partials, int count) {
  using Op = typename PartOp<Part>::type;
  __shared__ Part lds[kMaxWavesPerWG];
  Part s = Op::zero();
  for (int i = threadIdx.x; i < count; i += blockDim.x) s = Op::add(s, partials[i]);
  return block_reduce<Op>(s, lds);
}

// ---------------------------------------------------------------------------
// Variant 1, implicit barrier: kernel 1 writes one partial per workgroup,
// kernel 2 (one workgroup) combines them.
// ---------------------------------------------------------------------------
template <class M, int IPT, bool NT, bool PIPE>
__global__ __launch_bounds__(1024) void k_partials(ReduceArgs a) {
  typename M::Part p = workgroup_partial<M, IPT, NT, PIPE>(a);
  if (threadIdx.x == 0) static_cast<typename M::Part*>(a.partials)[blockIdx.x] = p;
}

template <class Part>
__global__ __launch_bounds__(1024) void k_final(const Part* partials, int count, Part* out) {
  Part s = combine_partials<Part>(partials, count);
  if (threadIdx.x == 0) *out = s;
}

// One-wavefront final combine (no LDS, no barrier): lane l sums partials
// l, l + 64, ... in order, then the DPP wavefront combine.
template <class Part>
__global__ __launch_bounds__(64) void k_final_wave(const Part* partials, int count, Part* out) {
  using Op = typename PartOp<Part>::type;
  Part s = Op::zero();
#pragma unroll 8
  for (int i = threadIdx.x; i < count; i += kWave) s = Op::add(s, partials[i]);
  s = wave_reduce_dpp<Op>(s);
  if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Variant 2, one kernel with an atomic ticket: each workgroup publishes its
// partial (int64 or binary64) to its slot with a device-scope atomic store,
// waits for it to complete, then takes a ticket; the workgroup that draws
// the last ticket acquires and does the ordered final combine.  The
// partials being atomics, no workgroup writes back its L2.  The ticket is
// two-level (one line per group of blockIdx % g, then the ticket line),
// every line wrapping to zero on its last arrival, so the tail of a launch
// does not queue all of its workgroups on one line; under RED_FLAG_XCD the
// XCD arrival tree counts instead.
// ---------------------------------------------------------------------------
template <class M, int IPT, bool NT, bool PIPE>
__global__ __launch_bounds__(1024) void k_atomic(ReduceArgs a) {
  using Part = typename M::Part;
  __shared__ int is_last;
  Part p = workgroup_partial<M, IPT, NT, PIPE>(a);
  BarrierWords* w = a.words;
  if (threadIdx.x == 0) {
    publish(static_cast<Part*>(a.partials) + blockIdx.x, p);
    // The partial is complete before the ticket: only the last workgroup
    // pays a fence (its acquire).
    drain_stores();
    bool last;
    if (a.xcd_nxcc > 1) {
      // The workgroups count themselves on the XCD arrival tree, whose last
      // arrival takes the ticket (its uniformity check does not matter: the
      // partials need no L2 write-back).
      bool ok = true;
      last = xcd_tree_arrive<false>(w, w->ticket, gridDim.x, kBarrierXcd | a.xcd_nxcc, &ok);
    } else {
      // Two-level ticket: the workgroups with equal blockIdx % g count on
      // one line per group, the last of each group on the ticket line;
      // every line wraps to zero on its last arrival.
      const unsigned G = gridDim.x;
      const unsigned g = default_barrier_groups(G);
      const unsigned grp = blockIdx.x % g;
      const unsigned members = (G - grp + g - 1) / g;
      const unsigned active = G < g ? G : g;
      last = false;
      if (g <= 1 || wrap_inc(&w->group[grp].v, members - 1) == members - 1)
        last = wrap_inc(&w->ticket.v, (g <= 1 ? G : active) - 1) == (g <= 1 ? G : active) - 1;
    }
    is_last = last;
  }
  __syncthreads();
  if (!is_last) return;
  // Last workgroup: every thread acquires before reading the others' data.
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  Part s = combine_partials<Part>(static_cast<const Part*>(a.partials), gridDim.x);
  if (threadIdx.x == 0) *static_cast<Part*>(a.out) = s;
}

// ---------------------------------------------------------------------------
// Variant 3, explicit barrier: one cooperative (co-resident) kernel; every
// workgroup publishes its partial (device-scope atomic store) and arrives
// at the grid barrier, workgroup 0 waits for all of them and combines.
// Only workgroup 0 reads after the barrier, so it is split (arrive / wait):
// the others leave on arrival, with no L2 write-back and no acquire.
// ---------------------------------------------------------------------------
template <class M, int IPT, bool NT, bool PIPE>
__global__ __launch_bounds__(1024) void k_persistent(ReduceArgs a) {
  using Part = typename M::Part;
  unsigned gen = grid_barrier_gen(a.words);
  Part p = workgroup_partial<M, IPT, NT, PIPE>(a);
  if (threadIdx.x == 0) publish(static_cast<Part*>(a.partials) + blockIdx.x, p);
  // Workgroup 0 alone reads the partials: the others arrive and leave.
  grid_barrier_to(a.words, gridDim.x, a.bar_groups, a.spin_limit, gen, blockIdx.x == 0);
  if (blockIdx.x != 0) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  Part s = combine_partials<Part>(static_cast<const Part*>(a.partials), gridDim.x);
  if (threadIdx.x == 0) *static_cast<Part*>(a.out) = s;
}

// ---------------------------------------------------------------------------
// Variant 4, one workgroup: the whole sum in one workgroup, written directly
// (no partials, no device-wide synchronization).
// ---------------------------------------------------------------------------
template <class M, int IPT, bool NT, bool PIPE>
__global__ __launch_bounds__(1024) void k_single(ReduceArgs a) {
  typename M::Part p = workgroup_partial<M, IPT, NT, PIPE>(a);
  if (threadIdx.x == 0) *static_cast<typename M::Part*>(a.out) = p;
}

template <class Part>
__global__ void k_write_zero(Part* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = Part(0);
}

// ---------------------------------------------------------------------------
// Host dispatch
// ---------------------------------------------------------------------------
namespace {

// Element modes by (dtype, acc).
enum ModeId { kI32 = 0, kF32C, kF32P, kF16C, kF16P, kBF16C, kBF16P, kNumModes };

int mode_of(int dtype, int acc) {
  switch (dtype) {
    case RED_I32: return kI32;
    case RED_F32: return acc == RED_ACC_PLAIN ? kF32P : kF32C;
    case RED_F16: return acc == RED_ACC_PLAIN ? kF16P : kF16C;
    case RED_BF16: return acc == RED_ACC_PLAIN ? kBF16P : kBF16C;
  }
  return -1;
}

int elem_size(int dtype) { return dtype == RED_I32 || dtype == RED_F32 ? 4 : 2; }

constexpr int kIpts[4] = {1, 2, 4, 8};
int ipt_index(int ipt) { return ipt == 1 ? 0 : ipt == 2 ? 1 : ipt == 4 ? 2 : ipt == 8 ? 3 : -1; }

struct KernelSet {
  const void* partials;
  const void* atomic;
  const void* persistent;
  const void* single;
};

template <class M, int IPT, bool NT, bool PIPE>
KernelSet make_set() {
  return KernelSet{reinterpret_cast<const void*>(&k_partials<M, IPT, NT, PIPE>),
                   reinterpret_cast<const void*>(&k_atomic<M, IPT, NT, PIPE>),
                   reinterpret_cast<const void*>(&k_persistent<M, IPT, NT, PIPE>),
                   reinterpret_cast<const void*>(&k_single<M, IPT, NT, PIPE>)};
}

template <class M, bool NT, bool PIPE>
void fill_ipts(KernelSet* row) {
  row[0] = make_set<M, 1, NT, PIPE>();
  row[1] = make_set<M, 2, NT, PIPE>();
  row[2] = make_set<M, 4, NT, PIPE>();
  row[3] = make_set<M, 8, NT, PIPE>();
}

template <class M>
void fill_mode(KernelSet (*m)[2][4]) {
  fill_ipts<M, false, false>(m[0][0]);
  fill_ipts<M, false, true>(m[0][1]);
  fill_ipts<M, true, false>(m[1][0]);
  fill_ipts<M, true, true>(m[1][1]);
}

struct Table {
  KernelSet k[kNumModes][2][2][4];  // mode, nontemporal, pipelined, ipt index
  Table() {
    fill_mode<ModeI32>(k[kI32]);
    fill_mode<ModeF32Comp>(k[kF32C]);
    fill_mode<ModeF32Plain>(k[kF32P]);
    fill_mode<ModeHalfComp<F16>>(k[kF16C]);
    fill_mode<ModeHalfPlain<F16>>(k[kF16P]);
    fill_mode<ModeHalfComp<Bf16>>(k[kBF16C]);
    fill_mode<ModeHalfPlain<Bf16>>(k[kBF16P]);
  }
};

const Table& table() {
  static const Table t;
  return t;
}

constexpr int kFinalWG = 256;

}  // namespace

int validate_plan(const red_plan& p) {
  if (p.variant < RED_VARIANT_RELAUNCH || p.variant > RED_VARIANT_SINGLE)
    return set_error(RED_EINVAL, "plan: variant %d out of range", p.variant);
  if (p.wg < 64 || p.wg > 1024 || p.wg % 64 != 0)
    return set_error(RED_EINVAL, "plan: workgroup size %d must be a multiple of 64 in [64, 1024]", p.wg);
  if (ipt_index(p.ipt) < 0) return set_error(RED_EINVAL, "plan: ipt %d must be 1, 2, 4 or 8", p.ipt);
  if (p.grid < 0 || p.grid > RED_MAX_GRID)
    return set_error(RED_EINVAL, "plan: grid %d out of range [0, %d]", p.grid, RED_MAX_GRID);
  if (p.flags & ~(RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH | RED_FLAG_PIPELINE | RED_FLAG_XCD))
    return set_error(RED_EINVAL, "plan: unknown flags 0x%x", p.flags);
  return RED_OK;
}

// Performance model of Section VII-A (Eq. 1-5) between one workgroup
// ("basic": latency T, throughput Thr_basic) and the whole device ("more":
// T + T_sync, Thr_more).  With C = T * Thr (Eq. 1), n bytes go to the basic
// configuration when n <= C_basic; between the two concurrencies when
// n < N_m = (T + T_sync) * Thr_basic (Eq. 4); beyond both when
// n < N_l = T_sync * Thr_more * Thr_basic / (Thr_more - Thr_basic) (Eq. 5).
// Constants measured on MI355X (one 1024-thread workgroup with two 16-byte
// loads per thread; the device-wide atomic-ticket variant on a grid sized
// by the work); the small-size sweep puts the measured crossover at about
// 2^17 fp32 elements, the model at (T + T_sync) * Thr_basic = 500 KB.
constexpr double kModelTBasicUs = 4.2;        // one-workgroup kernel, fixed cost
constexpr double kModelTsyncUs = 0.8;         // extra fixed cost of the device-wide kernel
constexpr double kModelThrBasicGBps = 100.0;  // one workgroup
constexpr double kModelThrMoreGBps = 7000.0;  // whole device
// Above this many bytes the two-kernel relaunch variant overtakes the
// atomic ticket (its publication cost grows with the grid): measured
// device times per call 7.7 against 8.0 us at 1 MiB, 9.1 against 8.1 us at
// 2 MiB.
constexpr int64_t kAtomicMaxBytes = 1LL << 20;

int64_t single_wg_switch_bytes() {
  const double tb = kModelThrBasicGBps * 1e3, tm = kModelThrMoreGBps * 1e3;  // bytes / us
  const double c_basic = kModelTBasicUs * tb;                                // Eq. 1
  const double c_more = kModelTBasicUs * tm;
  const double n_m = (kModelTBasicUs + kModelTsyncUs) * tb;                  // Eq. 4
  const double n_l = kModelTsyncUs * tm * tb / (tm - tb);                    // Eq. 5
  // Scenario 2 applies when N_m lies between the concurrencies.
  double n = (n_m > c_basic && n_m <= c_more) ? n_m : std::max(c_basic, n_l);
  return (int64_t)n;
}

// Default plan (measured on MI355X): below the model's switch point one
// 1024-thread workgroup; up to kAtomicMaxBytes the atomic-ticket variant;
// beyond, the relaunch variant with 256 threads x 4 loads of 16 bytes, two
// workgroups per CU (32 KiB in flight per CU) and nontemporal loads.
red_plan default_plan(int dtype, int64_t n, const DeviceInfo& dev) {
  red_plan p;
  const int64_t bytes = n * (dtype == RED_I32 || dtype == RED_F32 ? 4 : 2);
  p.flags = RED_FLAG_NONTEMPORAL;
  if (bytes < single_wg_switch_bytes()) {
    p.variant = RED_VARIANT_SINGLE;
    p.wg = 1024;
    p.ipt = 2;
    p.grid = 1;
    p.flags = 0;
    return p;
  }
  p.variant = bytes <= kAtomicMaxBytes ? RED_VARIANT_ATOMIC : RED_VARIANT_RELAUNCH;
  p.wg = 256;
  p.ipt = 4;
  p.grid = 2 * dev.cus;  // capped by the work at launch
  return p;
}

int reduce_max_coresident(int dtype, int acc, int ipt, bool nt, bool pipe, int wg, const DeviceInfo& dev,
                          int* n_wg) {
  int m = mode_of(dtype, acc);
  int ii = ipt_index(ipt);
  if (m < 0 || ii < 0) return set_error(RED_EINVAL, "bad dtype/ipt");
  int per_cu = 0;
  RED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, table().k[m][nt ? 1 : 0][pipe ? 1 : 0][ii].persistent,
                                                       wg, 0));
  *n_wg = per_cu * dev.cus;
  return RED_OK;
}

int reduce_launch(const ReduceLaunch& rl, const void* x, int64_t n, void* out, Workspace* ws,
                  hipStream_t s, const DeviceInfo& dev) {
  const int m = mode_of(rl.dtype, rl.acc);
  const bool is_int = rl.dtype == RED_I32;
  if (n == 0) {
    void* zargs[] = {&out};
    const void* fn = is_int ? reinterpret_cast<const void*>(&k_write_zero<long long>)
                            : reinterpret_cast<const void*>(&k_write_zero<double>);
    return launch(fn, 1, 64, zargs, s, false);
  }
  const int es = elem_size(rl.dtype);
  const int ve = 16 / es;
  ReduceArgs a;
  a.x = x;
  uintptr_t addr = reinterpret_cast<uintptr_t>(x);
  int64_t head = (int64_t)(((16 - (addr & 15)) & 15) / es);
  a.head = std::min<int64_t>(head, n);
  a.nvec = (n - a.head) / ve;
  a.tail = n - a.head - a.nvec * ve;
  a.partials = ws->partials;
  a.words = ws->words;
  a.out = out;
  a.spin_limit = watchdog_spins();
  a.bar_groups = 1;
  const bool xcd = (rl.plan.flags & RED_FLAG_XCD) != 0 && xcd_tree_fits(dev.nxcc);
  a.xcd_nxcc = xcd ? (unsigned)dev.nxcc : 0u;

  const red_plan& p = rl.plan;
  const int ii = ipt_index(p.ipt);
  const bool nt = (p.flags & RED_FLAG_NONTEMPORAL) != 0;
  const bool pipe = (p.flags & RED_FLAG_PIPELINE) != 0;
  const KernelSet& ks = table().k[m][nt ? 1 : 0][pipe ? 1 : 0][ii];
  // Grid: the requested size, else enough workgroups for the work, capped
  // at 4 per compute unit (and at the co-resident limit for the persistent
  // variant).
  const int64_t tile = (int64_t)p.wg * p.ipt;
  int64_t want = std::max<int64_t>(1, (a.nvec + tile - 1) / tile);
  int grid = (int)std::min<int64_t>(want, p.grid > 0 ? (int64_t)p.grid : 4LL * dev.cus);
  grid = std::max(1, std::min(grid, std::min(rl.max_grid, RED_MAX_GRID)));
  void* args[] = {&a};
  // The stream's kernel timer, unless the caller rules out its events.
  auto launch_k = [&](const void* fn, int g, bool coop) {
    return rl.timed ? launch_timed(fn, g, p.wg, args, s, coop) : launch(fn, g, p.wg, args, s, coop);
  };
  switch (p.variant) {
    case RED_VARIANT_RELAUNCH: {
      int rc = launch_k(ks.partials, grid, false);
      if (rc) return rc;
      // Up to 1024 partials: one wavefront (at most 16 loads per lane);
      // beyond: one 256-thread workgroup.
      const bool wave = grid <= 1024;
      void* part = ws->partials;
      void* fargs[] = {&part, &grid, &out};
      const void* fn = is_int ? (wave ? reinterpret_cast<const void*>(&k_final_wave<long long>)
                                      : reinterpret_cast<const void*>(&k_final<long long>))
                              : (wave ? reinterpret_cast<const void*>(&k_final_wave<double>)
                                      : reinterpret_cast<const void*>(&k_final<double>));
      return launch(fn, 1, wave ? kWave : kFinalWG, fargs, s, false);
    }
    case RED_VARIANT_SINGLE: {
      return launch_k(ks.single, 1, false);
    }
    case RED_VARIANT_ATOMIC: {
      return launch_k(ks.atomic, grid, false);
    }
    case RED_VARIANT_PERSISTENT: {
      int maxg = 0;
      int rc = reduce_max_coresident(rl.dtype, rl.acc, p.ipt, nt, pipe, p.wg, dev, &maxg);
      if (rc) return rc;
      if (p.grid > 0 && p.grid > maxg)
        return set_error(RED_EINVAL, "persistent plan: grid %d exceeds the %d co-resident workgroups",
                         p.grid, maxg);
      grid = std::min(grid, maxg);
      if (grid < 1) return set_error(RED_EINVAL, "persistent kernel cannot be resident");
      a.bar_groups = xcd ? (kBarrierXcd | (unsigned)dev.nxcc) : barrier_groups(grid);
      return launch_k(ks.persistent, grid, (p.flags & RED_FLAG_PLAIN_LAUNCH) == 0);
    }
  }
  return set_error(RED_EINVAL, "unknown variant %d", p.variant);
}

}  // namespace redsum
