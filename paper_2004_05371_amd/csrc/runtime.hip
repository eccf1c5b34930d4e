// C-ABI entry points of libredsum: validation, device and workspace
// management, plan table, autotuner, segmented-batch graph cache.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <hip/hip_ext.h>

#include "device_prims.h"
#include "internal.h"

namespace redsum {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string t_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(RED_EHIP, "%s failed: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ---------------------------------------------------------------------------
// Global state
// ---------------------------------------------------------------------------
namespace {

std::mutex g_mu;
std::map<int, DeviceInfo> g_dev;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

// Plan table: (kind, dtype, acc, bucket) -> plan.  kind 0 = red_sum,
// 1 = segmented (dtype = nseg bucket, acc = total-size bucket).
std::map<std::tuple<int, int, int, int>, red_plan> g_plans;

struct GraphKey {
  int dev;
  hipStream_t s;
  const void* x;
  const void* off;
  int64_t nseg;
  void* out;
  int variant, wg, ipt, grid, nt;
  auto tie() const { return std::tie(dev, s, x, off, nseg, out, variant, wg, ipt, grid, nt); }
  bool operator<(const GraphKey& o) const { return tie() < o.tie(); }
  bool operator==(const GraphKey& o) const { return tie() == o.tie(); }
};
struct GraphEntry {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
};
std::map<GraphKey, GraphEntry> g_graphs;
std::list<GraphKey> g_graph_lru;  // least recently used first
constexpr size_t kMaxGraphs = 64;
std::map<int, hipStream_t> g_capture_streams;  // per device, for building graphs
std::mutex g_capture_mu;                        // serializes captures

// The library's capture stream of device `dev` (non-blocking, default
// priority), created on first use.
int capture_stream(int dev, hipStream_t* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_capture_streams.find(dev);
  if (it != g_capture_streams.end()) {
    *out = it->second;
    return RED_OK;
  }
  hipStream_t cs = nullptr;
  RED_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  g_capture_streams[dev] = cs;
  *out = cs;
  return RED_OK;
}

int bucket(int64_t n) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;  // ceil(log2 n)
}

}  // namespace

unsigned watchdog_spins() {
  static unsigned v = [] {
    const char* e = getenv("REDSUM_WATCHDOG_SPINS");
    long long x = e ? atoll(e) : 0;
    if (x <= 0 || x > 0x7FFFFFFF) x = 1 << 22;
    return (unsigned)x;
  }();
  return v;
}

unsigned barrier_groups(int grid) {
  static int forced = [] {
    const char* e = getenv("REDSUM_BARRIER_GROUPS");
    int x = e ? atoi(e) : 0;
    return (x >= 1 && x <= kMaxBarrierGroups) ? x : 0;
  }();
  return forced ? (unsigned)forced : default_barrier_groups((unsigned)grid);
}

bool stream_capturing(hipStream_t s) {
  if (!s) return false;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

int ensure_device(const DeviceInfo** info) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return set_error(RED_ENODEV, "no HIP device is available");
  }
  int dev = 0;
  RED_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) {
    *info = &it->second;
    return RED_OK;
  }
  hipDeviceProp_t prop;
  RED_HIP(hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(RED_ENODEV, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
  DeviceInfo d;
  d.id = dev;
  d.cus = prop.multiProcessorCount;
  int wc = 0;
  if (hipDeviceGetAttribute(&wc, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wc <= 0) wc = 100000;
  d.wallclock_khz = wc;
  d.clock_khz = prop.clockRate;
  d.l2_bytes = prop.l2CacheSize;
  d.hbm_bytes = (int64_t)prop.totalGlobalMem;
  d.coop = prop.cooperativeLaunch != 0;
  d.lds_per_wg = (int64_t)prop.sharedMemPerBlock;
  int nx = 1;
  if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nx < 1) {
    (void)hipGetLastError();
    nx = 1;
  }
  d.nxcc = nx;
  auto r = g_dev.emplace(dev, d);
  *info = &r.first->second;
  return RED_OK;
}

int get_workspace(hipStream_t s, Workspace** out) {
  int dev = 0;
  RED_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) {
    *out = &it->second;
    return RED_OK;
  }
  if (stream_capturing(s))
    return set_error(RED_EINVAL,
                     "the first call on a stream allocates its workspace and cannot be captured; "
                     "call once before capturing");
  Workspace w;
  hipError_t e = hipMalloc(&w.base, kWorkspaceBytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(RED_ENOMEM, "workspace allocation of %zu bytes failed: %s", kWorkspaceBytes,
                     hipGetErrorString(e));
  }
  e = hipMemset(w.base, 0, kWorkspaceBytes);
  if (e != hipSuccess) {
    (void)hipFree(w.base);
    return hip_fail(e, "hipMemset(workspace)");
  }
  char* p = static_cast<char*>(w.base);
  w.words = reinterpret_cast<BarrierWords*>(p);
  p += kWordsBytes;
  w.partials = p;
  p += kPartialBytes;
  w.carry_in = reinterpret_cast<SegCarry*>(p);
  p += kCarryBytes;
  w.carry_out = reinterpret_cast<SegCarry*>(p);
  p += kCarryBytes;
  w.seg_tickets = reinterpret_cast<unsigned*>(p);
  p += kTicketBytes;
  w.sink = reinterpret_cast<unsigned*>(p);
  p += kSinkBytes;
  w.stamps = reinterpret_cast<long long*>(p);
  auto r = g_ws.emplace(key, w);
  *out = &r.first->second;
  return RED_OK;
}

// ---------------------------------------------------------------------------
// Dominant-kernel timer
// ---------------------------------------------------------------------------
namespace {
struct KernelTimer {
  int period = 0;        // 0 = off; k = time every k-th launch
  uint64_t launches = 0; // launches seen while on
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;
};
std::map<std::pair<int, hipStream_t>, KernelTimer> g_timers;
}  // namespace

namespace {
// A slot of the stream's timer for this launch (every period-th launch
// while the timer is on), or -1; with `record`, its start event is
// recorded on the stream now.
int timer_acquire(hipStream_t s, bool record, hipEvent_t* start = nullptr, hipEvent_t* stop = nullptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_timers.find(std::make_pair(dev, s));
  if (it == g_timers.end() || it->second.period <= 0) return -1;
  if (stream_capturing(s)) return -1;
  KernelTimer& t = it->second;
  if (t.launches++ % (uint64_t)t.period != 0) return -1;
  if (t.used == t.ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return -1;
    if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    t.ev.emplace_back(a, b);
  }
  const int slot = (int)t.used++;
  if (record && hipEventRecord(t.ev[slot].first, s) != hipSuccess) {
    --t.used;
    return -1;
  }
  if (start) *start = t.ev[slot].first;
  if (stop) *stop = t.ev[slot].second;
  return slot;
}
}  // namespace

int timer_begin(hipStream_t s) { return timer_acquire(s, true); }

void timer_end(hipStream_t s, int slot) {
  if (slot < 0) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_timers.find(std::make_pair(dev, s));
  if (it == g_timers.end() || (size_t)slot >= it->second.ev.size()) return;
  (void)hipEventRecord(it->second.ev[slot].second, s);
}

int launch_timed(const void* fn, int grid, int block, void** args, hipStream_t s, bool cooperative,
                 size_t lds_bytes) {
  if (cooperative) {
    const int slot = timer_begin(s);
    const int rc = launch(fn, grid, block, args, s, true, lds_bytes);
    timer_end(s, slot);
    return rc;
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (timer_acquire(s, false, &a, &b) < 0) return launch(fn, grid, block, args, s, false, lds_bytes);
  // The events ride on the kernel's own dispatch: they take its start and
  // end, as a kernel trace reports them.
  const hipError_t e = hipExtLaunchKernel(fn, dim3(grid), dim3(block), args, lds_bytes, s, a, b, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_fail(e, "hipExtLaunchKernel");
  }
  return RED_OK;
}

int launch(const void* fn, int grid, int block, void** args, hipStream_t s, bool cooperative, size_t lds_bytes) {
  hipError_t e;
  if (cooperative)
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds_bytes, s);
  else
    e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds_bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (e == hipErrorCooperativeLaunchTooLarge)
      return set_error(RED_EINVAL, "cooperative launch of %d x %d is too large", grid, block);
    return hip_fail(e, cooperative ? "hipLaunchCooperativeKernel" : "hipLaunchKernel");
  }
  return RED_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the no-allocation entry point: barrier words, then one partial
// slot per workgroup, in one static device array per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = kWordsBytes + (size_t)RED_NOALLOC_MAX_GRID * 8;
static_assert(sizeof(BarrierWords) <= kWordsBytes, "barrier words fit their region");

}  // namespace redsum

// The array itself.  In host code its name is only a stand-in for the
// device symbol: every host use goes through the device address that
// scratch_address() looked up for the current device.
static __device__ __align__(256) unsigned char scratch[redsum::kScratchBytes];

namespace redsum {
namespace {

std::map<int, void*> g_scratch;  // device -> address of `scratch` on it

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_address(void** out) {
  int dev = 0;
  RED_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
      *out = it->second;
      return RED_OK;
    }
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return set_error(RED_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                     hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_scratch[dev] = ptr;
  *out = ptr;
  return RED_OK;
}

// Zeroes the first 8 bytes (the counter or tally, and the fall-back
// request of the generation line) of each of n lines of barrier words (a
// kernel, not a memset, so it also records as an ordinary kernel node
// under capture).
__global__ void k_zero_lines(Line* lines, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) *reinterpret_cast<unsigned long long*>(&lines[i].v) = 0ull;
}

}  // namespace
}  // namespace redsum

using namespace redsum;

namespace {

int check_dtype(int dtype) {
  if (dtype < RED_I32 || dtype > RED_BF16) return set_error(RED_EINVAL, "unknown dtype %d", dtype);
  return RED_OK;
}

int esize(int dtype) { return dtype == RED_I32 || dtype == RED_F32 ? 4 : 2; }

int validate_sum_args(int dtype, const void* x, int64_t n, void* out, const red_opts* opts) {
  int rc = check_dtype(dtype);
  if (rc) return rc;
  if (n < 0 || n >= ((int64_t)1 << 40)) return set_error(RED_EINVAL, "n = %lld out of range", (long long)n);
  if (!x && n > 0) return set_error(RED_EINVAL, "x is NULL");
  if (!out) return set_error(RED_EINVAL, "out is NULL");
  if (reinterpret_cast<uintptr_t>(x) % esize(dtype))
    return set_error(RED_EINVAL, "x is not aligned to its element size");
  if (reinterpret_cast<uintptr_t>(out) % 8) return set_error(RED_EINVAL, "out is not 8-byte aligned");
  if (opts) {
    if (opts->acc != RED_ACC_COMPENSATED && opts->acc != RED_ACC_PLAIN)
      return set_error(RED_EINVAL, "unknown accumulation %d", opts->acc);
    if (opts->flags & ~(RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH | RED_FLAG_PIPELINE | RED_FLAG_XCD))
      return set_error(RED_EINVAL, "unknown flags 0x%x", opts->flags);
    if (opts->plan.variant != RED_VARIANT_AUTO) {
      red_plan p = opts->plan;
      if (p.wg == 0) p.wg = 512;
      if (p.ipt == 0) p.ipt = 4;
      return validate_plan(p);
    }
  }
  return RED_OK;
}

// An explicit plan takes the default workgroup size / items per thread for
// fields left at 0.
red_plan complete_plan(red_plan p, const red_plan& dflt) {
  if (p.wg == 0) p.wg = dflt.wg;
  if (p.ipt == 0) p.ipt = dflt.ipt;
  return p;
}

red_plan lookup_plan(int dtype, int acc, int64_t n, const DeviceInfo& dev) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(std::make_tuple(0, dtype, dtype == RED_I32 ? 0 : acc, bucket(n)));
    if (it != g_plans.end()) return it->second;
  }
  return default_plan(dtype, n, dev);
}


int validate_seg_args(const float* x, const int64_t* offsets, int64_t nseg, double* out, const red_opts* opts) {
  if (nseg < 0 || nseg >= ((int64_t)1 << 31)) return set_error(RED_EINVAL, "nseg out of range");
  if (!offsets) return set_error(RED_EINVAL, "offsets is NULL");
  if (nseg > 0 && (!x || !out)) return set_error(RED_EINVAL, "x or out is NULL");
  if (reinterpret_cast<uintptr_t>(x) % 4) return set_error(RED_EINVAL, "x is not 4-byte aligned");
  if (reinterpret_cast<uintptr_t>(offsets) % 8) return set_error(RED_EINVAL, "offsets is not 8-byte aligned");
  if (reinterpret_cast<uintptr_t>(out) % 8) return set_error(RED_EINVAL, "out is not 8-byte aligned");
  if (opts) {
    const int forms = RED_FLAG_SEG_WORKGROUP | RED_FLAG_SEG_PIECES | RED_FLAG_SEG_RUNS;
    if (opts->flags & ~(RED_FLAG_NONTEMPORAL | RED_FLAG_NO_GRAPH | RED_FLAG_PLAIN_LAUNCH | RED_FLAG_XCD | forms))
      return set_error(RED_EINVAL, "unknown flags 0x%x", opts->flags);
    const int f = opts->flags & forms;
    if (f & (f - 1)) return set_error(RED_EINVAL, "segmented: at most one of the form flags");
    if (opts->plan.variant != RED_VARIANT_AUTO) {
      red_plan p = opts->plan;
      if (p.wg == 0) p.wg = 512;
      if (p.ipt == 0) p.ipt = 4;
      int rc = validate_plan(p);
      if (rc) return rc;
      if (opts->plan.variant != RED_VARIANT_RELAUNCH && opts->plan.variant != RED_VARIANT_ATOMIC &&
          opts->plan.variant != RED_VARIANT_PERSISTENT)
        return set_error(RED_EINVAL, "segmented: variant must be RELAUNCH, ATOMIC or PERSISTENT");
      if (p.wg > 512) return set_error(RED_EINVAL, "segmented: at most 512 threads per workgroup");
    }
  }
  return RED_OK;
}

// Median of a small vector.
double median(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  const size_t n = v.size();
  return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

}  // namespace

extern "C" {

const char* red_last_error(void) { return t_err.c_str(); }

int red_init(int device) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return set_error(RED_ENODEV, "no HIP device is available");
  }
  if (device < 0 || device >= count) return set_error(RED_ENODEV, "device %d does not exist", device);
  RED_HIP(hipSetDevice(device));
  const DeviceInfo* d;
  int rc = ensure_device(&d);
  if (rc) return rc;
  void* sp = nullptr;
  if ((rc = scratch_address(&sp))) return rc;
  Workspace* ws;
  return get_workspace(nullptr, &ws);
}

void red_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  // A process that never reached a device has nothing to release (and
  // makes no HIP call here).
  if (g_dev.empty() && g_ws.empty() && g_graphs.empty() && g_timers.empty() && g_capture_streams.empty())
    return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  // Nothing of the library may still run: graphs, events and workspaces go
  // below.
  for (auto& kv : g_dev) {
    (void)hipSetDevice(kv.first);
    (void)hipDeviceSynchronize();
  }
  for (auto& kv : g_graphs) {
    (void)hipSetDevice(kv.first.dev);
    if (kv.second.e) (void)hipGraphExecDestroy(kv.second.e);
    if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
  }
  g_graphs.clear();
  g_graph_lru.clear();
  for (auto& kv : g_timers) {
    (void)hipSetDevice(kv.first.first);
    for (auto& ab : kv.second.ev) {
      (void)hipEventDestroy(ab.first);
      (void)hipEventDestroy(ab.second);
    }
  }
  g_timers.clear();
  for (auto& kv : g_ws) {
    (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second.base);
  }
  g_ws.clear();
  for (auto& kv : g_capture_streams) {
    (void)hipSetDevice(kv.first);
    (void)hipStreamDestroy(kv.second);
  }
  g_capture_streams.clear();
  // Device records are kept: they hold no HIP object.
  (void)hipSetDevice(cur);
  (void)hipGetLastError();
}

int red_check_error(void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  Workspace* ws;
  if ((rc = get_workspace(s, &ws))) return rc;
  RED_HIP(hipStreamSynchronize(s));
  std::vector<BarrierWords> hw_buf(1);  // about 73 KB: on the heap
  BarrierWords& hw = hw_buf[0];
  RED_HIP(hipMemcpy(&hw, ws->words, sizeof(hw), hipMemcpyDeviceToHost));
  const unsigned err = hw.err.v;
  // Every completed launch leaves its arrival counters at zero; a counter
  // left over means some workgroups never completed an arrival.
  bool stale = hw.count.v || hw.count.pad[0] || hw.ticket.v || hw.ticket.pad[0] || hw.fb.v;
  for (const Line& g : hw.group) stale = stale || g.v || g.pad[0];
  for (const Line& g : hw.cls) stale = stale || g.v || g.pad[0];
  for (const Line& g : hw.node) stale = stale || g.v || g.pad[0];
  if (!err && !stale) return RED_OK;
  // Clear the error and every barrier word (the barrier was abandoned).
  RED_HIP(hipMemset(ws->words, 0, kWordsBytes));
  RED_HIP(hipMemset(ws->seg_tickets, 0, kTicketBytes));
  if (!err)
    return set_error(RED_ENOTSUP, "arrival counters were left incomplete (an abandoned barrier or ticket)");
  return set_error(RED_ETIMEOUT, "a grid-barrier watchdog fired on this stream");
}

int red_sum_ex(int dtype, const void* x, int64_t n, void* out, void* stream, const red_opts* opts) {
  int rc = validate_sum_args(dtype, x, n, out, opts);
  if (rc) return rc;
  const DeviceInfo* dev;
  if ((rc = ensure_device(&dev))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace* ws;
  if ((rc = get_workspace(s, &ws))) return rc;
  ReduceLaunch rl;
  rl.dtype = dtype;
  rl.acc = opts ? opts->acc : RED_ACC_COMPENSATED;
  rl.plan = (opts && opts->plan.variant != RED_VARIANT_AUTO)
                ? complete_plan(opts->plan, default_plan(dtype, n, *dev))
                : lookup_plan(dtype, rl.acc, n, *dev);
  if (opts) rl.plan.flags |= opts->flags & (RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH | RED_FLAG_PIPELINE | RED_FLAG_XCD);
  return reduce_launch(rl, x, n, out, ws, s, *dev);
}

int red_sum(int dtype, const void* x, int64_t n, void* out, void* stream) {
  return red_sum_ex(dtype, x, n, out, stream, nullptr);
}

int red_sum_noalloc(int dtype, const void* x, int64_t n, void* out, void* stream, const red_opts* opts) {
  int rc = validate_sum_args(dtype, x, n, out, opts);
  if (rc) return rc;
  if (opts && opts->plan.variant != RED_VARIANT_AUTO && opts->plan.grid > RED_NOALLOC_MAX_GRID)
    return set_error(RED_EINVAL, "red_sum_noalloc: grid %d exceeds the %d workgroups its scratch holds",
                     opts->plan.grid, RED_NOALLOC_MAX_GRID);
  const DeviceInfo* dev;
  if ((rc = ensure_device(&dev))) return rc;
  void* sp = nullptr;
  if ((rc = scratch_address(&sp))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws;  // views into the scratch; nothing else of a workspace is used
  ws.words = reinterpret_cast<BarrierWords*>(sp);
  ws.partials = static_cast<char*>(sp) + kWordsBytes;
  ReduceLaunch rl;
  rl.dtype = dtype;
  rl.acc = opts ? opts->acc : RED_ACC_COMPENSATED;
  rl.plan = (opts && opts->plan.variant != RED_VARIANT_AUTO)
                ? complete_plan(opts->plan, default_plan(dtype, n, *dev))
                : lookup_plan(dtype, rl.acc, n, *dev);
  if (opts) rl.plan.flags |= opts->flags & (RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH | RED_FLAG_PIPELINE | RED_FLAG_XCD);
  rl.timed = false;
  rl.max_grid = RED_NOALLOC_MAX_GRID;
  if (n > 0 && (rl.plan.variant == RED_VARIANT_ATOMIC || rl.plan.variant == RED_VARIANT_PERSISTENT)) {
    // The ticket, counters and accumulator start at zero (the array keeps
    // whatever the last call, or an abandoned barrier, left).
    Line* lines = static_cast<Line*>(sp);
    int nl = (int)(sizeof(BarrierWords) / sizeof(Line));
    void* zargs[] = {&lines, &nl};
    if ((rc = launch(reinterpret_cast<const void*>(&k_zero_lines), 1, 256, zargs, s, false))) return rc;
  }
  return reduce_launch(rl, x, n, out, &ws, s, *dev);
}

int red_set_plan(int dtype, int acc, int64_t n, const red_plan* plan) {
  int rc = check_dtype(dtype);
  if (rc) return rc;
  if (acc != RED_ACC_COMPENSATED && acc != RED_ACC_PLAIN) return set_error(RED_EINVAL, "bad acc");
  if (!plan || n < 0) return set_error(RED_EINVAL, "bad plan or n");
  if ((rc = validate_plan(*plan))) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans[std::make_tuple(0, dtype, dtype == RED_I32 ? 0 : acc, bucket(n))] = *plan;
  return RED_OK;
}

int red_get_plan(int dtype, int acc, int64_t n, red_plan* plan) {
  int rc = check_dtype(dtype);
  if (rc) return rc;
  if (acc != RED_ACC_COMPENSATED && acc != RED_ACC_PLAIN) return set_error(RED_EINVAL, "bad acc");
  if (!plan || n < 0) return set_error(RED_EINVAL, "bad plan or n");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(std::make_tuple(0, dtype, dtype == RED_I32 ? 0 : acc, bucket(n)));
    if (it != g_plans.end()) {
      *plan = it->second;
      return RED_OK;
    }
  }
  const DeviceInfo* dev;
  if ((rc = ensure_device(&dev))) {
    // Without a device the default plan is still defined (grid automatic).
    DeviceInfo none;
    none.cus = 256;
    *plan = default_plan(dtype, n, none);
    return RED_OK;
  }
  *plan = default_plan(dtype, n, *dev);
  return RED_OK;
}

int red_max_coresident(int wg_size, int32_t* n_wg) {
  if (!n_wg || wg_size < 64 || wg_size > 1024 || wg_size % 64) return set_error(RED_EINVAL, "bad arguments");
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  int n = 0;
  if ((rc = reduce_max_coresident(RED_F32, RED_ACC_COMPENSATED, 4, false, false, wg_size, *dev, &n))) return rc;
  *n_wg = n;
  return RED_OK;
}

int red_max_coresident_segmented(int ipt, int wg_size, int32_t* n_wg) {
  if (!n_wg || wg_size < 64 || wg_size > 512 || wg_size % 64) return set_error(RED_EINVAL, "bad arguments");
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  int n = 0;
  if ((rc = seg_max_coresident(ipt, wg_size, *dev, &n))) return rc;
  *n_wg = n;
  return RED_OK;
}

int red_device_info(int32_t* cus, int64_t* wallclock_khz, int64_t* clock_khz, int64_t* l2_bytes,
                    int64_t* hbm_bytes, int32_t* nxcc) {
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  if (nxcc) *nxcc = dev->nxcc;
  if (cus) *cus = dev->cus;
  if (wallclock_khz) *wallclock_khz = dev->wallclock_khz;
  if (clock_khz) *clock_khz = dev->clock_khz;
  if (l2_bytes) *l2_bytes = dev->l2_bytes;
  if (hbm_bytes) *hbm_bytes = dev->hbm_bytes;
  return RED_OK;
}

// Times `plan` on the caller's data: 3 warm-up calls, then the median of 10
// calls bracketed by events.
static int time_plan(int dtype, int acc, const red_plan& plan, const void* x, int64_t n, void* out,
                     hipStream_t s, double* us) {
  red_opts o;
  memset(&o, 0, sizeof o);
  o.plan = plan;
  o.acc = acc;
  hipEvent_t a, b;
  RED_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
  RED_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
  // Samples of k calls back to back between one event pair: the rate of a
  // stream of calls, as a caller's loop sees it (one call per sample would
  // time an isolated call's launch from an idle stream, which decides the
  // ranking of small inputs).  k makes a sample last about 200 us (1 to 32
  // calls, from the first warm sample's time); the median of 7 samples
  // after the warm ones, per call.
  std::vector<double> t;
  int rc = RED_OK;
  int k = 1;
  for (int i = 0; i < 10 && rc == RED_OK; ++i) {
    if (hipEventRecord(a, s) != hipSuccess) rc = set_error(RED_EHIP, "hipEventRecord");
    for (int j = 0; j < k && !rc; ++j) rc = red_sum_ex(dtype, x, n, out, s, &o);
    if (!rc && hipEventRecord(b, s) != hipSuccess) rc = set_error(RED_EHIP, "hipEventRecord");
    if (!rc && hipEventSynchronize(b) != hipSuccess) rc = set_error(RED_EHIP, "hipEventSynchronize");
    float ms = 0;
    if (!rc && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = set_error(RED_EHIP, "hipEventElapsedTime");
    if (rc) break;
    const double per = ms * 1e3 / k;
    if (i == 1) k = (int)std::min(32.0, std::max(1.0, 200.0 / std::max(per, 1e-3)));
    if (i >= 3) t.push_back(per);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  *us = median(t);
  return RED_OK;
}

int red_autotune_search(int dtype, int64_t n, int cus, int nxcc, int allow_xcd, int budget, red_cost_fn cost,
                        void* ctx, red_plan* best, double* best_us) {
  int rc = check_dtype(dtype);
  if (rc) return rc;
  if (n < 0 || cus < 1 || nxcc < 1 || !cost) return set_error(RED_EINVAL, "bad search arguments");
  DeviceInfo d;
  d.cus = cus;
  d.nxcc = nxcc;
  // Search: (1) nontemporal hint on the default shape; (2) every
  // (pipelined?, wg, ipt, grid) of the relaunch variant with that hint;
  // (3) one workgroup for small inputs; (4) the other synchronization
  // variants on the best shape.  `budget` caps the number of timed
  // candidates (0 = no cap).  The grid candidates start at one workgroup
  // per CU; the in-flight bytes per CU (wg * ipt * 16 * grid / CUs) is what
  // the shapes trade off.  The cost function may lower a candidate's grid
  // (co-residency of the persistent variant); the plan kept is the one it
  // timed.  The first candidate of the lowest cost wins.
  int timed = 0;
  red_plan cur = default_plan(dtype, n, d);
  double cur_us = 1e300;
  auto consider = [&](red_plan p) -> int {
    if (budget > 0 && timed >= budget) return RED_OK;
    const double us = cost(&p, ctx);
    ++timed;
    if (us < 0) return (int)us;  // the cost function's status
    if (us < cur_us) {
      cur_us = us;
      cur = p;
    }
    return RED_OK;
  };
  {
    red_plan p = cur;
    p.flags &= ~RED_FLAG_NONTEMPORAL;
    if ((rc = consider(p))) return rc;
    p.flags |= RED_FLAG_NONTEMPORAL;
    if ((rc = consider(p))) return rc;
  }
  const int nt_flag = cur.flags & RED_FLAG_NONTEMPORAL;
  const int64_t nvec = n / (16 / esize(dtype));
  const int mults[] = {1, 2, 3, 4, 6, 8, 12, 16};
  for (int pipe : {0, RED_FLAG_PIPELINE})
    for (int wg : {128, 256, 512, 1024})
      for (int ipt : {1, 2, 4, 8}) {
        const int64_t tile = (int64_t)wg * ipt;
        const int64_t want = std::max<int64_t>(1, (nvec + tile - 1) / tile);
        for (int m : mults) {
          const int64_t g = std::min<int64_t>({(int64_t)m * cus, want, (int64_t)RED_MAX_GRID});
          if ((rc = consider(red_plan{RED_VARIANT_RELAUNCH, wg, ipt, (int)g, nt_flag | pipe}))) return rc;
          if (g == want) break;
        }
      }
  // One workgroup (no device-wide synchronization) for small inputs.
  if (n * esize(dtype) <= 64 * single_wg_switch_bytes())
    for (int wg : {256, 512, 1024})
      for (int ipt : {1, 2, 4})
        for (int pipe : {0, RED_FLAG_PIPELINE})
          if ((rc = consider(red_plan{RED_VARIANT_SINGLE, wg, ipt, 1, nt_flag | pipe}))) return rc;
  const red_plan shape = cur;
  // XCD-aggregated publication relies on the dispatch order (checked in the
  // kernels); it is a candidate only when the caller allows it.
  const bool try_xcd = nxcc > 1 && allow_xcd;
  for (int v : {RED_VARIANT_ATOMIC, RED_VARIANT_PERSISTENT})
    for (int xcd : {0, try_xcd ? RED_FLAG_XCD : 0}) {
      if (shape.variant == RED_VARIANT_SINGLE) break;
      red_plan p = shape;
      p.variant = v;
      p.flags |= xcd;
      if ((rc = consider(p))) return rc;
      if (v == RED_VARIANT_PERSISTENT) {
        p.flags |= RED_FLAG_PLAIN_LAUNCH;
        if ((rc = consider(p))) return rc;
      }
      if (!xcd && !try_xcd) break;
    }
  if (timed == 0) return set_error(RED_EINVAL, "no candidate timed");
  if (best) *best = cur;
  if (best_us) *best_us = cur_us;
  return RED_OK;
}

namespace {
// Cost of a candidate on the GPU: the median of 7 timed samples of calls on the
// caller's data (a persistent candidate's grid capped at co-residency).
struct GpuCost {
  int dtype, acc;
  const void* x;
  int64_t n;
  void* out;
  hipStream_t s;
  const DeviceInfo* dev;
};
double gpu_cost(red_plan* p, void* c) {
  const GpuCost& k = *static_cast<const GpuCost*>(c);
  if (p->variant == RED_VARIANT_PERSISTENT) {
    int maxg = 0;
    int r = reduce_max_coresident(k.dtype, k.acc, p->ipt, (p->flags & RED_FLAG_NONTEMPORAL) != 0,
                                  (p->flags & RED_FLAG_PIPELINE) != 0, p->wg, *k.dev, &maxg);
    if (r) return (double)r;
    if (p->grid == 0 || p->grid > maxg) p->grid = maxg;
  }
  double us = 0;
  const int r = time_plan(k.dtype, k.acc, *p, k.x, k.n, k.out, k.s, &us);
  return r ? (double)r : us;
}
}  // namespace

int red_autotune(int dtype, int acc, const void* x, int64_t n, void* out, void* stream, int budget,
                 red_plan* best, double* best_us) {
  red_opts vo;
  memset(&vo, 0, sizeof vo);
  vo.acc = acc;
  int rc = validate_sum_args(dtype, x, n, out, &vo);
  if (rc) return rc;
  const DeviceInfo* dev;
  if ((rc = ensure_device(&dev))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(RED_EINVAL, "autotuning cannot run inside stream capture");
  const char* allow = getenv("REDSUM_ALLOW_XCD");
  GpuCost ctx{dtype, acc, x, n, out, s, dev};
  red_plan cur;
  double cur_us = 0;
  if ((rc = red_autotune_search(dtype, n, dev->cus, dev->nxcc, allow && atoi(allow) == 1, budget, gpu_cost, &ctx,
                                &cur, &cur_us)))
    return rc;
  // Finals (unbudgeted searches): the search keeps the lowest of several
  // hundred single timings, which favours a lucky one, and times the other
  // synchronization variants once each on the best shape.  The best shape
  // under each variant (relaunch, atomic ticket, persistent plain launch)
  // is timed again in interleaved rounds; the lowest median wins.
  if (budget == 0 && cur.variant != RED_VARIANT_SINGLE) {
    constexpr int kRounds = 5;
    const int keep = cur.flags & (RED_FLAG_NONTEMPORAL | RED_FLAG_PIPELINE | RED_FLAG_XCD);
    red_plan cand[3] = {cur, cur, cur};
    cand[0].variant = RED_VARIANT_RELAUNCH;
    cand[0].flags = keep & ~RED_FLAG_XCD;
    cand[1].variant = RED_VARIANT_ATOMIC;
    cand[1].flags = keep;
    cand[2].variant = RED_VARIANT_PERSISTENT;
    cand[2].flags = keep | RED_FLAG_PLAIN_LAUNCH;
    std::vector<double> t[3];
    for (int r = 0; r < kRounds; ++r)
      for (int k = 0; k < 3; ++k) {
        const double us = gpu_cost(&cand[k], &ctx);
        if (us < 0) return (int)us;
        t[k].push_back(us);
      }
    int bk = 0;
    for (int k = 1; k < 3; ++k)
      if (median(t[k]) < median(t[bk])) bk = k;
    cur = cand[bk];
    cur_us = median(t[bk]);
  }
  if ((rc = red_set_plan(dtype, acc, n, &cur))) return rc;
  if (best) *best = cur;
  if (best_us) *best_us = cur_us;
  return RED_OK;
}

// ---------------------------------------------------------------------------
// Segmented batches
// ---------------------------------------------------------------------------
static int seg_direct(const SegLaunch& sl, const float* x, const int64_t* offsets, int64_t nseg, double* out,
                      Workspace* ws, hipStream_t s, const DeviceInfo& dev) {
  return seg_launch(sl, x, offsets, nseg, out, ws, s, dev);
}

int stencil_jacobi_1d(float* u, float* scratch, int64_t n, int32_t steps, float r, int32_t steps_per_sync,
                      void* stream, const red_opts* opts) {
  if (n < 0 || n >= ((int64_t)1 << 40)) return set_error(RED_EINVAL, "n out of range");
  if (steps < 0) return set_error(RED_EINVAL, "steps must be >= 0");
  if (steps_per_sync < 0) return set_error(RED_EINVAL, "steps_per_sync must be >= 0");
  if (n > 0 && (!u || !scratch)) return set_error(RED_EINVAL, "u or scratch is NULL");
  if (reinterpret_cast<uintptr_t>(u) % 4 || reinterpret_cast<uintptr_t>(scratch) % 4)
    return set_error(RED_EINVAL, "u and scratch must be 4-byte aligned");
  if (n > 0) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(u), b0 = reinterpret_cast<uintptr_t>(scratch);
    const uintptr_t bytes = (uintptr_t)n * 4;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return set_error(RED_EINVAL, "u and scratch overlap");
  }
  red_plan p{RED_VARIANT_AUTO, 0, 1, 0, 0};  // wg 0: chosen by stencil_launch
  if (opts) {
    if (opts->flags & ~(RED_FLAG_PLAIN_LAUNCH | RED_FLAG_XCD))
      return set_error(RED_EINVAL, "unknown flags 0x%x", opts->flags);
    const red_plan& q = opts->plan;
    if (q.variant != RED_VARIANT_AUTO && q.variant != RED_VARIANT_RELAUNCH && q.variant != RED_VARIANT_PERSISTENT)
      return set_error(RED_EINVAL, "stencil: variant must be AUTO, RELAUNCH or PERSISTENT");
    if (q.wg != 0 && (q.wg < 64 || q.wg > 1024 || q.wg % 64)) return set_error(RED_EINVAL, "bad wg %d", q.wg);
    if (q.grid < 0 || q.grid > RED_MAX_GRID) return set_error(RED_EINVAL, "bad grid %d", q.grid);
    if (q.flags & ~(RED_FLAG_PLAIN_LAUNCH | RED_FLAG_XCD)) return set_error(RED_EINVAL, "bad plan flags");
    p.variant = q.variant;
    if (q.wg) p.wg = q.wg;
    p.grid = q.grid;
    p.flags = q.flags | opts->flags;
  }
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  if (n < 3 || steps == 0) return RED_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace* ws;
  if ((rc = get_workspace(s, &ws))) return rc;
  return stencil_launch(u, scratch, n, steps, r, steps_per_sync, p, ws, s, *dev);
}

int red_sum_segmented_ex(const float* x, const int64_t* offsets, int64_t nseg, double* out, void* stream,
                         const red_opts* opts) {
  int rc = validate_seg_args(x, offsets, nseg, out, opts);
  if (rc) return rc;
  const DeviceInfo* dev;
  if ((rc = ensure_device(&dev))) return rc;
  if (nseg == 0) return RED_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace* ws;
  if ((rc = get_workspace(s, &ws))) return rc;
  SegLaunch sl;
  const bool no_graph = opts ? (opts->flags & RED_FLAG_NO_GRAPH) != 0 : false;
  if (opts && opts->plan.variant != RED_VARIANT_AUTO) {
    sl.plan = complete_plan(opts->plan, default_seg_plan(nseg, *dev));
  } else {
    sl.plan = default_seg_plan(nseg, *dev);
    std::lock_guard<std::mutex> lk(g_mu);
    // Installed plans are keyed by the nseg bucket only on this path (the
    // total size lives on the device).
    auto it = g_plans.find(std::make_tuple(1, bucket(nseg), 0, 0));
    if (it != g_plans.end()) sl.plan = it->second;
  }
  if (opts)
    sl.plan.flags |= opts->flags & (RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH | RED_FLAG_XCD |
                                    RED_FLAG_SEG_WORKGROUP | RED_FLAG_SEG_PIECES | RED_FLAG_SEG_RUNS);
  if ((sl.plan.flags & RED_FLAG_SEG_RUNS) && sl.plan.ipt > 4)
    return set_error(RED_EINVAL, "segmented: the reduce-by-key form takes at most 4 loads per thread");
  // Cooperative launches, the null stream and a caller's own capture
  // launch directly; otherwise the launch is replayed from a cached graph.
  // The persistent (grid-barrier) form goes into the graph too when it is
  // launched as an ordinary, occupancy-capped grid: one persistent kernel
  // per replay.
  const bool coop = sl.plan.variant == RED_VARIANT_PERSISTENT && !(sl.plan.flags & RED_FLAG_PLAIN_LAUNCH);
  if (no_graph || !s || coop || stream_capturing(s)) return seg_direct(sl, x, offsets, nseg, out, ws, s, *dev);
  GraphKey key{dev->id, s, x, offsets, nseg, out, sl.plan.variant, sl.plan.wg, sl.plan.ipt, sl.plan.grid,
               sl.plan.flags};
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
      exec = it->second.e;
      // most recently used at the back
      g_graph_lru.remove(key);
      g_graph_lru.push_back(key);
    }
  }
  if (!exec) {
    // Capture the one launch into a graph on the library's own capture
    // stream (the caller's stream is never put into capture mode); the
    // kernels use the workspace of the caller's stream.
    hipStream_t cs = nullptr;
    if ((rc = capture_stream(dev->id, &cs))) return rc;
    std::lock_guard<std::mutex> capture_lock(g_capture_mu);  // one capture at a time on cs
    RED_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    rc = seg_launch(sl, x, offsets, nseg, out, ws, cs, *dev);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "hipGraphInstantiate");
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_graphs.size() >= kMaxGraphs && !g_graph_lru.empty()) {
      auto old = g_graphs.find(g_graph_lru.front());
      if (old != g_graphs.end()) {
        // A replay of the evicted graph may still run on its stream.
        (void)hipStreamSynchronize(old->first.s);
        (void)hipGraphExecDestroy(old->second.e);
        (void)hipGraphDestroy(old->second.g);
        g_graphs.erase(old);
      }
      g_graph_lru.pop_front();
    }
    g_graphs[key] = GraphEntry{g, exec};
    g_graph_lru.push_back(key);
  }
  RED_HIP(hipGraphLaunch(exec, s));
  return RED_OK;
}

int red_kernel_timer(void* stream, int enable) {
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_mu);
  if (enable < 0) return set_error(RED_EINVAL, "enable must be >= 0");
  KernelTimer& t = g_timers[std::make_pair(dev->id, s)];
  t.period = enable;
  t.launches = 0;
  t.used = 0;
  return RED_OK;
}

int red_kernel_timer_read(void* stream, double* mean_us, double* min_us, int64_t* count) {
  const DeviceInfo* dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RED_HIP(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_timers.find(std::make_pair(dev->id, s));
  double sum = 0, mn = 1e300;
  int64_t n = 0;
  if (it != g_timers.end()) {
    KernelTimer& t = it->second;
    for (size_t i = 0; i < t.used; ++i) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, t.ev[i].first, t.ev[i].second) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      sum += ms * 1e3;
      mn = std::min(mn, (double)ms * 1e3);
      ++n;
    }
    t.used = 0;
  }
  if (mean_us) *mean_us = n ? sum / n : 0.0;
  if (min_us) *min_us = n ? mn : 0.0;
  if (count) *count = n;
  return RED_OK;
}

int red_set_segmented_plan(int64_t nseg, const red_plan* plan) {
  if (!plan || nseg < 0) return set_error(RED_EINVAL, "bad plan or nseg");
  int rc = validate_plan(*plan);
  if (rc) return rc;
  if (plan->variant != RED_VARIANT_RELAUNCH && plan->variant != RED_VARIANT_ATOMIC &&
      plan->variant != RED_VARIANT_PERSISTENT)
    return set_error(RED_EINVAL, "segmented: variant must be RELAUNCH, ATOMIC or PERSISTENT");
  if (plan->wg > 512) return set_error(RED_EINVAL, "segmented: at most 512 threads per workgroup");
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans[std::make_tuple(1, bucket(nseg), 0, 0)] = *plan;
  return RED_OK;
}

int red_get_segmented_plan(int64_t nseg, red_plan* plan) {
  if (!plan || nseg < 0) return set_error(RED_EINVAL, "bad plan or nseg");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(std::make_tuple(1, bucket(nseg), 0, 0));
    if (it != g_plans.end()) {
      *plan = it->second;
      return RED_OK;
    }
  }
  const DeviceInfo* dev;
  DeviceInfo none;
  none.cus = 256;
  *plan = default_seg_plan(nseg, ensure_device(&dev) == RED_OK ? *dev : none);
  return RED_OK;
}

int red_sum_segmented(const float* x, const int64_t* offsets, int64_t nseg, double* out, void* stream) {
  return red_sum_segmented_ex(x, offsets, nseg, out, stream, nullptr);
}

int red_sum_segmented_loop(const float* x, const int64_t* host_offsets, int64_t nseg, double* out,
                           void* stream) {
  if (nseg < 0 || !host_offsets) return set_error(RED_EINVAL, "bad offsets / nseg");
  if (nseg > 0 && (!x || !out)) return set_error(RED_EINVAL, "x or out is NULL");
  if (host_offsets[0] != 0) return set_error(RED_EINVAL, "offsets[0] must be 0");
  for (int64_t k = 0; k < nseg; ++k)
    if (host_offsets[k + 1] < host_offsets[k]) return set_error(RED_EINVAL, "offsets decrease at %lld", (long long)k);
  red_opts o;
  memset(&o, 0, sizeof o);
  o.acc = RED_ACC_COMPENSATED;
  o.plan = red_plan{RED_VARIANT_ATOMIC, 512, 4, 0, 0};
  for (int64_t k = 0; k < nseg; ++k) {
    int rc = red_sum_ex(RED_F32, x + host_offsets[k], host_offsets[k + 1] - host_offsets[k], out + k, stream, &o);
    if (rc) return rc;
  }
  return RED_OK;
}

int red_autotune_segmented(const float* x, const int64_t* offsets, int64_t nseg, double* out, void* stream,
                           int budget, red_plan* best, double* best_us) {
  int rc = validate_seg_args(x, offsets, nseg, out, nullptr);
  if (rc) return rc;
  const DeviceInfo* dev;
  if ((rc = ensure_device(&dev))) return rc;
  if (nseg == 0) return set_error(RED_EINVAL, "nothing to tune");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(RED_EINVAL, "autotuning cannot run inside stream capture");
  Workspace* ws;
  if ((rc = get_workspace(s, &ws))) return rc;
  // Each candidate: one warm launch, then kReps back-to-back launches timed
  // one by one with events (median).  The best few are then timed again in
  // interleaved rounds, so that a slow or fast stretch of the device does
  // not pick the plan.
  constexpr int kReps = 8, kFinalists = 4, kRounds = 3;
  struct Events {
    hipEvent_t e[2 * kReps] = {};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  for (hipEvent_t& x : ev.e) RED_HIP(hipEventCreateWithFlags(&x, hipEventDisableSystemFence));
  auto time_plan = [&](const red_plan& p, double* us) -> int {
    SegLaunch sl{p};
    int r = seg_launch(sl, x, offsets, nseg, out, ws, s, *dev);
    if (r) return r;
    for (int i = 0; i < kReps; ++i) {
      RED_HIP(hipEventRecord(ev.e[2 * i], s));
      if ((r = seg_launch(sl, x, offsets, nseg, out, ws, s, *dev))) return r;
      RED_HIP(hipEventRecord(ev.e[2 * i + 1], s));
    }
    RED_HIP(hipEventSynchronize(ev.e[2 * kReps - 1]));
    std::vector<double> t;
    for (int i = 0; i < kReps; ++i) {
      float ms = 0;
      RED_HIP(hipEventElapsedTime(&ms, ev.e[2 * i], ev.e[2 * i + 1]));
      t.push_back(ms * 1e3);
    }
    *us = median(t);
    return RED_OK;
  };
  std::vector<std::pair<double, red_plan>> timed_plans;
  int timed = 0;
  auto consider = [&](red_plan p) -> int {
    if (budget > 0 && timed >= budget) return RED_OK;
    double us = 0;
    int r = time_plan(p, &us);
    if (r) return r;
    ++timed;
    timed_plans.push_back({us, p});
    return RED_OK;
  };
  red_plan base = default_seg_plan(nseg, *dev);
  {
    red_plan p = base;
    p.flags &= ~RED_FLAG_NONTEMPORAL;
    rc = consider(p);
    p.flags |= RED_FLAG_NONTEMPORAL;
    if (!rc) rc = consider(p);
  }
  if (rc) return rc;
  const int nt_flag = (timed_plans.size() == 2 && timed_plans[0].first < timed_plans[1].first)
                          ? 0 : RED_FLAG_NONTEMPORAL;
  for (int v : {RED_VARIANT_RELAUNCH, RED_VARIANT_ATOMIC})
    for (int wg : {128, 256, 512})
      for (int ipt : {2, 4, 8})
        for (int m : {1, 2, 3, 4, 5, 6, 8})
          if (!rc) rc = consider(red_plan{v, wg, ipt, std::min(m * dev->cus, RED_MAX_GRID), nt_flag});
  if (rc) return rc;
  if (timed_plans.empty()) return set_error(RED_EINVAL, "no plan timed (budget 0?)");
  std::stable_sort(timed_plans.begin(), timed_plans.end(),
                   [](const std::pair<double, red_plan>& u, const std::pair<double, red_plan>& v) {
                     return u.first < v.first;
                   });
  const size_t nf = std::min<size_t>(kFinalists, timed_plans.size());
  std::vector<std::vector<double>> rounds(nf);
  for (int r = 0; r < kRounds; ++r)
    for (size_t k = 0; k < nf; ++k) {
      double us = 0;
      if ((rc = time_plan(timed_plans[k].second, &us))) return rc;
      rounds[k].push_back(us);
    }
  red_plan cur = timed_plans[0].second;
  double cur_us = 1e300;
  for (size_t k = 0; k < nf; ++k) {
    const double us = median(rounds[k]);
    if (us < cur_us) {
      cur_us = us;
      cur = timed_plans[k].second;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans[std::make_tuple(1, bucket(nseg), 0, 0)] = cur;
  }
  if (best) *best = cur;
  if (best_us) *best_us = cur_us;
  return RED_OK;
}

}  // extern "C"
