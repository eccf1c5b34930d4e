// Host-side shared declarations of libredsum (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/redsum.h"

namespace redsum {

struct BarrierWords;

// One carry slot of the segmented reduction: the binary64 sum of the piece
// of segment `seg` that falls in one slice, and the number of slices the
// segment spans (written with the first piece, for the fix-up kernel).
struct SegCarry {
  long long seg;
  double val;
  long long np;
};

struct DeviceInfo {
  int id = -1;
  int cus = 0;
  int64_t wallclock_khz = 0;
  int64_t clock_khz = 0;
  int64_t l2_bytes = 0;
  int64_t hbm_bytes = 0;
  int nxcc = 1;  // XCDs (accelerator complex dies) of the device
  int64_t lds_per_wg = 65536;  // largest LDS allocation of one workgroup
  bool coop = false;
};

// Library-owned device memory of one (device, stream).
struct Workspace {
  void* base = nullptr;
  BarrierWords* words = nullptr;   // barrier / ticket / error words
  void* partials = nullptr;        // RED_MAX_GRID x 8 bytes
  SegCarry* carry_in = nullptr;    // kMaxChunks slots
  SegCarry* carry_out = nullptr;   // kMaxChunks slots
  unsigned* seg_tickets = nullptr; // kMaxChunks counters
  unsigned* sink = nullptr;        // RED_MAX_GRID words for probes
  long long* stamps = nullptr;     // 2 x RED_MAX_GRID timestamps for probes
};

// Segmented batches are cut into at most this many chunks (carry slots and
// tickets per chunk).
constexpr int64_t kMaxChunks = 65536;

// Workspace layout sizes.
constexpr size_t kWordsBytes = 81920;  // BarrierWords (the XCD tree's lines), rounded up
constexpr size_t kPartialBytes = (size_t)RED_MAX_GRID * 8;
constexpr size_t kCarryBytes = (size_t)kMaxChunks * sizeof(SegCarry);
constexpr size_t kTicketBytes = (size_t)kMaxChunks * 4;
constexpr size_t kSinkBytes = (size_t)RED_MAX_GRID * 4;
constexpr size_t kStampBytes = (size_t)RED_MAX_GRID * 16;
constexpr size_t kWorkspaceBytes =
    kWordsBytes + kPartialBytes + 2 * kCarryBytes + kTicketBytes + kSinkBytes + kStampBytes;

// Errors ---------------------------------------------------------------
int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define RED_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::redsum::hip_fail(e_, #call); \
  } while (0)

// Device / workspace ---------------------------------------------------------
int ensure_device(const DeviceInfo** info);  // current device, initialized
int get_workspace(hipStream_t s, Workspace** ws);  // allocates outside capture
bool stream_capturing(hipStream_t s);
unsigned watchdog_spins();
unsigned barrier_groups(int grid);  // REDSUM_BARRIER_GROUPS, else the default policy

// Dominant-kernel timer: timer_begin records a slot's start event and
// returns the slot (or -1 when the timer is off / the stream is
// capturing), timer_end records its stop event; the two bracket whatever
// is launched between them.  launch_timed launches one kernel whose
// events, when a slot is due, are the kernel's own start and end
// (hipExtLaunchKernel); a cooperative launch is bracketed instead.
int timer_begin(hipStream_t s);
void timer_end(hipStream_t s, int slot);
int launch_timed(const void* fn, int grid, int block, void** args, hipStream_t s, bool cooperative,
                 size_t lds_bytes = 0);

// Kernel launch (uniform signature: one argument struct by value).
int launch(const void* fn, int grid, int block, void** args, hipStream_t s, bool cooperative, size_t lds_bytes = 0);

// Reductions ---------------------------------------------------------------
struct ReduceLaunch {
  int dtype, acc;
  red_plan plan;  // plan.flags: RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH
  bool timed = true;             // may carry the stream's kernel-timer events
  int max_grid = RED_MAX_GRID;   // partial slots the workspace holds
};
int validate_plan(const red_plan& p);
red_plan default_plan(int dtype, int64_t n, const DeviceInfo& dev);
int64_t single_wg_switch_bytes();  // Eq. 5 switch point (bytes) of the default plan
int reduce_launch(const ReduceLaunch& rl, const void* x, int64_t n, void* out, Workspace* ws,
                  hipStream_t s, const DeviceInfo& dev);
int reduce_max_coresident(int dtype, int acc, int ipt, bool nt, bool pipe, int wg, const DeviceInfo& dev,
                          int* n_wg);

// Segmented ------------------------------------------------------------------
struct SegLaunch {
  red_plan plan;  // variant: RED_VARIANT_ATOMIC (ticket) or RED_VARIANT_PERSISTENT
};
red_plan default_seg_plan(int64_t nseg, const DeviceInfo& dev);
int seg_launch(const SegLaunch& sl, const float* x, const int64_t* offsets, int64_t nseg, double* out,
               Workspace* ws, hipStream_t s, const DeviceInfo& dev);
int seg_max_coresident(int ipt, int wg, const DeviceInfo& dev, int* n_wg);

// Probes -------------------------------------------------------------------
int bw_proxy_launch(const void* x, int64_t nbytes, int n_wg, int wg, bool nt, Workspace* ws, hipStream_t s);

// Iterative stencil ---------------------------------------------------------
int stencil_launch(float* u, float* scratch, int64_t n, int steps, float r, int steps_per_sync, const red_plan& p,
                   Workspace* ws, hipStream_t s, const DeviceInfo& dev);

}  // namespace redsum
