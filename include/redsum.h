/*
 * redsum -- device-wide sum reduction for AMD Instinct MI355X (gfx950).
 *
 * C ABI of the shared library libredsum.so.  Every entry point takes plain
 * pointers and sizes; no C++ type or exception crosses this boundary.
 *
 * The operation is the reduction case study of Zhang, Wahib, Zhang,
 * Matsuoka, "A Study of Single and Multi-device Synchronization Methods in
 * Nvidia GPUs" (arXiv 2004.05371), Section VII ("Case Study: Reduction
 * Operator"): the sum of the elements of an array, computed by a per-thread
 * grid-stride accumulation, a warp (here: 64-lane wavefront) combine, a block
 * (workgroup) combine, and a device-wide synchronization before the final
 * combine of the per-block partials -- either an implicit barrier between
 * two kernel launches (Section VII-C, implicit variant) or a grid barrier
 * inside one persistent cooperative kernel (Section VII-C, explicit
 * variant).  The latency probes measure the synchronization levels studied
 * in Sections IV and V with the methods of Section IX (Eq. 6, 7, 8).
 *
 * Conventions for every entry point
 *   - Return value: RED_OK (0) or a negative red_status.  On error a
 *     thread-local message is available from red_last_error().
 *   - Arguments are validated before any HIP call is made.
 *   - "device pointer" means memory of the current HIP device (hipMalloc or
 *     torch CUDA tensors); the caller owns it.  The library never frees or
 *     retains caller memory.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Reductions are stream-ordered and asynchronous: results are valid once
 *     the stream has been synchronized.  Probes are synchronous.
 *   - The library owns one workspace per (device, stream) (per-workgroup
 *     partials, barrier words, carry slots, error word), allocated on first
 *     use outside of stream capture, freed by red_shutdown().  Calls that
 *     overlap on the same stream are ordered by the stream; calls on
 *     different streams use different workspaces.
 */
#ifndef REDSUM_H
#define REDSUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Input element types. */
typedef enum {
    RED_I32 = 0,  /* int32 in, int64 out (exact)                           */
    RED_F32 = 1,  /* binary32 in, binary64 out                             */
    RED_F16 = 2,  /* binary16 in, binary64 out                             */
    RED_BF16 = 3  /* bfloat16 in, binary64 out                             */
} red_dtype;

/* Status codes. */
typedef enum {
    RED_OK = 0,
    RED_EINVAL = -1,   /* invalid argument (null pointer, n < 0, bad dtype,
                          misaligned pointer, plan out of range, oversized
                          cooperative grid)                                  */
    RED_ENOTSUP = -2,  /* valid request this build does not support        */
    RED_EHIP = -3,     /* a HIP runtime call failed (message has details)   */
    RED_ETIMEOUT = -4, /* a device-side grid-barrier watchdog fired         */
    RED_ENOMEM = -5,   /* workspace allocation failed                       */
    RED_ENODEV = -6    /* no usable gfx950 device                           */
} red_status;

/* Device-wide synchronization used between the per-workgroup partials and
 * the final combine (Section VII-C). */
typedef enum {
    RED_VARIANT_AUTO = 0,       /* tuned plan if one is installed, else default */
    RED_VARIANT_RELAUNCH = 1,   /* implicit barrier: partials kernel, then a
                                   one-workgroup final kernel on the same stream */
    RED_VARIANT_ATOMIC = 2,     /* one kernel; the last workgroup to take an
                                   atomic ticket does the final combine        */
    RED_VARIANT_PERSISTENT = 3, /* one cooperative kernel; grid barrier, then
                                   workgroup 0 does the final combine (the
                                   barrier is split: workgroup 0 alone waits
                                   for every arrival; the others leave)        */
    RED_VARIANT_SINGLE = 4      /* one workgroup, no device-wide
                                   synchronization at all: the "use fewer
                                   workers" side of the performance model
                                   (Section VII-A, Eq. 2-5), for small n      */
} red_variant;

/* In-register accumulation of floating-point inputs. */
typedef enum {
    RED_ACC_COMPENSATED = 0, /* fp32 (sum, error) pairs updated by TwoSum     */
    RED_ACC_PLAIN = 1        /* plain fp32 accumulation                        */
} red_acc;

/* Cross-lane method of the wavefront combine (probe selection). */
typedef enum {
    RED_WAVE_DPP = 0,      /* DPP quad_perm / row_ror / row_bcast moves       */
    RED_WAVE_SWIZZLE = 1,  /* ds_swizzle xor butterfly within 32 lanes        */
    RED_WAVE_BPERMUTE = 2, /* ds_bpermute xor butterfly over 64 lanes         */
    RED_WAVE_DPP_STEP = 3  /* a single DPP add step (latency of one move+add) */
} red_wave_op;

/* Value type carried through the wavefront probe's combine. */
typedef enum {
    RED_WAVE_T_F32 = 0,  /* float                                              */
    RED_WAVE_T_I32 = 1,  /* 32-bit integer (wrapping adds)                     */
    RED_WAVE_T_F64 = 2,  /* double: two 32-bit cross-lane moves per step       */
    RED_WAVE_T_I64 = 3,  /* 64-bit integer: two moves per step                 */
    RED_WAVE_T_COMP = 4  /* compensated fp32 (sum, error) pair combined by
                            TwoSum: the reduction's own combine, two moves    */
} red_wave_type;

/* Plan / option flags. */
#define RED_FLAG_NONTEMPORAL 1  /* streaming loads with the nontemporal hint  */
#define RED_FLAG_NO_GRAPH 2     /* segmented: launch directly, no hipGraph    */
#define RED_FLAG_PLAIN_LAUNCH 4 /* persistent variants: ordinary launch of a
                                   grid capped at the co-resident limit
                                   (occupancy x CUs) instead of the
                                   cooperative launch API; the barrier
                                   watchdog guards against a grid that is
                                   not fully resident                       */
#define RED_FLAG_PIPELINE 8     /* reductions: double-buffered loop that
                                   issues the next tile's loads before the
                                   current tile's arithmetic                */
#define RED_FLAG_XCD 16         /* workgroups count their arrivals on an
                                   XCD arrival tree (nodes of 64, one line
                                   per XCD, then one top line) instead of
                                   one counter per group.  Grid barriers
                                   (stencil, segmented grid-barrier
                                   fix-up) then release with one L2
                                   write-back per XCD instead of one per
                                   workgroup; that relies on the
                                   round-robin dispatch of workgroups over
                                   the XCDs, which the tree checks against
                                   every workgroup's XCC_ID register, and a
                                   barrier that finds a mismatch falls back
                                   to a release by every workgroup (correct,
                                   slower).  The atomic and persistent
                                   reductions publish their partials with
                                   device-scope atomic stores (no L2
                                   write-back at all), so for them the flag
                                   only changes how arrivals are counted   */
/* Segmented batches: force one way of cutting and walking the slices
 * (at most one of the three; by default the device picks from the mean
 * segment length).  For experiments and tests. */
#define RED_FLAG_SEG_WORKGROUP 32 /* one slice per workgroup                 */
#define RED_FLAG_SEG_PIECES 64    /* one slice per wavefront, one wavefront
                                     combine per piece of a segment         */
#define RED_FLAG_SEG_RUNS 128     /* one slice per wavefront, reduce-by-key
                                     over runs of consecutive values (plan
                                     ipt <= 4, RED_EINVAL otherwise)        */

/* Launch plan of one reduction. */
typedef struct {
    int32_t variant; /* red_variant, not RED_VARIANT_AUTO when installed     */
    int32_t wg;      /* workgroup size in threads: 64..1024, multiple of 64  */
    int32_t ipt;     /* 16-byte loads per thread per loop iteration: 1,2,4,8 */
    int32_t grid;    /* number of workgroups, 1..RED_MAX_GRID; 0 = automatic */
    int32_t flags;   /* RED_FLAG_NONTEMPORAL | RED_FLAG_PLAIN_LAUNCH |
                        RED_FLAG_PIPELINE | RED_FLAG_XCD                    */
} red_plan;

#define RED_MAX_GRID 8192

/* Options of red_sum_ex / red_sum_segmented_ex.  A zero-initialized struct
 * means: automatic plan, compensated accumulation. */
typedef struct {
    red_plan plan;   /* plan.variant == RED_VARIANT_AUTO selects the installed
                        plan (or the default) and ignores the other fields;
                        with an explicit variant, wg / ipt left at 0 take
                        the default values (grid 0 is automatic)            */
    int32_t acc;     /* red_acc                                             */
    int32_t flags;   /* RED_FLAG_* (OR-ed with plan.flags); other bits must
                        be zero                                             */
} red_opts;

/* ---------------------------------------------------------------------
 * Initialization
 * ------------------------------------------------------------------- */

/* Select and check `device` (must be gfx950), query its properties and
 * allocate the workspace of the null stream.  Idempotent.  Other entry
 * points call it implicitly for the current device.
 * Errors: RED_ENODEV (no device / not gfx950), RED_EHIP, RED_ENOMEM. */
int red_init(int device);

/* Free every workspace and cached graph.  Safe to call more than once. */
void red_shutdown(void);

/* Thread-local description of the last error of this thread ("" if none).
 * The pointer stays valid until the next library call on this thread. */
const char *red_last_error(void);

/* Synchronize `stream`, then report a grid-barrier watchdog timeout raised
 * by an earlier persistent kernel on that stream (RED_ETIMEOUT), or arrival
 * counters left incomplete (RED_ENOTSUP: an abandoned barrier or ticket),
 * clearing the flag and the barrier words.  RED_OK if none. */
int red_check_error(void *stream);

/* ---------------------------------------------------------------------
 * Reductions (Section VII)
 * ------------------------------------------------------------------- */

/* out = sum of x[0..n).
 *   dtype  red_dtype of x.
 *   x      device pointer, n elements, aligned to the element size (any
 *          16-byte misalignment is handled); may be NULL only if n == 0.
 *   n      number of elements, 0 <= n < 2^40.
 *   out    device pointer to one int64_t (RED_I32) or one double (float
 *          dtypes), written exactly once, asynchronously.  n == 0 writes 0.
 *   stream hipStream_t or NULL.
 * int32 sums are exact.  Floating-point inputs are accumulated in fp32 with
 * TwoSum compensation per thread and through the wavefront and workgroup
 * combines; the per-workgroup partials are combined in binary64 in index
 * order.  Results are bit-identical across repeated calls with the same plan.
 * NaN propagates; +inf with -inf gives NaN.
 * Errors: RED_EINVAL (validation), RED_EHIP, RED_ENOMEM. */
int red_sum(int dtype, const void *x, int64_t n, void *out, void *stream);

/* red_sum with explicit options (variant, plan, accumulation). */
int red_sum_ex(int dtype, const void *x, int64_t n, void *out, void *stream, const red_opts *opts);

/* Largest grid (workgroups, hence per-workgroup partials) of
 * red_sum_noalloc. */
#define RED_NOALLOC_MAX_GRID 2048

/* red_sum_ex that allocates nothing, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, plans, kernels and results as
 * red_sum_ex (the same plan gives the same bits).
 *   Scratch: the partials and barrier words live in one static device
 *   array of the library (80 KiB of words + RED_NOALLOC_MAX_GRID x 8 bytes,
 *   held by every device the library runs on until the process ends), not
 *   in a per-stream workspace.  Its address on each device is looked up
 *   once, by red_init or by the first call on that device (a lookup, not an
 *   allocation; that first call must not be under capture).
 *   Limit: an explicit opts->plan.grid above RED_NOALLOC_MAX_GRID is
 *   rejected with RED_EINVAL; an automatic grid is capped there.
 *   Sharing: every call on one device uses that device's one array, and the
 *   array keeps the last call's contents.  Calls that overlap on one
 *   device (two streams, two threads) race; serialize them.  The barrier
 *   and ticket words are cleared by a small kernel at the start of each
 *   call of the atomic-ticket and persistent variants, which alone use them.
 *   No kernel-timer events are recorded (red_kernel_timer does not see
 *   these calls), and a persistent variant's watchdog is not reported by
 *   red_check_error (which reads the stream's workspace).
 * Errors: RED_EINVAL (validation, grid above the limit), RED_ENODEV,
 * RED_EHIP. */
int red_sum_noalloc(int dtype, const void *x, int64_t n, void *out, void *stream, const red_opts *opts);

/* Per-segment sums of a CSR batch: out[k] = sum of x[offsets[k] ..
 * offsets[k+1]) for k in [0, nseg).
 *   x       device pointer to binary32 values (aligned to 4 bytes).
 *   offsets device pointer to nseg + 1 non-decreasing int64 offsets with
 *           offsets[0] == 0 (not checked on the device).
 *   nseg    number of segments, 0 <= nseg < 2^31.
 *   out     device pointer to nseg doubles.  Empty segments give 0.
 * A fixed grid: every workgroup (long segments) or every wavefront (short
 * ones) owns an equal slice of the elements and sums the pieces of the
 * segments that meet its slice; for very short segments a wavefront
 * reduces by key over runs of consecutive values with a segmented scan
 * across its lanes.  The pieces of segments that cross slice boundaries
 * are combined in slice order in binary64, by default by the wavefront
 * that publishes a segment's last piece, found with an atomic ticket
 * (red_sum_segmented_ex lists the other ways).  The kernels are
 * captured in a hipGraph on the first call for a given (x, offsets, nseg,
 * out, stream, plan) and replayed afterwards; when the stream is already
 * being captured by the caller they are simply launched into that
 * capture.
 * Errors: RED_EINVAL, RED_EHIP, RED_ENOMEM. */
int red_sum_segmented(const float *x, const int64_t *offsets, int64_t nseg, double *out, void *stream);

/* red_sum_segmented with explicit options.  opts->plan.variant selects how
 * the pieces of segments cut by slice boundaries are summed:
 * RED_VARIANT_RELAUNCH (a second, small kernel after the implicit barrier
 * between launches; both kernels go into the graph), RED_VARIANT_ATOMIC
 * (the last contributor, found by an atomic ticket; the pieces are
 * published with device-scope atomic stores, no L2 write-back) or
 * RED_VARIANT_PERSISTENT (the owning slice after a grid barrier that
 * neither writes back nor invalidates an L2, the pieces being published;
 * co-resident grid: a cooperative launch is made directly, not from a
 * graph; with RED_FLAG_PLAIN_LAUNCH the grid, capped at the co-resident
 * count, is an ordinary launch, and that one persistent kernel is captured
 * and replayed like the other fix-ups; a grid that does not stay resident
 * ends on the barrier watchdog, reported by red_check_error).  plan.wg is at
 * most 512 here (RED_EINVAL otherwise); grid x wg / 64 wavefront slices
 * are capped at 65536.
 * RED_FLAG_NO_GRAPH disables graph capture; RED_FLAG_SEG_WORKGROUP,
 * RED_FLAG_SEG_PIECES or RED_FLAG_SEG_RUNS forces one form (RED_EINVAL for
 * two of them, or for RED_FLAG_SEG_RUNS with plan.ipt > 4). */
int red_sum_segmented_ex(const float *x, const int64_t *offsets, int64_t nseg, double *out,
                         void *stream, const red_opts *opts);

/* Baseline for the segmented batch: one single-kernel reduction launch per
 * segment.  host_offsets is a HOST pointer to nseg + 1 offsets. */
int red_sum_segmented_loop(const float *x, const int64_t *host_offsets, int64_t nseg, double *out,
                           void *stream);

/* ---------------------------------------------------------------------
 * Iterative stencil (Section VII-B: a persistent kernel that holds the time
 * loop of an iterative stencil method can keep its data on chip across
 * grid barriers, where one launch per step cannot)
 * ------------------------------------------------------------------- */

/* `steps` explicit steps of the 1D heat equation (Jacobi smoothing) on
 * u[0..n), in place:
 *     u'[i] = u[i] + r * ((u[i-1] + u[i+1]) - 2 u[i])   1 <= i <= n-2,
 *     u[0] and u[n-1] unchanged,
 * every operation one binary32 operation in exactly this order (no fused
 * multiply-add), so the result is the same bit for bit whatever the form.
 *   u        device pointer to n floats, updated in place.
 *   scratch  device pointer to n floats owned by the caller, not
 *            overlapping u; its contents are overwritten.
 *   n        number of values, 0 <= n < 2^40; n < 3 or steps == 0 leaves u
 *            as it is.
 *   steps    number of steps, >= 0.
 *   r        the step's coefficient (stable for 0 <= r <= 1/2).
 *   steps_per_sync  persistent form: steps between grid barriers, which
 *            is also the halo width each workgroup keeps (1 = a barrier
 *            every step); 0 = chosen by the library: the widest halo up to
 *            128 that the window holds beside the block (the block
 *            length is set as for 8).  Any value gives the same result.
 *   opts     NULL or plan.variant:
 *            RED_VARIANT_RELAUNCH    one kernel launch per step (the
 *                                    implicit barrier), u and scratch
 *                                    alternating;
 *            RED_VARIANT_PERSISTENT  one launch holding the time loop: each
 *                                    workgroup keeps its block and halos
 *                                    (at most 16384 values) in its threads'
 *                                    registers and exchanges boundary values
 *                                    with its neighbours through u / scratch
 *                                    (device-scope atomic stores and loads)
 *                                    at a grid barrier every steps_per_sync
 *                                    steps;
 *            RED_VARIANT_AUTO        persistent when the array's windows fit
 *                                    the co-resident workgroups, else
 *                                    relaunch.
 *            plan.wg (persistent default: the fewest values per thread, 2
 *            to 32, whose workgroup stays within 1024 threads and is
 *            co-resident with the grid; relaunch default 512; a caller's
 *            size holds at most 32 values per thread), plan.grid (default
 *            one workgroup per CU, or as many 16 K-value windows as the
 *            array needs rounded up to a whole number per CU) and flags
 *            RED_FLAG_PLAIN_LAUNCH / RED_FLAG_XCD as for red_sum.
 * Asynchronous on `stream`.  RED_EINVAL for bad arguments, overlapping
 * arrays, or a persistent request whose windows do not fit the co-resident
 * workgroups; a grid-barrier watchdog timeout is reported by
 * red_check_error. */
int stencil_jacobi_1d(float *u, float *scratch, int64_t n, int32_t steps, float r, int32_t steps_per_sync,
                      void *stream, const red_opts *opts);

/* ---------------------------------------------------------------------
 * Plans and autotuning (performance model of Section VII-A/B as prior)
 * ------------------------------------------------------------------- */

/* Install `plan` for reductions of `dtype` with `acc` whose element count
 * has the same bit length as n (ceil(log2 n) bucket).  Plans are validated
 * (RED_EINVAL otherwise). */
int red_set_plan(int dtype, int acc, int64_t n, const red_plan *plan);

/* Plan that red_sum would use for (dtype, acc, n): the installed one, else
 * the default.  Writes *plan. */
int red_get_plan(int dtype, int acc, int64_t n, red_plan *plan);

/* Time candidate plans on the caller's data (x, n; out is overwritten) and
 * install the fastest for the (dtype, acc, n) bucket; writes it to *best and
 * its median time in microseconds to *best_us (either may be NULL).
 * Synchronous.  `budget` bounds the number of candidates timed (0 = all,
 * followed by finals: the best shape under the relaunch, atomic-ticket and
 * persistent plain-launch variants, timed again in 5 interleaved rounds,
 * the lowest median winning). */
int red_autotune(int dtype, int acc, const void *x, int64_t n, void *out, void *stream, int budget,
                 red_plan *best, double *best_us);

/* Cost of one candidate plan in microseconds (lower is better), or a
 * negative red_status to stop the search.  It may lower plan->grid (the
 * plan kept is the one it was given back). */
typedef double (*red_cost_fn)(red_plan *plan, void *ctx);

/* The candidate search of red_autotune on its own, with the cost of each
 * candidate supplied by the caller (red_autotune times it on the GPU; a
 * model or a test may supply another), for a device of `cus` compute units
 * and `nxcc` XCDs.  Candidates, in order: the default plan without and with
 * the nontemporal hint; every relaunch shape (pipelined or not) x wg {128,
 * 256, 512, 1024} x ipt {1, 2, 4, 8} x grid {1, 2, 3, 4, 6, 8, 12, 16} x
 * cus (up to the work's tile count); one-workgroup plans when n is within
 * 64 times the Eq. 4/5 switch point; then the atomic-ticket and persistent
 * (cooperative and plain launch) variants of the best shape, with and
 * without RED_FLAG_XCD when allow_xcd and nxcc > 1.  The first candidate
 * of the lowest cost wins; nothing is installed.  budget > 0 caps the
 * number of candidates costed.  No HIP call.
 * Errors: RED_EINVAL, or the cost function's negative status. */
int red_autotune_search(int dtype, int64_t n, int cus, int nxcc, int allow_xcd, int budget, red_cost_fn cost,
                        void *ctx, red_plan *best, double *best_us);

/* Install / read the plan of segmented batches whose nseg has the same
 * bit length as `nseg` (variant RED_VARIANT_ATOMIC or _PERSISTENT, wg at
 * most 512). */
int red_set_segmented_plan(int64_t nseg, const red_plan *plan);
int red_get_segmented_plan(int64_t nseg, red_plan *plan);

/* Autotune the segmented kernel on the caller's batch (synchronous) and
 * install the best plan for batches with the same nseg bit length.  The
 * search times the default plan with and without the nontemporal hint,
 * then every fix-up variant (RELAUNCH, ATOMIC) x wg {128, 256, 512} x ipt
 * {2, 4, 8} x grid {1, 2, 3, 4, 5, 6, 8} x CUs (8 back-to-back launches each,
 * median), and re-times the best 4 in 3 interleaved rounds.  budget > 0
 * caps the number of candidates timed in the first pass. */
int red_autotune_segmented(const float *x, const int64_t *offsets, int64_t nseg, double *out,
                           void *stream, int budget, red_plan *best, double *best_us);

/* ---------------------------------------------------------------------
 * Latency probes (Sections IV, V, IX).  Synchronous; results on the host.
 * Each fills ns (mean latency per operation, nanoseconds, by the host
 * differential of Eq. 7 between kernels with r1 and r2 repetitions),
 * sigma_ns (its uncertainty by Eq. 8 over `reps` timed pairs) and, if
 * non-NULL, cycles (in-kernel shader-clock cycles per operation, the
 * in-SM clock method of Section IX-C; wall-clock ns for the grid probe).
 * reps >= 2.
 * ------------------------------------------------------------------- */

/* One wavefront-level operation (red_wave_op) in a dependent chain, run by
 * every wave of one workgroup of wg_size threads, on float values (the
 * shuffle-based warp reduction of Section VII-D and Table V). */
int sync_bench_wave(int op, int wg_size, int reps, double *ns, double *sigma_ns, double *cycles,
                    void *stream);

/* sync_bench_wave on values of type `type` (red_wave_type); an unknown op
 * or type is RED_EINVAL. */
int sync_bench_wave_ex(int op, int type, int wg_size, int reps, double *ns, double *sigma_ns,
                       double *cycles, void *stream);

/* One workgroup barrier (s_barrier) in a chain, n_wg workgroups of wg_size
 * threads. */
int sync_bench_block(int wg_size, int n_wg, int reps, double *ns, double *sigma_ns, double *cycles,
                     void *stream);

/* Block-barrier throughput under load (Table II's throughput column, as
 * barriers completed rather than derived from a latency): wg_per_cu x CUs
 * workgroups of wg_size threads, all co-resident (RED_EINVAL otherwise),
 * each running barriers back to back for window_ticks ticks of the 100 MHz
 * wall clock (100 .. 1e8).  *barriers_per_us_per_cu receives the barriers
 * completed per microsecond per CU (summed over its workgroups), and
 * *cycles_per_barrier (if non-NULL) the mean shader-clock cycles between
 * one workgroup's barriers. */
int sync_bench_block_tput(int wg_size, int wg_per_cu, int64_t window_ticks, double *barriers_per_us_per_cu,
                          double *cycles_per_barrier, void *stream);

/* One grid barrier inside a cooperative kernel of n_wg workgroups of
 * wg_size threads (n_wg must be co-resident: RED_EINVAL otherwise). */
int sync_bench_grid(int n_wg, int wg_size, int reps, double *ns, double *sigma_ns, double *cycles,
                    void *stream);

/* sync_bench_grid with an explicit barrier shape: groups = 1 is the flat
 * centralized barrier, groups = 2..32 the two-level barrier whose first
 * level counts the workgroups with blockIdx % groups equal, -1 the
 * XCD-aggregated barrier (an arrival tree over the workgroups of each XCD
 * with one L2 write-back per XCD, see RED_FLAG_XCD), 0 the default policy.
 * -2 is the XCD-aggregated barrier with odd workgroups reporting the next
 * XCD: it drives the barrier's fall-back (every workgroup releases its own
 * stores when one ran off its XCD) from the host, for tests. */
int sync_bench_grid_ex(int n_wg, int wg_size, int groups, int reps, double *ns, double *sigma_ns,
                       double *cycles, void *stream);

/* sync_bench_grid_ex with the two repetition counts of Eq. 7 fixed by the
 * caller (r1 > r2 > 0, r1 <= 65536) instead of calibrated: the
 * repeat-count invariance check of Section IX-C (the latency of one
 * barrier must not depend on r1, r2).  r1 = r2 = 0 calibrates. */
int sync_bench_grid_r(int n_wg, int wg_size, int groups, int64_t r1, int64_t r2, int reps, double *ns,
                      double *sigma_ns, double *cycles, void *stream);

/* sync_bench_grid_r for the grid barrier that carries only data published
 * with device-scope atomic stores and read with device-scope atomic loads
 * (the barrier of the persistent reduction's partials and of the segmented
 * grid-barrier fix-up): no arrival writes back an L2 and no workgroup
 * invalidates one after the wait, so it measures the arrival counting and
 * the wait alone.  Arguments, shapes (groups) and errors as in
 * sync_bench_grid_r. */
int sync_bench_grid_published(int n_wg, int wg_size, int groups, int64_t r1, int64_t r2, int reps, double *ns,
                              double *sigma_ns, double *cycles, void *stream);

/* Launch overhead of a kernel boundary (the implicit barrier) by kernel
 * fusion, Eq. 6, with (i, j) = (8, 1) launches of n_wg x wg_size kernels
 * that wait 5 us per unit.  cooperative selects the launch type: 0 ordinary
 * launches, 1 the cooperative launch API, 2 ordinary kernels replayed from
 * a captured hipGraph (i kernels in one graph against j in another; the
 * graphs are captured on a private stream and replayed on `stream`, which
 * must not be capturing); other values: RED_EINVAL.  null_kernel_ns (if
 * non-NULL) receives the total latency of one null kernel in ns: for
 * ordinary and cooperative launches by the Section IV formula (host clock
 * around 1 and around 5 launches, each followed by a synchronization); for
 * the graph type, where one replay launches every kernel of the graph, by
 * the Eq. 7 differential between graphs of 40 and of 5 null kernels timed
 * with events (the cost of one more null kernel inside a graph). */
int sync_bench_relaunch(int n_wg, int wg_size, int cooperative, int reps, double *ns,
                        double *sigma_ns, double *null_kernel_ns, void *stream);

/* sync_bench_relaunch with the launch counts (i, j) of Eq. 6 (1 <= i, j <=
 * 64, i != j) and the wait unit in ticks of the device's 100 MHz wall
 * clock (0 = 5 us) chosen by the caller: the overhead per launch must not
 * depend on (i, j). */
int sync_bench_relaunch_ex(int n_wg, int wg_size, int cooperative, int i, int j, int64_t unit_ticks, int reps,
                           double *ns, double *sigma_ns, double *null_kernel_ns, void *stream);

/* Method check of Eq. 7 with a known answer: one workgroup of a kernel
 * that waits r x unit_ticks ticks of the 100 MHz wall clock, with r = r1
 * and r = r2 (r1 > r2 >= 1, r1 x unit_ticks <= 1e8); *ns receives Eq. 7's
 * latency per unit, which must come out as unit_ticks x 10 ns, and
 * *sigma_ns its Eq. 8 uncertainty. */
int sync_bench_spin(int64_t unit_ticks, int64_t r1, int64_t r2, int reps, double *ns, double *sigma_ns,
                    void *stream);

/* Values of one wavefront combine (the warp reduction of Section VII-D):
 * host_in holds 64 values of red_wave_type `type` (4 bytes each for
 * float / int32, 8 for double / int64 / the compensated pair), value l for
 * lane l; after combine `op` every lane's result is written to host_out
 * (64 values, same layout).  The full combines (DPP, ds_swizzle,
 * ds_bpermute) return the sum of the 64 values to every lane (integers
 * wrap modulo 2^32 or 2^64); RED_WAVE_DPP_STEP returns v[l] + v[l-1]
 * inside each 16-lane row and v[l] at a row's first lane.  Synchronous. */
int sync_check_wave(int op, int type, const void *host_in, void *host_out, void *stream);

/* Grid-barrier ordering check: every workgroup of a cooperative kernel
 * records the 100 MHz wall clock before and after one grid barrier; writes
 * max(before) and min(after) (in clock ticks) to host *max_before and
 * *min_after.  A correct barrier gives max_before <= min_after. */
int sync_check_grid_order(int n_wg, int wg_size, int64_t *max_before, int64_t *min_after,
                          void *stream);

/* Grid-barrier visibility check: a cooperative kernel of `rounds` rounds in
 * which every workgroup stores one value with an ordinary store, meets the
 * others at a grid barrier, and reads every workgroup's value with ordinary
 * loads (the same addresses each round), then meets them again.  *errors
 * (host) receives the number of reads that did not see the round's value;
 * a correct barrier gives 0.  groups as in sync_bench_grid_ex.  Errors:
 * RED_EINVAL (bad arguments, grid not co-resident), RED_ETIMEOUT (watchdog),
 * RED_EHIP. */
int sync_check_grid_visibility(int n_wg, int wg_size, int groups, int rounds, int64_t *errors, void *stream);

/* sync_check_grid_visibility for the barrier of sync_bench_grid_published:
 * every value is stored with a device-scope atomic store and read with
 * device-scope atomic loads.  Arguments and errors as there. */
int sync_check_grid_visibility_published(int n_wg, int wg_size, int groups, int rounds, int64_t *errors,
                                         void *stream);

/* Watchdog check: a cooperative kernel in which workgroup `skip_wg` never
 * arrives at the grid barrier while the others wait with a spin limit of
 * `spin_limit` polls; returns RED_ETIMEOUT when the watchdog fires (the
 * expected outcome), RED_OK if not.  Every wave exits. */
int sync_check_watchdog(int n_wg, int wg_size, int skip_wg, int spin_limit, void *stream);

/* Largest number of co-resident workgroups of wg_size threads for the
 * persistent reduction kernel (occupancy x compute units). */
int red_max_coresident(int wg_size, int32_t *n_wg);

/* Largest number of co-resident workgroups of wg_size threads (at most
 * 512) for the segmented kernel with `ipt` loads per thread: the grid
 * limit of the RED_VARIANT_PERSISTENT (grid barrier) fix-up of
 * red_sum_segmented_ex.  Errors: RED_EINVAL, RED_ENODEV, RED_EHIP. */
int red_max_coresident_segmented(int ipt, int wg_size, int32_t *n_wg);

/* Device facts: compute units, wall-clock rate (kHz), shader clock (kHz),
 * L2 bytes (per XCD), HBM bytes, number of XCDs.  Any pointer may be NULL. */
int red_device_info(int32_t *cus, int64_t *wallclock_khz, int64_t *clock_khz, int64_t *l2_bytes,
                    int64_t *hbm_bytes, int32_t *nxcc);

/* XCD (hardware XCC_ID) on which each of n_wg workgroups of an ordinary
 * launch ran; host_xcc receives n_wg ints.  Synchronous. */
int sync_xcc_map(int n_wg, int wg_size, int32_t *host_xcc, void *stream);

/* ---------------------------------------------------------------------
 * Measurement helpers (not part of a reduction)
 * ------------------------------------------------------------------- */

/* While enabled on `stream`, reduction / segmented / stencil launches on it
 * time their dominant streaming kernel (the partials kernel of the relaunch
 * variant, the single kernel otherwise) with a pair of HIP events without
 * system-scope fences.  An ordinary launch of a reduction kernel carries
 * the events in its own dispatch (hipExtLaunchKernel), so they take the
 * kernel's start and end as a kernel trace does; a cooperative launch, the
 * segmented batch (slice and fix-up kernels) and the persistent stencil
 * are bracketed by events recorded before and after them.  enable = 0
 * turns the timer off; enable = k > 0 times every k-th launch (k > 1 keeps
 * the events' own cost off most launches).  Enabling clears earlier
 * records.  Not recorded inside stream capture. */
int red_kernel_timer(void *stream, int enable);

/* Synchronize `stream` and report the timed launches: mean and minimum
 * duration in microseconds and their number (any pointer may be NULL). */
int red_kernel_timer_read(void *stream, double *mean_us, double *min_us, int64_t *count);

/* Read-only bandwidth ceiling (Section VII-B bandwidth proxy): a
 * grid-stride read of nbytes of x (16-byte aligned) with 16-byte loads
 * and two integer adds per load, writing one word per workgroup to the
 * workspace.  Asynchronous. */
int red_bw_proxy(const void *x, int64_t nbytes, int n_wg, int wg_size, void *stream);

/* red_bw_proxy with flags: RED_FLAG_NONTEMPORAL issues the loads with the
 * nontemporal hint (the hint the reductions stream with), other bits
 * RED_EINVAL.  Without it the loads are ordinary, which also fills the
 * memory-side cache (the benchmark's cache flush relies on that). */
int red_bw_proxy_ex(const void *x, int64_t nbytes, int n_wg, int wg_size, int flags, void *stream);

/* Host-side probe formulas, exported so host logic can be tested without a
 * GPU: Eq. 6, Eq. 7, Eq. 8 (from two sample arrays of length nsamp). */
double red_eq6_overhead(double lat_ij, double lat_ji, int i, int j);
double red_eq7_latency(double lat_k1, double lat_k2, int64_t r1, int64_t r2);
double red_eq8_sigma(const double *k1, const double *k2, int nsamp, int64_t r1, int64_t r2);

#ifdef __cplusplus
}
#endif

#endif /* REDSUM_H */
