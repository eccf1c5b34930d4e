// Device primitives of the sum reduction on gfx950 (CDNA4, wave64).
//
// Levels of the synchronization hierarchy used by the reduction case study
// (Section VII-C of Zhang et al., arXiv 2004.05371):
//   * lane          : per-thread accumulation of a grid-stride share
//                     (the "summing" step), with 16-byte vector loads;
//   * wavefront     : a 64-lane cross-lane combine (the paper's warp
//                     shuffle reduction, Section VII-D) done with DPP moves,
//                     ds_swizzle or ds_bpermute;
//   * workgroup     : per-wave partials staged in LDS, one s_barrier, and a
//                     second wavefront combine in wave 0 (the paper's
//                     block_reduce);
//   * grid          : a software grid barrier on device-scope atomics for a
//                     cooperative (co-resident) launch (the paper's
//                     grid.sync), bounded by a watchdog.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace redsum {

constexpr int kWave = 64;
constexpr int kMaxWavesPerWG = 16;  // 1024 threads

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Combine operations for the cross-lane trees.  Every T is a whole number of
// 32-bit words; zero() is the identity.
// ---------------------------------------------------------------------------
struct OpI64 {
  using T = long long;
  __device__ static T zero() { return 0; }
  __device__ static T add(T a, T b) { return a + b; }
};
struct OpF64 {
  using T = double;
  __device__ static T zero() { return 0.0; }
  __device__ static T add(T a, T b) { return a + b; }
};
struct OpF32 {
  using T = float;
  __device__ static T zero() { return 0.0f; }
  __device__ static T add(T a, T b) { return a + b; }
};

// Error-free transformation of a sum (Knuth's TwoSum, branch free):
// s + e == a + b exactly, s = fl(a + b).  Needs round-to-nearest and no
// reassociation (this file is never compiled with fast-math).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bp = s - a;
  float ap = s - bp;
  e = (a - ap) + (b - bp);
}

// Compensated fp32 value: the represented number is s + c.
struct CompF32 {
  float s, c;
};
// binary64 value of a compensated pair.  Once s is infinite or NaN the
// TwoSum error terms are NaN (inf - inf), so c is dropped: the sum of
// finite inputs with +inf is +inf, and NaN / (+inf with -inf) stay NaN.
__device__ __forceinline__ double comp_to_double(CompF32 a) {
  return __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
}

struct OpComp {
  using T = CompF32;
  __device__ static T zero() { return CompF32{0.0f, 0.0f}; }
  __device__ static T add(T a, T b) {
    CompF32 r;
    float e;
    two_sum(a.s, b.s, r.s, e);
    r.c = (a.c + b.c) + e;
    return r;
  }
};

// ---------------------------------------------------------------------------
// Word-wise cross-lane moves
// ---------------------------------------------------------------------------
template <class T>
struct Words {
  static_assert(sizeof(T) % 4 == 0, "cross-lane values are whole 32-bit words");
  static constexpr int N = sizeof(T) / 4;
};

// DPP move of every word of v.  Lanes whose source is invalid or whose row
// is masked off receive 0 (the identity of every Op above).
template <int CTRL, int ROW_MASK, int BANK_MASK, class T>
__device__ __forceinline__ T dpp_move(T v) {
  int w[Words<T>::N];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < Words<T>::N; ++i)
    w[i] = __builtin_amdgcn_update_dpp(0, w[i], CTRL, ROW_MASK, BANK_MASK, true);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

template <class T>
__device__ __forceinline__ T read_lane(T v, int lane) {
  int w[Words<T>::N];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < Words<T>::N; ++i) w[i] = __builtin_amdgcn_readlane(w[i], lane);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

template <int PATTERN, class T>
__device__ __forceinline__ T swizzle_move(T v) {
  int w[Words<T>::N];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < Words<T>::N; ++i) w[i] = __builtin_amdgcn_ds_swizzle(w[i], PATTERN);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

template <class T>
__device__ __forceinline__ T bpermute_move(T v, int src_lane) {
  int w[Words<T>::N];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < Words<T>::N; ++i) w[i] = __builtin_amdgcn_ds_bpermute(src_lane << 2, w[i]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// DPP control codes (GFX9 encoding).
constexpr int kQuadPerm1032 = 0xB1;  // quad_perm:[1,0,3,2]  (lane ^ 1)
constexpr int kQuadPerm2301 = 0x4E;  // quad_perm:[2,3,0,1]  (lane ^ 2)
constexpr int kRowRor4 = 0x124;      // rotate right by 4 within a 16-lane row
constexpr int kRowRor8 = 0x128;      // rotate right by 8 within a row
constexpr int kRowShr1 = 0x111;      // shift right by 1 within a row
constexpr int kRowShr2 = 0x112;      // shift right by 2 within a row
constexpr int kRowShr4 = 0x114;      // shift right by 4 within a row
constexpr int kRowShr8 = 0x118;      // shift right by 8 within a row
constexpr int kRowBcast15 = 0x142;   // lane 15 of each row -> next row
constexpr int kRowBcast31 = 0x143;   // lane 31 -> rows 2 and 3

// ---------------------------------------------------------------------------
// Wavefront combine: 64 lane values -> one value, returned uniformly (SGPR
// broadcast) to every lane.  All 64 lanes must be active.  The order of the
// combine is fixed, so results are deterministic.
// ---------------------------------------------------------------------------
// DPP: two quad_perm steps and two row rotations leave every lane of a
// 16-lane row with the row total; row_bcast:15 then adds row r-1 into rows
// 1 and 3, and row_bcast:31 adds rows 0+1 into row 3, so lane 63 holds the
// wave total (6 steps = log2 64).
template <class Op>
__device__ __forceinline__ typename Op::T wave_reduce_dpp(typename Op::T v) {
  v = Op::add(v, dpp_move<kQuadPerm1032, 0xF, 0xF>(v));
  v = Op::add(v, dpp_move<kQuadPerm2301, 0xF, 0xF>(v));
  v = Op::add(v, dpp_move<kRowRor4, 0xF, 0xF>(v));
  v = Op::add(v, dpp_move<kRowRor8, 0xF, 0xF>(v));
  v = Op::add(v, dpp_move<kRowBcast15, 0xA, 0xF>(v));
  v = Op::add(v, dpp_move<kRowBcast31, 0xC, 0xF>(v));
  return read_lane(v, 63);
}

// Segmented inclusive scan across the wavefront (reduce-by-key): lane l
// ends with v summed in binary64 over lanes j..l, where j is the last lane
// at or below l whose flag is set (lane 0 if none), and f with the OR of
// the flags of lanes 0..l.  Hillis-Steele inside each 16-lane row (row
// shifts 1, 2, 4, 8), then row 0 into row 1 and row 2 into row 3
// (row_bcast:15), then rows 0-1 into rows 2-3 (row_bcast:31).  A lane whose
// source is invalid receives (0, 0), the identity.  Fixed order, so the
// result is deterministic.  All 64 lanes must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void segscan_step(double& v, int& f) {
  const double pv = dpp_move<CTRL, ROW_MASK, 0xF>(v);
  const int pf = dpp_move<CTRL, ROW_MASK, 0xF>(f);
  v = f ? v : pv + v;
  f = f | pf;
}

__device__ __forceinline__ void wave_segscan(double& v, int& f) {
  segscan_step<kRowShr1, 0xF>(v, f);
  segscan_step<kRowShr2, 0xF>(v, f);
  segscan_step<kRowShr4, 0xF>(v, f);
  segscan_step<kRowShr8, 0xF>(v, f);
  segscan_step<kRowBcast15, 0xA>(v, f);
  segscan_step<kRowBcast31, 0xC>(v, f);
}

// ds_swizzle: xor butterfly (masks 1, 2, 4, 8, 16) inside each 32-lane half
// (bit-mode pattern: and_mask = 0x1F, xor_mask in bits 14:10), then the two
// half totals.
template <class Op>
__device__ __forceinline__ typename Op::T wave_reduce_swizzle(typename Op::T v) {
  v = Op::add(v, swizzle_move<0x1F | (1 << 10)>(v));
  v = Op::add(v, swizzle_move<0x1F | (2 << 10)>(v));
  v = Op::add(v, swizzle_move<0x1F | (4 << 10)>(v));
  v = Op::add(v, swizzle_move<0x1F | (8 << 10)>(v));
  v = Op::add(v, swizzle_move<0x1F | (16 << 10)>(v));
  return Op::add(read_lane(v, 0), read_lane(v, 32));
}

// ds_bpermute: xor butterfly over all 64 lanes (6 steps).
template <class Op>
__device__ __forceinline__ typename Op::T wave_reduce_bpermute(typename Op::T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int k = 1; k < kWave; k <<= 1) v = Op::add(v, bpermute_move(v, lane ^ k));
  return read_lane(v, 0);
}

// ---------------------------------------------------------------------------
// Workgroup combine: per-wave totals -> LDS -> s_barrier -> wave 0 combines.
// Returns the workgroup total in every lane of wave 0 (other waves get
// zero()).  `lds` holds at least kMaxWavesPerWG values.  The caller must
// place a __syncthreads() before reusing `lds`.
// ---------------------------------------------------------------------------
template <class Op>
__device__ __forceinline__ typename Op::T block_reduce(typename Op::T v, typename Op::T* lds) {
  using T = typename Op::T;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int nwaves = blockDim.x / kWave;
  T w = wave_reduce_dpp<Op>(v);
  if (lane == 0) lds[wave] = w;
  __syncthreads();
  T r = Op::zero();
  if (wave == 0) {
    T u = lane < nwaves ? lds[lane] : Op::zero();
    r = wave_reduce_dpp<Op>(u);
  }
  return r;
}

// ---------------------------------------------------------------------------
// Element modes: input type, 16-byte vector, per-thread accumulator, the
// Op of the cross-lane combine and the partial stored per workgroup.
// ---------------------------------------------------------------------------
// int32 -> int64, exact.
struct ModeI32 {
  using In = int32_t;
  using Vec = v4i;
  static constexpr int kVE = 4;
  using Acc = long long;
  using Op = OpI64;
  using Part = long long;
  __device__ static Acc zero() { return 0; }
  __device__ static void add_elem(Acc& a, In x) { a += (long long)x; }
  __device__ static void add_vec(Acc& a, Vec v) {
    a += (long long)v.x;
    a += (long long)v.y;
    a += (long long)v.z;
    a += (long long)v.w;
  }
  __device__ static Part to_part(Acc a) { return a; }
};

// fp32, plain fp32 accumulation.
struct ModeF32Plain {
  using In = float;
  using Vec = v4f;
  static constexpr int kVE = 4;
  using Acc = float;
  using Op = OpF32;
  using Part = double;
  __device__ static Acc zero() { return 0.0f; }
  __device__ static void add_elem(Acc& a, In x) { a += x; }
  __device__ static void add_vec(Acc& a, Vec v) {
    a += v.x;
    a += v.y;
    a += v.z;
    a += v.w;
  }
  __device__ static Part to_part(Acc a) { return (double)a; }
};

// fp32, TwoSum-compensated: every element enters the (s, c) pair through an
// error-free TwoSum, the rounding errors accumulate in c.
struct ModeF32Comp {
  using In = float;
  using Vec = v4f;
  static constexpr int kVE = 4;
  using Acc = CompF32;
  using Op = OpComp;
  using Part = double;
  __device__ static Acc zero() { return CompF32{0.0f, 0.0f}; }
  __device__ static void add_elem(Acc& a, In x) {
    float e;
    two_sum(a.s, x, a.s, e);
    a.c += e;
  }
  __device__ static void add_vec(Acc& a, Vec v) {
    add_elem(a, v.x);
    add_elem(a, v.y);
    add_elem(a, v.z);
    add_elem(a, v.w);
  }
  // s and c are fp32, so their binary64 sum is exact unless c is far below
  // ulp(s); the final combine is in binary64.
  __device__ static Part to_part(Acc a) { return comp_to_double(a); }
};

// 16-bit inputs: exact widening to fp32.
struct Bf16 {
  __device__ static float lo(unsigned w) { return __uint_as_float(w << 16); }
  __device__ static float hi(unsigned w) { return __uint_as_float(w & 0xFFFF0000u); }
  __device__ static float one(uint16_t b) { return __uint_as_float((unsigned)b << 16); }
};
struct F16 {
  __device__ static float lo(unsigned w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xFFFFu));
  }
  __device__ static float hi(unsigned w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
  }
  __device__ static float one(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
};

// 16-bit inputs, compensated: the eight values of a 16-byte vector are
// widened exactly and summed pairwise in fp32 (a sum of 16-bit values is
// exact unless their exponents lie further apart than the fp32 significand
// can bridge; otherwise each of the three levels rounds once), and the
// vector's sum enters the (s, c) pair through one TwoSum.  About 2.75 VALU
// operations per element instead of 5 for a TwoSum per pair.
template <class H>
struct ModeHalfComp {
  using In = uint16_t;
  using Vec = v4u;
  static constexpr int kVE = 8;
  using Acc = CompF32;
  using Op = OpComp;
  using Part = double;
  __device__ static Acc zero() { return CompF32{0.0f, 0.0f}; }
  __device__ static void add_f(Acc& a, float x) {
    float e;
    two_sum(a.s, x, a.s, e);
    a.c += e;
  }
  __device__ static void add_elem(Acc& a, In x) { add_f(a, H::one(x)); }
  __device__ static void add_vec(Acc& a, Vec v) {
    const float p0 = H::lo(v.x) + H::hi(v.x);
    const float p1 = H::lo(v.y) + H::hi(v.y);
    const float p2 = H::lo(v.z) + H::hi(v.z);
    const float p3 = H::lo(v.w) + H::hi(v.w);
    add_f(a, (p0 + p1) + (p2 + p3));
  }
  __device__ static Part to_part(Acc a) { return comp_to_double(a); }
};

// 16-bit inputs, plain fp32 accumulation.
template <class H>
struct ModeHalfPlain {
  using In = uint16_t;
  using Vec = v4u;
  static constexpr int kVE = 8;
  using Acc = float;
  using Op = OpF32;
  using Part = double;
  __device__ static Acc zero() { return 0.0f; }
  __device__ static void add_elem(Acc& a, In x) { a += H::one(x); }
  __device__ static void add_vec(Acc& a, Vec v) {
    a += H::lo(v.x);
    a += H::hi(v.x);
    a += H::lo(v.y);
    a += H::hi(v.y);
    a += H::lo(v.z);
    a += H::hi(v.z);
    a += H::lo(v.w);
    a += H::hi(v.w);
  }
  __device__ static Part to_part(Acc a) { return (double)a; }
};

// Op used to combine stored partials (binary64 for floats, int64 for ints).
template <class Part>
struct PartOp;
template <>
struct PartOp<long long> {
  using type = OpI64;
};
template <>
struct PartOp<double> {
  using type = OpF64;
};

template <bool NT, class Vec>
__device__ __forceinline__ Vec load_vec(const Vec* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Hardware id of the XCD (accelerator complex die) the calling wave runs on
// (the 4-bit XCC_ID hardware register of gfx94x / gfx950).
__device__ __forceinline__ unsigned xcc_id() {
  return (unsigned)__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 0xFu;
}

// ---------------------------------------------------------------------------
// Workspace words of one (device, stream).  Each word that is polled or hit
// by atomics sits on its own 128-byte line.
// ---------------------------------------------------------------------------
constexpr int kMaxBarrierGroups = 32;
constexpr unsigned kTreeFanIn = 64;       // arrivals per first-level node of the XCD tree
constexpr int kMaxTreeClasses = 16;       // residue classes (XCDs) of the XCD tree
constexpr int kMaxTreeNodes = 144;        // first-level nodes: 8192 / kTreeFanIn + kMaxTreeClasses

struct alignas(128) Line {
  unsigned v;
  unsigned pad[31];
};
struct BarrierWords {
  Line count;   // arrivals at the current grid barrier (top level)
  Line gen;     // grid-barrier generation (v, incremented by the last
                // arrival); pad[0]: the generation whose fall-back release
                // the last arrival requests (XCD tree)
  Line ticket;  // atomic-final variant: groups (or workgroups) done, or the XCD tree's top
  Line err;     // watchdog flag (nonzero after a timeout)
  Line group[kMaxBarrierGroups];  // arrivals per group (two-level barrier and ticket)
  Line cls[kMaxTreeClasses];      // XCD tree, second level: node completions per class
  Line node[kMaxTreeNodes];       // XCD tree, first level: arrivals per node
  Line fb;                        // XCD tree: fall-back releases done (v)
};


__device__ __forceinline__ unsigned relaxed_add(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Relaxed device-scope increment that wraps: returns the old value and
// stores old + 1, or 0 when old >= last (the last of last + 1 arrivals
// leaves the counter at zero in the same atomic).
__device__ __forceinline__ unsigned wrap_inc(unsigned* p, unsigned last) {
  return __builtin_amdgcn_atomic_inc32(p, last, __ATOMIC_RELAXED, "agent");
}

// Publication by device-scope atomic stores.  A relaxed agent-scope atomic
// store is coherent across the XCDs (the store carries device scope, so it
// is written through this XCD's L2), so a value published this way needs no
// L2 write-back (buffer_wbl2) before the arrival that announces it: it only
// has to be complete, which a wait on the store counter ensures.  What the
// reader loads after its acquire is then the published value.  Only for
// data that every writer publishes this way.
template <class T>
__device__ __forceinline__ void publish(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads a value stored with publish() by another workgroup (device scope:
// no stale copy in this XCD's L2 is returned).
template <class T>
__device__ __forceinline__ T load_published(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until every store of this wave (published values included) is
// complete; no compiler reordering of memory accesses across it.
__device__ __forceinline__ void drain_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// ---------------------------------------------------------------------------
// XCD-aggregated publication over an arrival tree.
//
// The dispatcher hands workgroups to the XCDs round-robin: within one
// launch workgroup g runs on XCD (g + off) mod nxcc for a launch-wide offset
// off (measured on MI355X), so the workgroups of one residue class
// r = g mod nxcc share one XCD and its L2.  A store is in that L2 once the
// issuing wave's memory counter has drained.  So instead of one L2
// write-back per workgroup (an agent-scope release fence), the workgroups
// of a class drain their stores and count themselves, and the last of the
// class performs ONE agent-scope release (write-back of that L2, which holds
// every member's stores) before it arrives at the top level.
//
// Counting is by workgroup index, so every level completes whatever the
// dispatch; atomics on one line serialize (about 60 ns each on MI355X), so
// the count is a tree:
//   level 1  nodes of kTreeFanIn consecutive members of class r (member
//            j = g / nxcc in node j / kTreeFanIn), one line per node;
//   level 2  the last arrival of each node of class r, on the class line
//            (skipped when the class has one node);
//   level 3  the last arrival of each class, on the top line.
// Measured on MI355X, a level costs about as much as 16 serialized
// arrivals, and the agent-scope acquire that every waiting workgroup needs
// after the barrier (an L2 invalidation, about 56 ns each, queued per XCD)
// dominates beyond that; so nodes hold 64 members, one level per class up
// to 512 workgroups.
//
// The dispatch rule is checked on the way, at no extra atomic: every counter
// is a 64-bit tally that adds (1, k, k^2) for a key k in three fields
// (count: bits 0-15, sum of k: bits 16-31, sum of k^2: bits 32-63).  By the
// Cauchy-Schwarz inequality, count * sum(k^2) = sum(k)^2 exactly when all
// keys are equal.  Keys: the physical XCD (XCC_ID register) at levels 1 and
// 2, the dispatch offset that XCD implies at level 3, and kTreeBad for an
// arrival whose own subtree was not uniform.  The last arrival of the tree
// thus learns whether every workgroup ran on the XCD its class implies; if
// one did not, its stores may sit in another XCD's L2, and the caller falls
// back (the grid barrier asks every workgroup to release on its own).
// ---------------------------------------------------------------------------
constexpr unsigned kErrTimeout = 1u;
constexpr unsigned kBarrierXcd = 0x100u;   // groups value: XCD-aggregated barrier (| nxcc)
constexpr unsigned kBarrierSkew = 0x200u;  // with kBarrierXcd: odd workgroups report the next XCD
                                           // (drives the fall-back from the host in tests)
constexpr unsigned kTreeBad = 15u;         // key of an arrival whose subtree saw two XCDs

// Whether the XCD tree serves a device of nxcc XCDs (more than one, each
// with its own class line and a key below kTreeBad).
__host__ __device__ constexpr bool xcd_tree_fits(int nxcc) {
  return nxcc > 1 && nxcc < (int)kTreeBad && nxcc <= kMaxTreeClasses;
}

__device__ __forceinline__ unsigned long long* tally_word(Line& l) {
  return reinterpret_cast<unsigned long long*>(&l.v);  // v and pad[0]
}

__device__ __forceinline__ unsigned long long tally_term(unsigned k) {
  return 1ull | ((unsigned long long)k << 16) | ((unsigned long long)(k * k) << 32);
}

__device__ __forceinline__ bool tally_uniform(unsigned long long t) {
  const unsigned long long c = t & 0xFFFFull, s1 = (t >> 16) & 0xFFFFull, s2 = t >> 32;
  return c * s2 == s1 * s1;
}

// Adds key k to the tally in `l`; true for the arrival that completes
// `expected` arrivals, which also resets the tally and sets *uniform to
// whether every key of the tally was k, and k is not kTreeBad.
__device__ __forceinline__ bool tally_arrive(Line& l, unsigned k, unsigned expected, bool* uniform) {
  const unsigned long long t =
      __hip_atomic_fetch_add(tally_word(l), tally_term(k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned)(t & 0xFFFFull) != expected - 1) return false;
  __hip_atomic_store(tally_word(l), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *uniform = tally_uniform(t + tally_term(k)) && k != kTreeBad;
  return true;
}

// Counts this workgroup on the XCD tree whose top line is `top`; returns
// true for the one last arrival of the grid, which has then seen every
// workgroup arrive, with *ok telling whether every workgroup ran on the XCD
// its class implies (then, with RELEASE, every class's stores have been
// released; without, the caller's data is published by device-scope atomic
// stores and only the count matters).
// Thread 0 only; every wave of the workgroup must have drained its stores
// (s_waitcnt) before the workgroup barrier that precedes this call.
template <bool RELEASE = true>
__device__ __forceinline__ bool xcd_tree_arrive(BarrierWords* w, Line& top, unsigned nblocks, unsigned groups,
                                                bool* ok) {
  const unsigned nxcc = groups & 0xFFu;
  const unsigned g = blockIdx.x, r = g % nxcc, j = g / nxcc;
  const unsigned members = (nblocks - r + nxcc - 1) / nxcc;  // of class r
  const unsigned nodes = (members + kTreeFanIn - 1) / kTreeFanIn;
  const unsigned node = j / kTreeFanIn;
  const unsigned nsize = members - node * kTreeFanIn < kTreeFanIn ? members - node * kTreeFanIn : kTreeFanIn;
  unsigned key = xcc_id();
  if ((groups & kBarrierSkew) && (g & 1u)) key = (key + 1u) % nxcc;
  if (key >= nxcc) key = kTreeBad;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  bool u = true;
  if (!tally_arrive(w->node[r + nxcc * node], key, nsize, &u)) return false;
  if (!u) key = kTreeBad;
  if (nodes > 1) {
    if (!tally_arrive(w->cls[r], key, nodes, &u)) return false;
    if (!u) key = kTreeBad;
  }
  // The class is complete: one write-back of this XCD's L2 publishes the
  // stores of every member that ran here.  Either way the resets of the
  // lines below complete before the arrival above (a barrier reuses them).
  if constexpr (RELEASE)
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
  else
    drain_stores();
  const unsigned off = key == kTreeBad ? kTreeBad : (key + nxcc - r) % nxcc;
  const unsigned active = nblocks < nxcc ? nblocks : nxcc;
  if (!tally_arrive(top, off, active, &u)) return false;
  *ok = u;
  return true;
}

// ---------------------------------------------------------------------------
// Grid barrier for a launch of `nblocks` co-resident workgroups.
//
// Sense-reversing barrier in three shapes (`groups`):
//   1        flat: every workgroup releases (one L2 write-back) and
//            increments the single counter;
//   2..32    two-level: the first level counts the workgroups with equal
//            blockIdx.x % groups (each still releasing on its own), the
//            last of a group acquires and increments the top counter;
//   kBarrierXcd | nxcc
//            XCD-aggregated: the arrival tree above, one L2 write-back per
//            XCD.  When the tree reports a workgroup off its class's XCD,
//            the last arrival requests a fall-back before it opens the
//            barrier: every other workgroup, still waiting, releases its
//            own stores and acknowledges on the `fb` line; the last arrival
//            waits for all acknowledgements (bounded like every wait here).
// Thread 0 of each workgroup keeps the generation in `gen` (read once per
// launch with grid_barrier_gen, then advanced by each barrier, so no
// barrier waits for a load of it before arriving); the counters of the
// flat and two-level shapes wrap to zero on their last arrival (the XCD
// tree's tallies are reset by theirs); the last top-level arrival
// acquires, releases and bumps the generation;
// the others poll it with relaxed device-scope loads (s_sleep between
// polls, so polling neither invalidates the L2 nor floods the atomic unit)
// and acquire once after the wait.  Each hop is a release / relaxed RMW /
// acquire chain, so every workgroup's stores happen before every
// workgroup's loads after the barrier.  Every wait is bounded by
// `spin_limit` polls: on expiry the workgroup sets the error word and
// leaves, so the kernel always ends (a grid in which not every block
// arrives deadlocks, Section VIII-B of the paper).  Counters are back at
// zero after every completed barrier.  Returns false on timeout.
// ---------------------------------------------------------------------------
// The barrier generation at the start of a launch, for thread 0 of each
// workgroup to pass to its grid_barrier calls.  A barrier completes only
// once every workgroup has arrived, so every workgroup that reads this
// before its first arrival reads the same value.
__device__ __forceinline__ unsigned grid_barrier_gen(BarrierWords* w) {
  return threadIdx.x == 0 ? __hip_atomic_load(&w->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
}

// How a grid barrier passes data between workgroups.
enum BarrierMode {
  // Ordinary stores before, ordinary loads after: every arrival releases
  // (on the XCD tree, one L2 write-back per XCD, with the fall-back below),
  // every workgroup acquires after the wait.
  kBarFenced = 0,
  // One-sided: only the workgroups with `waiter` set wait (and acquire);
  // what they read was stored with publish() and drained, so no arrival
  // releases and no fall-back is needed (nor possible: the others may have
  // left).
  kBarOneSided = 1,
  // Two-sided, with every value that crosses the barrier stored with
  // publish() (drained before the arrival) and loaded with a device-scope
  // atomic load: no workgroup releases or acquires.
  kBarPublished = 2,
};

// Thread 0's part of one grid barrier: arrive, then open the barrier (last
// arrival) or wait for it; returns 1 on timeout.  One polling loop serves
// the waiting workgroups and, during a fall-back, the last arrival (which
// then waits for the other workgroups' release acknowledgements before it
// opens the barrier); a second loop for the last arrival raised the
// register count of the persistent kernels that hold 8 loads per lane
// from 59 to 107 VGPRs.  `waiter` matters in kBarOneSided only.
template <int MODE = kBarFenced>
__device__ __forceinline__ int grid_barrier_thread0(BarrierWords* w, unsigned nblocks, unsigned groups,
                                                    unsigned spin_limit, unsigned g, bool waiter = true) {
  constexpr bool ONE_SIDED = MODE == kBarOneSided;
  constexpr bool FENCED = MODE == kBarFenced;
  const bool xcd = (groups & kBarrierXcd) != 0;
  int to = 0;
  bool last = false, ok = true;
  if (xcd) {
    last = xcd_tree_arrive<FENCED>(w, w->count, nblocks, groups, &ok);
  } else {
    if constexpr (FENCED) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // Counters wrap to zero on their last arrival (atomic increment with a
    // limit), so no reset store has to complete before the next barrier.
    if (groups <= 1) {
      last = wrap_inc(&w->count.v, nblocks - 1) == nblocks - 1;
    } else {
      const unsigned grp = blockIdx.x % groups;
      const unsigned members = (nblocks - grp + groups - 1) / groups;
      const unsigned active = nblocks < groups ? nblocks : groups;
      if (wrap_inc(&w->group[grp].v, members - 1) == members - 1) {
        if constexpr (FENCED) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        last = wrap_inc(&w->count.v, active - 1) == active - 1;
      }
    }
  }
  // The last arrival opens the barrier now, or after a fall-back: it asks
  // every other workgroup to release its own stores, then waits below for
  // their acknowledgements.
  const bool fallback = FENCED && last && !ok && nblocks > 1;
  if (ONE_SIDED && !last && !waiter) return 0;
  if (fallback) __hip_atomic_store(&w->gen.pad[0], g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!last || fallback) {
    unsigned spins = 0;
    bool released = false;
    for (;;) {
      if (fallback) {
        if (__hip_atomic_load(&w->fb.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1) break;
      } else {
        unsigned cur, req;
        if (xcd) {
          const unsigned long long both = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&w->gen.v),
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          cur = (unsigned)both;
          req = (unsigned)(both >> 32);
        } else {
          cur = __hip_atomic_load(&w->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          req = 0u;
        }
        if (cur != g) break;
        if (xcd && !released && req == g + 1u) {  // fall-back requested for this barrier
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          relaxed_add(&w->fb.v, 1u);
          released = true;
        }
      }
      if (++spins > spin_limit) {
        __hip_atomic_store(&w->err.v, kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        to = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (fallback) __hip_atomic_store(&w->fb.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (last) {
    // Published data: nothing to pass on; the XCD tree's line resets
    // complete first.
    if constexpr (FENCED)
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    else
      drain_stores();
    relaxed_add(&w->gen.v, 1u);
  }
  if (FENCED || (ONE_SIDED && waiter)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return to;
}

// One-sided grid barrier: every workgroup arrives, and only the workgroups
// with `waiter` set wait for all arrivals and acquire; the others return at
// once (they must not read what other workgroups stored before the
// barrier).  What the waiters read must have been stored with publish():
// every wave drains its stores before the workgroup barrier that precedes
// the arrival, so no arrival writes back an L2 and no XCD placement
// matters.  For a persistent reduction whose workgroup 0 alone combines
// the partials: the other workgroups skip the L2 write-back, the wait and
// the agent-scope acquire (write-backs and invalidations queue up per XCD).
// `waiter` is uniform across the workgroup.  Returns false on timeout
// (waiters).
__device__ __forceinline__ bool grid_barrier_to(BarrierWords* w, unsigned nblocks, unsigned groups,
                                                unsigned spin_limit, unsigned& gen, bool waiter) {
  __shared__ int timed_out;
  drain_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    timed_out = grid_barrier_thread0<kBarOneSided>(w, nblocks, groups, spin_limit, gen, waiter);
    gen = gen + 1u;
  }
  __syncthreads();
  return timed_out == 0;
}

// Grid barrier for data that crosses it only by publish() and device-scope
// atomic loads (kBarPublished): no L2 write-back at any arrival and no L2
// invalidation after the wait.  Returns false on timeout.
__device__ __forceinline__ bool grid_barrier_published(BarrierWords* w, unsigned nblocks, unsigned groups,
                                                       unsigned spin_limit, unsigned& gen) {
  __shared__ int timed_out;
  drain_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    timed_out = grid_barrier_thread0<kBarPublished>(w, nblocks, groups, spin_limit, gen);
    gen = gen + 1u;
  }
  __syncthreads();
  return timed_out == 0;
}

__device__ __forceinline__ bool grid_barrier(BarrierWords* w, unsigned nblocks, unsigned groups,
                                             unsigned spin_limit, unsigned& gen) {
  __shared__ int timed_out;
  // Every wave drains its own stores first, so they are in its XCD's L2
  // when thread 0's release writes that L2 back (the stores of a workgroup
  // may come from any of its waves).
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    timed_out = grid_barrier_thread0(w, nblocks, groups, spin_limit, gen);
    gen = gen + 1u;
  }
  __syncthreads();
  return timed_out == 0;
}

// Default number of barrier groups for a grid of n workgroups: flat below
// 64 workgroups, else a multiple of 8 (whole XCDs) giving about 64 members
// per group, between 8 and kMaxBarrierGroups.
__host__ __device__ inline unsigned default_barrier_groups(unsigned n) {
  if (n < 64) return 1u;
  unsigned g = ((n / 64 + 7) / 8) * 8;  // about 64 members per group
  return g < 8u ? 8u : (g > (unsigned)kMaxBarrierGroups ? (unsigned)kMaxBarrierGroups : g);
}

}  // namespace redsum
