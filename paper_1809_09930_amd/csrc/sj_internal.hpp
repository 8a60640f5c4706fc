// Internal declarations shared by the translation units of libselfjoin.
// Everything here is gfx950 (CDNA4, wave64) code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "../../include/selfjoin.h"

namespace sj {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // 4 waves per workgroup everywhere
constexpr int kWavesPerBlock = kBlock / kWave;

// A library error carried as an exception inside the library only; the C ABI
// converts it into a return code plus the thread-local message.
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define SJ_HIP(call) ::sj::check_hip((call), #call)

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of `mask` in lanes below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  uint32_t lo = uniform_u32((uint32_t)v), hi = uniform_u32((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Canonical predicate of Section 3.1 on positions of cell-ordered rows: row a
// of XA against row b of XB (rows of dp floats in the reordered dimension
// order), summed in binary64 in the caller's dimension order (inv_perm maps a
// caller dimension to its reordered position), every operation separately
// rounded (no contraction), accepted iff the sum is <= eps2.  Every device
// filter sends the pairs it cannot decide here, so this is the one place the
// include/exclude decision is taken in FP64.
// The body is inlined into the kernels that do nothing but recheck (one pair
// per lane), with the loop unrolled U times so that the loads of several
// dimensions are in flight together; unrolling keeps the order of the
// additions.  The join kernels call it out of line and not unrolled
// (SJ_RECHECK_INLINE), as their rare band lanes would otherwise carry its
// registers everywhere.
template <int U>
static __device__ __forceinline__ bool canonical_within_body(const float *__restrict__ XA,
                                                             uint32_t a,
                                                             const float *__restrict__ XB,
                                                             uint32_t b,
                                                             const uint16_t *__restrict__ inv_perm,
                                                             uint32_t d, uint32_t dp, double eps2) {
#pragma clang fp contract(off)
  const float *pa = XA + (uint64_t)a * dp;
  const float *pb = XB + (uint64_t)b * dp;
  double acc = 0.0;
#pragma unroll U
  for (uint32_t t = 0; t < d; ++t) {
    const uint32_t r = inv_perm[t];
    const double diff = (double)pa[r] - (double)pb[r];
    const double sq = diff * diff;
    acc = acc + sq;
  }
  return acc <= eps2;
}
#ifndef SJ_RECHECK_INLINE
#define SJ_RECHECK_INLINE __noinline__
#endif
static __device__ SJ_RECHECK_INLINE bool canonical_within(const float *__restrict__ XA, uint32_t a,
                                                          const float *__restrict__ XB, uint32_t b,
                                                          const uint16_t *__restrict__ inv_perm,
                                                          uint32_t d, uint32_t dp, double eps2) {
  return canonical_within_body<1>(XA, a, XB, b, inv_perm, d, dp, eps2);
}

// float <-> order-preserving uint32 (for atomic min/max of finite floats)
__device__ __host__ __forceinline__ uint32_t float_to_ordered(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __host__ __forceinline__ float ordered_to_float(uint32_t u) {
  uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __builtin_bit_cast(float, b);
}

// ---------------------------------------------------------------------------
// Work units of the distance kernels.
//
// A work unit pairs a block of up to 64*RQ query points of one cell A with a
// stretch of A's candidate runs.  A run is a maximal range of consecutive
// non-empty cells adjacent to A; since points are stored grouped by cell in
// cell order, a run is one contiguous range of point positions [c0, c1).
// The unit covers runs run_first..run_last, starting at c_begin inside the
// first and ending at c_end inside the last.
// ---------------------------------------------------------------------------
struct WorkUnit {
  uint32_t q0, q1;          // query slots [q0, q1): positions, or indices into a query list
  uint32_t run_first, run_last;
  uint32_t c_begin, c_end;  // candidate position bounds inside the first / last run
  uint32_t cell;            // query cell A
  uint32_t pad;
};
static_assert(sizeof(WorkUnit) == 32, "WorkUnit layout");

// ---------------------------------------------------------------------------
// Primitives (sj_prims.hip)
// ---------------------------------------------------------------------------
// Exclusive prefix sum of n values in place-or-out; returns the total through
// *d_total (device) when non-null.  `tmp` is scratch from scan_tmp_bytes().
size_t scan_tmp_bytes(uint64_t n);
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n,
                        uint32_t *d_total, void *tmp, hipStream_t s);
void exclusive_scan_u64(const uint64_t *in, uint64_t *out, uint64_t n,
                        uint64_t *d_total, void *tmp, hipStream_t s);

// Stable LSD radix sort of 64-bit keys (optionally with 32-bit values) over
// the bit ranges listed in `shifts`: digits of widths[p] bits (1..8; 8 when
// widths is null) at each shift.  Sorted output ends in keys[0]/vals[0];
// keys[1]/vals[1] are the ping-pong buffers.
// With d_count non-null, n is the capacity that sizes the launches and only
// the first min(*d_count, n) keys are sorted (for captured graphs, where
// the count is known on the device only).
size_t radix_tmp_bytes(uint64_t n);
void radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], uint64_t n,
                    const int *shifts, int n_passes, void *tmp, hipStream_t s,
                    const unsigned long long *d_count = nullptr,
                    const int *widths = nullptr);
void launch_fill_u64(unsigned long long *p, uint64_t count, unsigned long long v, hipStream_t s);

// out[i] = (i / run) * stride + i % run (runs of `run` consecutive values,
// stride >= run apart); widen u32 -> u64; narrow u64 -> u32 (low half).
void launch_iota_strided(uint32_t *out, uint64_t count, uint64_t stride, uint32_t run,
                         hipStream_t s);
void launch_widen(const uint32_t *in, uint64_t *out, uint64_t count, hipStream_t s);
void launch_narrow(const uint64_t *in, uint32_t *out, uint64_t count, hipStream_t s);

// ---------------------------------------------------------------------------
// Index build (sj_index.hip)
// ---------------------------------------------------------------------------
struct DeviceIndex;  // defined in sj_index.hip

// ---------------------------------------------------------------------------
// Distance kernels (sj_join.hip)
// ---------------------------------------------------------------------------
struct JoinLaunch {
  const float *X;           // [n][dp] points in cell order, reordered dims, zero padded
  const uint32_t *orig_id;  // [n] position -> caller index
  const float *Xq;          // query rows (X itself in a self-join), same layout
  const uint32_t *qid;      // query position -> caller query index
  const uint16_t *inv_perm; // [d] caller dim t -> reordered position
  const WorkUnit *wu;
  uint64_t n_wu;
  const uint2 *runs;
  const uint32_t *qlist;    // query positions (indirect mode) or null
  uint32_t d, dp;
  float lo, hi;             // FP32 accept / reject thresholds (band between them)
  double eps2;              // canonical threshold
  int symmetric;            // 1: emit both orders, only qpos <= cpos
  int count_only;           // 1: count pairs with s <= hi, emit nothing
  int shortc;
  uint64_t *out;            // pair keys (i << 32 | j)
  uint64_t capacity;
  unsigned long long *cursor;    // pairs produced (may exceed capacity)
  unsigned long long *rechecks;  // FP64 rechecks performed
  int rq;                   // queries per lane (1, 2 or 4; fp32_rq_for); units hold 64*rq queries
  int norm;                 // 1: norm form with the tables QA / CR
  const float *QA, *CR;     // [.][norm_table_row(dp)] query (of Xq) / candidate (of X) tables
  uint32_t skip_below;      // candidates with caller index below this are skipped (0: none)
  unsigned long long *skipped;  // += skipped candidates x live queries of the wave
};

// Queries per lane the FP32 kernel uses for padded dimension dp.
// (1 when small_cells: the units of small cells use one query per lane.)
int fp32_rq_for(uint32_t dp, bool norm, bool small_cells);
// Floats per point in each norm-form table.
int norm_table_row(uint32_t dp);
// Builds the norm-form tables of the cell-ordered rows X ([n][dp]) for the
// bounds s_hi / s_lo and margin factor kappa; *nsum += sum of squared norms.
void launch_norm_tables(const float *X, uint64_t n, uint32_t dp, double s_hi, double s_lo,
                        double kappa, float *QA, float *CR, double *nsum, hipStream_t s);
// Padded dimension count the kernels support for d (0 if unsupported).
uint32_t padded_dim(uint32_t d);
void launch_join_fp32(const JoinLaunch &a, hipStream_t s);

// Symmetric result batches over caller-index ranges (the batch of queries
// [i0, i1) runs after every batch below i0).  k_mirror_split takes the
// batch's join output (i << 32 | j, every j >= i0) and keeps (i, j) when
// j >= i; for j > i it adds the mirror (j, i) to `out` when j < i1, else to
// `spill` (a later batch's pair).  k_spill_take moves the spilled pairs with
// i < i1 from `spill_in` to `out` and the rest to `spill_out`.  Slots are
// taken with one atomic per block of 16,384 entries and stream; counts
// beyond a capacity are still counted.
void launch_mirror_split(const uint64_t *in, uint64_t n, uint32_t i1, uint64_t *out,
                         unsigned long long *out_cnt, uint64_t out_cap, uint64_t *spill,
                         unsigned long long *spill_cnt, uint64_t spill_cap, hipStream_t s);
void launch_spill_take(const uint64_t *spill_in, uint64_t n, uint32_t i1, uint64_t *out,
                       unsigned long long *out_cnt, uint64_t out_cap, uint64_t *spill_out,
                       unsigned long long *spill_cnt, uint64_t spill_cap, hipStream_t s);

// Unpack sorted keys [first, first+count) to (i, j) columns and optionally
// recompute FP32 distances.
// Keys are (i << ishift) | j with both fields `ishift` bits wide; i is a
// row of the query points (Xq, qpos_of), j of the indexed points (X, pos_of).
void launch_unpack(const uint64_t *keys, uint64_t count, uint32_t *out_i,
                   uint32_t *out_j, float *out_dist, const float *Xq,
                   const uint32_t *qpos_of, const float *X, const uint32_t *pos_of,
                   const uint16_t *inv_perm, uint32_t d, uint32_t dp, hipStream_t s,
                   uint32_t ishift = 32);

}  // namespace sj
