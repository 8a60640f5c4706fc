// Matrix-core distance filter (sj_mfma.hip).
#pragma once

#include "sj_internal.hpp"

namespace sj {

constexpr int kFmtF16 = 0;
constexpr int kFmtBF16 = 1;

// Constants of the error band (see k_mfma_thresholds).
struct MfmaBand {
  double u;          // relative error of centring + quantisation per coordinate
  double eta_term;   // 2 * flush threshold * sqrt(d)
  double gamma_acc;  // gamma_K(2^-23) of the FP32 accumulation
  double s_hi, s_lo; // eps2/(1-g64), eps2/(1+g64)
};

// Everything a work unit of the matrix-core filter reads.
struct MfmaView {
  const void *XA, *XB;      // [n_pad][kp] 16-bit operands (candidate rows / query columns)
  const float *cn;          // [n_pad] candidate norms, the MFMA's initial accumulator
  const float *thi, *tlo;   // per-point thresholds
  const float *X;           // FP32 candidate rows (recheck)
  const float *Xq;          // FP32 query rows (X itself in a self-join)
  const uint16_t *inv_perm;
  const uint2 *runs;
  const uint32_t *qlist;    // query positions, or null for contiguous slots
  uint32_t d, dp;
  double eps2;
  int symmetric;
  uint32_t pshift;          // key = key_hi | pos_q << pshift | pos_c
  uint64_t key_hi;
  // Deferred FP64 rechecks: band pairs (pos_q << 32 | pos_c) are appended
  // here and rechecked by launch_band_recheck; null: rechecked in place.
  uint64_t *band;
  uint64_t band_cap;
  unsigned long long *band_cursor;
  // Query-box prefilter of the workgroup kernel: `hi` is the FP32 reject
  // threshold of a sum of at most dp squared differences (the FP32
  // filter's); pad_row is a candidate row with zero operands and norm +inf.
  float hi;
  uint32_t pad_row;
};

struct MfmaLaunch {
  int fmt;
  uint32_t kp;
  MfmaView view;
  const WorkUnit *wu;
  uint64_t n_wu;
  uint64_t *out;
  uint64_t capacity;
  unsigned long long *cursor, *rechecks;
  int per_wave;  // 1: one wave per work unit (units of mfma_wave_queries())
  int hits_frequent;  // 1: most tiles hold a result or band pair (no per-tile minimum first)
  int box;            // workgroup units: candidates tested against the query box first
};

// One job of a batched launch.
struct BatchJob {
  MfmaView view;
  const uint32_t *orig_id;
  int32_t variant;  // instantiation (K padding, format) of the batched kernel
  uint32_t pad;
};

uint32_t mfma_kp(uint32_t d);
int mfma_qb(uint32_t kp);
// Query slots of one work unit of the single-join matrix kernel (a whole
// workgroup); the batched kernel uses 32*mfma_qb per wave.
uint32_t mfma_wg_queries(uint32_t kp);
// Query slots of one work unit of the per-wave single-join kernel.
uint32_t mfma_wave_queries();
void launch_mfma_prep(int fmt, const float *X, uint64_t n, uint64_t n_pad, uint32_t d, uint32_t dp,
                      uint32_t kp, const float *centre, void *XA, void *XB, float *cn,
                      double *norm2, double *dist_c, double *fold_err,
                      unsigned long long *maxima, hipStream_t s);
void launch_mfma_thresholds(uint64_t n, uint64_t n_pad, const MfmaBand &band, const double *norm2,
                            const double *dist_c, const unsigned long long *maxima, float *thi,
                            float *tlo, hipStream_t s);
// Emits keys of cell-order positions (launch_pos_to_id maps them to
// caller indices in place).
// Rechecks the band pairs collected by a launch with view.band set (their
// count is read on the device, at most view.band_cap) and appends the
// accepted ones to out like the join does; *rechecks += their count.
void launch_band_recheck(const MfmaView &v, uint64_t *out, uint64_t capacity,
                         unsigned long long *cursor, unsigned long long *rechecks, hipStream_t s);
void launch_join_mfma(const MfmaLaunch &a, hipStream_t s);
void launch_pos_to_id(uint64_t *keys, uint64_t count, const uint32_t *qid,
                      const uint32_t *orig_id, hipStream_t s);

// Batched path: variant index of (kp, fmt), or -1 when kp is not supported
// (kp <= 80); workgroups per CU the persistent kernel fits.
int batched_variant(uint32_t kp, int fmt);
int batched_blocks_per_cu();
void launch_join_batched(const BatchJob *jobs, const WorkUnit *wus, uint64_t n_wu, uint32_t grab,
                         unsigned int *queue, uint64_t *out, const unsigned long long *capacity,
                         unsigned long long *cursor, unsigned long long *rechecks, uint32_t grid,
                         uint64_t *band, uint64_t band_cap, unsigned long long *band_cursor,
                         hipStream_t s);
// Deferred FP64 recheck of the band list of a batched launch (band == null
// in launch_join_batched: rechecked in place instead).
void launch_band_recheck_batched(const BatchJob *jobs, const uint64_t *band,
                                 const unsigned long long *band_count, uint64_t band_cap,
                                 uint64_t *out, const unsigned long long *capacity,
                                 unsigned long long *cursor, unsigned long long *rechecks,
                                 uint32_t grid, hipStream_t s);
void launch_pos_to_id_batched(uint64_t *keys, const unsigned long long *count,
                              const unsigned long long *capacity, const BatchJob *jobs,
                              uint32_t grid, hipStream_t s);
void launch_job_bounds(const uint64_t *keys, const unsigned long long *count,
                       const unsigned long long *capacity, unsigned long long *first,
                       unsigned long long *last, uint32_t grid, hipStream_t s);

}  // namespace sj
