// Index-build launchers (sj_index.hip).
#pragma once

#include "sj_internal.hpp"

namespace sj {

constexpr int kKeyMaxDims = 16;  // most dimensions one linearised cell key covers

constexpr int kFineMaxDims = 16;

// Sort key of a point: (cell key << fine_bits) | fine key.
// Cell key: sum over r < k of c_r * mult[r], with
// c_r = clamp(floor(((double)x[dim[r]] - org[r]) / w), 0, cmax[r]).
// Fine key: Morton interleave of fb-bit coordinates of the first fm
// reordered dimensions over their bounding box, so that points of a cell
// are laid out along a space-filling curve (consecutive positions are near
// each other).
struct KeyParams {
  uint32_t k;
  uint32_t dim[kKeyMaxDims];
  double org[kKeyMaxDims];
  uint64_t mult[kKeyMaxDims];
  uint64_t cmax[kKeyMaxDims];
  double w;
  uint32_t fm, fb;                 // fine dimensions and bits per dimension
  uint32_t fdim[kFineMaxDims];
  double forg[kFineMaxDims], fscale[kFineMaxDims];
};

// Decoding and neighbour search over the cell-key table.
struct NbrParams {
  uint32_t k;
  uint64_t mult[kKeyMaxDims];
  uint64_t m[kKeyMaxDims];  // cells along each indexed dimension
  uint64_t n_off;           // 3^k
  uint32_t nfence;          // LDS fence entries
  uint32_t fstride;         // table entries per fence entry (1: whole table in LDS)
};

void launch_minmax(const float *P, uint64_t n, uint32_t d, uint32_t *gmin, uint32_t *gmax,
                   uint32_t *bad, hipStream_t s);
// var[t] = sample variance, var[d + t] = sample mean of dimension t over the
// rows 0, stride, 2 stride, ... (m rows).
void launch_variance(const float *P, uint32_t d, uint64_t stride, uint64_t m, double *var,
                     hipStream_t s);
void launch_cellkey(const float *P, uint64_t n, uint32_t d, const KeyParams &kp, uint64_t *keys,
                    uint32_t *ids, hipStream_t s);
// Sort keys of query points Q [m][d] in an indexed set's grid kp; queries
// outside [lo_t, hi_t] in some dimension t get far_key (see k_query_keys),
// and *n_far (device, zeroed by the caller) counts them.
void launch_query_keys(const float *Q, uint64_t m, uint32_t d, const KeyParams &kp,
                       const double *lo, const double *hi, uint64_t far_key, uint64_t *keys,
                       uint32_t *ids, unsigned long long *n_far, hipStream_t s);
void launch_gather(const float *P, uint64_t n, uint32_t d, uint32_t dp, const uint32_t *perm,
                   const uint32_t *sorted_ids, float *X, uint32_t *orig_id, uint32_t *pos_of,
                   hipStream_t s);
// Non-empty cells of sorted keys (cell part = key >> fine_shift).
void launch_compact(const uint64_t *keys, uint64_t n, uint32_t fine_shift, uint32_t *flag_tmp,
                    uint32_t *d_ncell, uint64_t *cell_key, uint32_t *cell_start, void *scan_tmp,
                    hipStream_t s);
// Adjacent non-empty cells of the query cells qkey[0 .. nq) in the table
// cell_key[0 .. ncell) (qkey = cell_key, nq = ncell in a self-join).
void launch_neighbors(int pass, const uint64_t *qkey, uint64_t nq, const uint64_t *cell_key,
                      const uint32_t *cell_start, uint64_t ncell, const NbrParams &np,
                      uint32_t *nbr_count, uint64_t *cand_sum, const uint32_t *nbr_off,
                      uint32_t *nbr_cell, hipStream_t s);
void launch_runs(int pass, int sym, uint64_t ncell, const uint32_t *cell_start,
                 const uint32_t *nbr_off, const uint32_t *nbr_cell, uint32_t *run_count,
                 const uint32_t *run_off, uint2 *runs, hipStream_t s);
// Union runs of groups of at most kGroupMaxCells consecutive cells (two
// passes: count into gcount, then write at the scanned offsets goff).
constexpr uint32_t kGroupMaxCells = 3;
void launch_group_runs(int pass, uint64_t ngroup, const uint32_t *gfirst, const uint32_t *run_off,
                       const uint2 *runs, uint32_t *gcount, const uint32_t *goff, uint2 *gruns,
                       hipStream_t s);
// Work units in three steps: per cell (query blocks, run total), per query
// block (units, evaluated pairs), per query block (fill).  With per_block,
// run_off / run_total are indexed by query block (each block has runs of
// its own, the SORTIDU ranges) instead of by cell.
void launch_wu_cells(uint64_t ncell, uint32_t tq, const uint32_t *cell_start,
                     const uint32_t *qlist, uint64_t nq, const uint32_t *run_off,
                     const uint2 *runs, uint32_t *nqb, uint64_t *run_total, hipStream_t s);
void launch_wu_count(uint64_t nqb_total, int sym, uint64_t ncell, uint32_t tq, uint32_t tc,
                     const uint32_t *cell_start, const uint32_t *qlist, uint64_t nq,
                     const uint32_t *qb_off, const uint32_t *run_off, const uint2 *runs,
                     const uint64_t *run_total, uint32_t *units, uint64_t *eval, hipStream_t s,
                     int per_block = 0);
void launch_wu_fill(uint64_t nqb_total, int sym, uint64_t ncell, uint32_t tq, uint32_t tc,
                    const uint32_t *cell_start, const uint32_t *qlist, uint64_t nq,
                    const uint32_t *qb_off, const uint32_t *run_off, const uint2 *runs,
                    const uint64_t *run_total, const uint32_t *unit_off, WorkUnit *wu,
                    uint64_t *order_key, hipStream_t s, int per_block = 0);
// SORTIDU search along u (Section 4.3) for blocks of queries.
struct USearch {
  uint32_t ur, dp;   // reordered column of u in the query rows, row stride
  uint64_t fmask;    // fine (quantised u) part of a sort key
  double org, scale; // quantisation of u, as in the sort key
  uint32_t fmax;
  double eps;
};
// Per query block t of contiguous query slots (blocks as in the work units:
// qb_off over the query cells, tq slots each): its candidate ranges in the
// adjacent cells of the indexed side (nbr_off / nbr_cell into ecell_start,
// sorted keys ekey), restricted to the points within eps of the block's
// u-range, ranges that touch merged; sym keeps cells B >= A and starts A's
// own range at the block's first query.  pass 0: rcount[t] ranges of
// rlen[t] candidates; pass 1: the ranges from roff[t].
void launch_qb_ranges(int pass, int sym, uint64_t nqb_total, uint64_t ncell, uint32_t tq,
                      const uint32_t *cell_start, const uint32_t *qb_off,
                      const uint32_t *nbr_off, const uint32_t *nbr_cell,
                      const uint32_t *ecell_start, const uint64_t *ekey, const float *Xq,
                      const USearch &us, uint32_t *rcount, uint64_t *rlen,
                      const uint32_t *roff, uint2 *ranges, hipStream_t s);
// dst[i] = src[(uint32_t)keys[i]] (work units in the order of sorted keys)
void launch_gather_wu(const WorkUnit *src, const uint64_t *keys, uint64_t n, WorkUnit *dst,
                      hipStream_t s);
void launch_cell_products(uint64_t ncell, const uint32_t *cell_start, const uint64_t *cand_sum,
                          uint64_t *out, hipStream_t s);
// out[A] = ceil(|A| / tq) * tq * cand_sum[A] (lane work of A's units of tq
// query slots, idle slots included)
void launch_cell_slot_work(uint64_t ncell, const uint32_t *cell_start, const uint64_t *cand_sum,
                           uint32_t tq, uint64_t *out, hipStream_t s);

// counts[i] += number of keys (i << 32 | .) among the sorted keys
// [0, count) (counts zeroed by the caller; chunks may be added one by one).
void launch_row_counts(const uint64_t *keys, uint64_t count, unsigned long long *counts,
                       hipStream_t s);

}  // namespace sj
