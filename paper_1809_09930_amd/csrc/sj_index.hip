// Grid index build on the device (Section 3.2.1 grid index, Section 4.1
// indexing k of the n dimensions, Section 4.2 variance reorder):
//   ingest/validate -> per-dimension min/max, sample variance -> cell keys
//   over the first k reordered dimensions -> radix sort by key -> gather the
//   points in cell order (reordered, zero-padded rows) -> compact the
//   non-empty cells -> adjacent cells by binary search in an LDS-staged key
//   table -> candidate runs -> work units for the distance kernels.
#include "sj_index.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace sj {

namespace {

// ---------------------------------------------------------------------------
// a1: per-dimension min/max of the caller's rows and a non-finite flag.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_minmax(const float *__restrict__ P, uint64_t total,
                                                   uint32_t d, uint32_t *__restrict__ gmin,
                                                   uint32_t *__restrict__ gmax,
                                                   uint32_t *__restrict__ bad) {
  __shared__ uint32_t smin[SJ_MAX_DIM], smax[SJ_MAX_DIM];
  __shared__ uint32_t sbad;
  for (uint32_t t = threadIdx.x; t < d; t += kBlock) {
    smin[t] = 0xffffffffu;
    smax[t] = 0u;
  }
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint32_t step = (uint32_t)(stride % d);
  uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t t = (uint32_t)(e % d);
  uint32_t lmin = 0xffffffffu, lmax = 0u;
  uint32_t lt = t;  // dimension the local min/max belongs to (only when step == 0)
  for (; e < total; e += stride) {
    const float v = P[e];
    if (!__builtin_isfinite(v)) {
      sbad = 1;
    } else {
      const uint32_t u = float_to_ordered(v);
      if (step == 0) {
        lmin = min(lmin, u);
        lmax = max(lmax, u);
      } else {
        atomicMin(&smin[t], u);
        atomicMax(&smax[t], u);
      }
    }
    t += step;
    if (t >= d) t -= d;
  }
  if (step == 0 && lmax != 0u) {
    atomicMin(&smin[lt], lmin);
    atomicMax(&smax[lt], lmax);
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < d; q += kBlock) {
    if (smax[q] != 0u) {
      atomicMin(&gmin[q], smin[q]);
      atomicMax(&gmax[q], smax[q]);
    }
  }
  if (threadIdx.x == 0 && sbad) atomicOr(bad, 1u);
}

__global__ void k_init_minmax(uint32_t *gmin, uint32_t *gmax, uint32_t *bad, uint32_t d) {
  for (uint32_t t = threadIdx.x; t < d; t += blockDim.x) {
    gmin[t] = 0xffffffffu;
    gmax[t] = 0u;
  }
  if (threadIdx.x == 0) *bad = 0u;
}

// ---------------------------------------------------------------------------
// a2: variance of every dimension over a strided sample (one workgroup per
// dimension, fixed-order reductions: deterministic).
// ---------------------------------------------------------------------------
__device__ double block_sum_f64(double v) {
  __shared__ double red[kBlock];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kBlock) void k_variance(const float *__restrict__ P, uint32_t d,
                                                     uint64_t stride, uint64_t m,
                                                     double *__restrict__ var) {
  const uint32_t t = blockIdx.x;
  double s = 0.0;
  for (uint64_t i = threadIdx.x; i < m; i += kBlock) s += (double)P[i * stride * d + t];
  const double mean = block_sum_f64(s) / (double)m;
  double q = 0.0;
  for (uint64_t i = threadIdx.x; i < m; i += kBlock) {
    const double x = (double)P[i * stride * d + t] - mean;
    q += x * x;
  }
  const double ss = block_sum_f64(q);
  if (threadIdx.x == 0) {
    var[t] = m > 1 ? ss / (double)(m - 1) : 0.0;
    var[d + t] = mean;
  }
}

// ---------------------------------------------------------------------------
// a3: linearised cell key over the first k reordered dimensions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sort_key(const float *__restrict__ x, const KeyParams &kp) {
  uint64_t key = 0;
  for (uint32_t r = 0; r < kp.k; ++r) {
    const double xv = (double)x[kp.dim[r]];
    double c = floor((xv - kp.org[r]) / kp.w);
    c = c < 0.0 ? 0.0 : c;
    uint64_t ci = (uint64_t)c;
    ci = ci > kp.cmax[r] ? kp.cmax[r] : ci;
    key += ci * kp.mult[r];
  }
  uint64_t fine = 0;
  if (kp.fm) {
    uint32_t f[kFineMaxDims];
    const uint32_t fmax = (1u << kp.fb) - 1u;
    for (uint32_t r = 0; r < kp.fm; ++r) {
      double v = ((double)x[kp.fdim[r]] - kp.forg[r]) * kp.fscale[r];
      v = v < 0.0 ? 0.0 : v;
      uint32_t q = (uint32_t)v;
      f[r] = q > fmax ? fmax : q;
    }
    for (int b = (int)kp.fb - 1; b >= 0; --b)
      for (uint32_t r = 0; r < kp.fm; ++r) fine = (fine << 1) | ((f[r] >> b) & 1u);
  }
  return (key << (kp.fm * kp.fb)) | fine;
}

__global__ __launch_bounds__(kBlock) void k_cellkey(const float *__restrict__ P, uint64_t n,
                                                    uint32_t d, KeyParams kp,
                                                    uint64_t *__restrict__ keys,
                                                    uint32_t *__restrict__ ids) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  keys[i] = sort_key(P + i * d, kp);
  ids[i] = (uint32_t)i;
}

// Keys of query points in the grid of an indexed set E (the general join
// Q join_eps E of Section 3.1).  A query with some coordinate more than
// two cell widths outside E's range [lo_t, hi_t] (lo = lo_t - 2w and
// hi = hi_t + 2w here, caller's dimension order) is farther than eps from
// every point of E: it gets far_key, which sorts after every cell key, and
// is counted in *n_far.  The others are clamped into E's grid like E's own
// points; a clamped query searches cells that include all of its true
// neighbour cells.
__global__ __launch_bounds__(kBlock) void k_query_keys(const float *__restrict__ Q, uint64_t m,
                                                       uint32_t d, KeyParams kp,
                                                       const double *__restrict__ lo,
                                                       const double *__restrict__ hi,
                                                       uint64_t far_key,
                                                       uint64_t *__restrict__ keys,
                                                       uint32_t *__restrict__ ids,
                                                       unsigned long long *__restrict__ n_far) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  bool far = false;
  if (i < m) {
    const float *x = Q + i * d;
    for (uint32_t t = 0; t < d; ++t) {
      const double v = (double)x[t];
      far = far || v < lo[t] || v > hi[t];
    }
    keys[i] = far ? far_key : sort_key(x, kp);
    ids[i] = (uint32_t)i;
  }
  const uint64_t fm = ballot(far);
  if (lane_id() == 0 && fm) atomicAdd(n_far, (unsigned long long)__builtin_popcountll(fm));
}

// ---------------------------------------------------------------------------
// a4: gather rows in cell order: X[p][r] = P[id_p][perm[r]], zero padded.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gather(const float *__restrict__ P, uint64_t n,
                                                   uint32_t d, uint32_t dp,
                                                   const uint32_t *__restrict__ perm,
                                                   const uint32_t *__restrict__ sorted_ids,
                                                   float *__restrict__ X,
                                                   uint32_t *__restrict__ orig_id,
                                                   uint32_t *__restrict__ pos_of) {
  // grid-stride: n * dp elements may exceed the 2^32 work-items of a dispatch
  const uint64_t total = n * dp;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint64_t p = e / dp;
    const uint32_t r = (uint32_t)(e - p * dp);
    const uint32_t id = sorted_ids[p];
    X[e] = r < d ? P[(uint64_t)id * d + perm[r]] : 0.0f;
    if (r == 0) {
      orig_id[p] = id;
      pos_of[id] = (uint32_t)p;
    }
  }
}

// ---------------------------------------------------------------------------
// a5: compaction of the non-empty cells.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_cell_flags(const uint64_t *__restrict__ keys,
                                                       uint64_t n, uint32_t sh,
                                                       uint32_t *__restrict__ flag) {
  const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  flag[p] = (p == 0 || (keys[p] >> sh) != (keys[p - 1] >> sh)) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_cell_write(const uint64_t *__restrict__ keys,
                                                       uint64_t n, uint32_t sh,
                                                       const uint32_t *__restrict__ cidx,
                                                       uint64_t *__restrict__ cell_key,
                                                       uint32_t *__restrict__ cell_start) {
  const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const bool first = (p == 0 || (keys[p] >> sh) != (keys[p - 1] >> sh));
  if (first) {
    cell_key[cidx[p]] = keys[p] >> sh;
    cell_start[cidx[p]] = (uint32_t)p;
  }
  // cell index of p is cidx[p] when p starts a cell, else cidx[p] - 1
  if (p == n - 1) cell_start[cidx[p] + (first ? 1u : 0u)] = (uint32_t)n;
}

// ---------------------------------------------------------------------------
// a6: adjacent non-empty cells (Section 3.2.1: only the 3^k cells around a
// query cell can hold its neighbours; Section 5.5: each is found by binary
// search over the non-empty cell ids).  One wave per query cell, 64 offsets
// per step; the cell-key table is staged in LDS, whole when it fits, else
// as a fence of every stride-th key that narrows the search to a short
// stretch of the table in global memory.  The searches wait on dependent
// loads, so a workgroup of 16 waves shares one fence: two of them fill a CU
// with 32 waves where workgroups of 4 waves would leave it at 8.
// ---------------------------------------------------------------------------
constexpr int kFenceMax = 8192;  // 64 KiB of u64 keys in LDS
constexpr int kNbrBlock = 1024;
constexpr int kNbrWaves = kNbrBlock / kWave;

// First table position whose key is >= key (ncell if none).  The fence
// holds cell_key[f * fstride]; when fstride is 1 it is the whole table.
__device__ __forceinline__ uint64_t lower_bound_cell(uint64_t key,
                                                    const uint64_t *__restrict__ fence,
                                                    uint32_t nfence, uint32_t fstride,
                                                    const uint64_t *__restrict__ cell_key,
                                                    uint64_t ncell) {
  uint32_t lo = 0, hi = nfence;  // first fence entry >= key
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (fence[mid] < key) lo = mid + 1; else hi = mid;
  }
  if (fstride == 1 || lo == 0) return (uint64_t)lo * fstride;
  // cell_key[(lo-1) fstride] < key <= cell_key[lo fstride] (or the end)
  uint64_t a = (uint64_t)(lo - 1) * fstride + 1, b = (uint64_t)lo * fstride;
  if (b > ncell) b = ncell;
  while (a < b) {
    const uint64_t mid = (a + b) >> 1;
    if (cell_key[mid] < key) a = mid + 1; else b = mid;
  }
  return a;
}

// Query cells are qkey[0 .. nq) (the table itself in a self-join); the
// table is cell_key[0 .. ncell) with its cell_start.  The 3^k offsets are
// taken in groups of three that differ only in the last indexed dimension,
// the least significant digit of the key (multiplier 1): their keys are
// consecutive, so one search finds the position of the smallest and the
// other two are the entries after it.  Each lane takes one group; groups
// and the cells inside a group come in ascending key order, so the
// neighbour list of a cell is written sorted.
__global__ __launch_bounds__(kNbrBlock) void k_neighbors(
    int pass, const uint64_t *__restrict__ qkey, uint64_t nq,
    const uint64_t *__restrict__ cell_key, const uint32_t *__restrict__ cell_start,
    uint64_t ncell, NbrParams np, uint32_t *__restrict__ nbr_count,
    uint64_t *__restrict__ cand_sum, const uint32_t *__restrict__ nbr_off,
    uint32_t *__restrict__ nbr_cell) {
  __shared__ uint64_t fence[kFenceMax];
  for (uint32_t i = threadIdx.x; i < np.nfence; i += kNbrBlock)
    fence[i] = cell_key[(uint64_t)i * np.fstride];
  __syncthreads();
  const uint32_t l = lane_id();
  const uint64_t wid = (uint64_t)blockIdx.x * kNbrWaves + threadIdx.x / kWave;
  const uint64_t nw = (uint64_t)gridDim.x * kNbrWaves;
  const uint32_t kl = np.k - 1;                   // the last indexed dimension
  const uint32_t ng = (uint32_t)(np.n_off / 3);  // 3^(k-1) <= 3^15 groups
  for (uint64_t A = wid; A < nq; A += nw) {
    const uint64_t keyA = qkey[A];
    int64_t cA[kKeyMaxDims];
    for (uint32_t r = 0; r < np.k; ++r) cA[r] = (int64_t)((keyA / np.mult[r]) % np.m[r]);
    const bool lo_ok = cA[kl] >= 1;                       // the cell below exists
    const bool hi_ok = cA[kl] + 1 < (int64_t)np.m[kl];  // the cell above exists
    uint32_t count = 0, wpos = (pass == 1) ? nbr_off[A] : 0u;
    uint64_t csum = 0;
    for (uint32_t base = 0; base < ng; base += kWave) {
      const uint32_t g = base + l;
      bool ok = g < ng;
      uint64_t keyB = keyA;  // the group's key with the last digit of A
      uint32_t rem = g;
      for (int r = (int)kl - 1; r >= 0; --r) {  // dimension 0 is the most significant digit
        const int64_t delta = (int64_t)(rem % 3u) - 1;
        rem /= 3u;
        const int64_t c = cA[r] + delta;
        ok = ok && c >= 0 && c < (int64_t)np.m[r];
        keyB += (uint64_t)delta * np.mult[r];
      }
      // keys keyB - 1, keyB, keyB + 1 (those inside the grid), ascending
      int64_t Bx[3] = {-1, -1, -1};
      if (ok) {
        const uint64_t first = lo_ok ? keyB - 1 : keyB;
        uint64_t q = lower_bound_cell(first, fence, np.nfence, np.fstride, cell_key, ncell);
        for (uint32_t t = 0; t < 3; ++t) {
          const uint64_t kk = keyB + t - 1;
          if ((t == 0 && !lo_ok) || (t == 2 && !hi_ok)) continue;
          // q is the first position with key >= kk
          if (q < ncell && (np.fstride == 1 ? fence[q] : cell_key[q]) == kk) Bx[t] = (int64_t)q++;
        }
      }
      const uint64_t m0 = ballot(Bx[0] >= 0), m1 = ballot(Bx[1] >= 0), m2 = ballot(Bx[2] >= 0);
      const uint32_t found = (uint32_t)(__builtin_popcountll(m0) + __builtin_popcountll(m1) +
                                        __builtin_popcountll(m2));
      if (pass == 0) {
        count += found;
        for (uint32_t t = 0; t < 3; ++t)
          if (Bx[t] >= 0) csum += (uint64_t)(cell_start[Bx[t] + 1] - cell_start[Bx[t]]);
      } else {
        uint32_t w = wpos + lanes_below(m0) + lanes_below(m1) + lanes_below(m2);
        for (uint32_t t = 0; t < 3; ++t)
          if (Bx[t] >= 0) nbr_cell[w++] = (uint32_t)Bx[t];
        wpos += found;
      }
    }
    if (pass == 0) {
      // wave-wide sum of the candidate counts
      for (int off = 32; off > 0; off >>= 1) csum += __shfl_xor(csum, off);
      if (l == 0) {
        nbr_count[A] = count;
        cand_sum[A] = csum;
      }
    }
  }
}

// Candidate runs: maximal stretches of consecutive cell indices in A's
// (sorted) neighbour list, as position ranges.  sym = 1 keeps only B >= A.
__global__ __launch_bounds__(kBlock) void k_runs(int pass, int sym, uint64_t ncell,
                                                 const uint32_t *__restrict__ cell_start,
                                                 const uint32_t *__restrict__ nbr_off,
                                                 const uint32_t *__restrict__ nbr_cell,
                                                 uint32_t *__restrict__ run_count,
                                                 const uint32_t *__restrict__ run_off,
                                                 uint2 *__restrict__ runs) {
  const uint64_t A = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (A >= ncell) return;
  const uint32_t b0 = nbr_off[A], b1 = nbr_off[A + 1];
  uint32_t cnt = 0, w = pass ? run_off[A] : 0u;
  uint32_t i = b0;
  while (i < b1) {
    uint32_t B = nbr_cell[i];
    if (sym && B < A) { ++i; continue; }
    uint32_t last = B;
    ++i;
    while (i < b1 && nbr_cell[i] == last + 1) { last = nbr_cell[i]; ++i; }
    if (pass) runs[w++] = make_uint2(cell_start[B], cell_start[last + 1]);
    ++cnt;
  }
  if (!pass) run_count[A] = cnt;
}

// Union of the candidate runs of each group of consecutive cells
// [gfirst[g], gfirst[g + 1]) (at most kGroupMaxCells cells): the cells' run
// lists, each sorted and disjoint, merged in position order with
// overlapping or touching ranges joined, so that no candidate appears
// twice.  pass 0 counts the group's runs, pass 1 writes them at goff[g].
__global__ __launch_bounds__(kBlock) void k_group_runs(int pass, uint64_t ngroup,
                                                       const uint32_t *__restrict__ gfirst,
                                                       const uint32_t *__restrict__ run_off,
                                                       const uint2 *__restrict__ runs,
                                                       uint32_t *__restrict__ gcount,
                                                       const uint32_t *__restrict__ goff,
                                                       uint2 *__restrict__ gruns) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ngroup) return;
  const uint32_t a0 = gfirst[g], na = gfirst[g + 1] - a0;
  uint32_t at[kGroupMaxCells], end[kGroupMaxCells];
  for (uint32_t i = 0; i < kGroupMaxCells; ++i) {
    at[i] = i < na ? run_off[a0 + i] : 0u;
    end[i] = i < na ? run_off[a0 + i + 1] : 0u;
  }
  uint32_t cnt = 0, w = pass ? goff[g] : 0u;
  bool have = false;
  uint2 cur = make_uint2(0u, 0u);
  for (;;) {
    int best = -1;
    uint32_t bx = 0xffffffffu;
    for (uint32_t i = 0; i < kGroupMaxCells; ++i)
      if (at[i] < end[i] && runs[at[i]].x < bx) {
        bx = runs[at[i]].x;
        best = (int)i;
      }
    if (best < 0) break;
    const uint2 r = runs[at[best]++];
    if (have && r.x <= cur.y) {
      cur.y = r.y > cur.y ? r.y : cur.y;
    } else {
      if (have) {
        if (pass) gruns[w + cnt] = cur;
        ++cnt;
      }
      cur = r;
      have = true;
    }
  }
  if (have) {
    if (pass) gruns[w + cnt] = cur;
    ++cnt;
  }
  if (!pass) gcount[g] = cnt;
}

// Work units (see WorkUnit).  Query slots of cell A are [qa, qb): positions
// in contiguous mode, indices into the sorted query list in list mode.
// In symmetric mode the first run of A starts at A itself and each query
// block only looks at candidates from its own first query onwards.
__device__ __forceinline__ void cell_query_slots(uint64_t A, const uint32_t *__restrict__ cell_start,
                                                 const uint32_t *__restrict__ qlist, uint64_t nq,
                                                 uint32_t *qa, uint32_t *qb) {
  const uint32_t s = cell_start[A], e = cell_start[A + 1];
  if (!qlist) {
    *qa = s;
    *qb = e;
    return;
  }
  uint64_t lo = 0, hi = nq;
  while (lo < hi) { uint64_t m = (lo + hi) >> 1; if (qlist[m] < s) lo = m + 1; else hi = m; }
  *qa = (uint32_t)lo;
  hi = nq;
  while (lo < hi) { uint64_t m = (lo + hi) >> 1; if (qlist[m] < e) lo = m + 1; else hi = m; }
  *qb = (uint32_t)lo;
}

// Per cell: its number of query blocks and the total length of its runs.
__global__ __launch_bounds__(kBlock) void k_wu_cells(
    uint64_t ncell, uint32_t tq, const uint32_t *__restrict__ cell_start,
    const uint32_t *__restrict__ qlist, uint64_t nq, const uint32_t *__restrict__ run_off,
    const uint2 *__restrict__ runs, uint32_t *__restrict__ nqb, uint64_t *__restrict__ run_total) {
  const uint64_t A = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (A >= ncell) return;
  uint32_t qa, qb;
  cell_query_slots(A, cell_start, qlist, nq, &qa, &qb);
  nqb[A] = (qb - qa + tq - 1) / tq;
  uint64_t total = 0;
  for (uint32_t r = run_off[A]; r < run_off[A + 1]; ++r) total += runs[r].y - runs[r].x;
  run_total[A] = total;
}

// Query block t: its cell (binary search over the scanned block counts),
// slot range and candidate count.
struct QBlock {
  uint32_t A, q0, q1;
  uint64_t L;       // candidates of the block
  uint32_t skip;
  uint32_t r0, r1;  // its runs [r0, r1)
};

__device__ __forceinline__ QBlock query_block(uint64_t t, int sym, uint64_t ncell, uint32_t tq,
                                              const uint32_t *__restrict__ cell_start,
                                              const uint32_t *__restrict__ qlist, uint64_t nq,
                                              const uint32_t *__restrict__ qb_off,
                                              const uint32_t *__restrict__ run_off,
                                              const uint2 *__restrict__ runs,
                                              const uint64_t *__restrict__ run_total,
                                              int per_block) {
  uint64_t lo = 0, hi = ncell;  // last cell with qb_off[A] <= t
  while (hi - lo > 1) {
    const uint64_t m = (lo + hi) >> 1;
    if (qb_off[m] <= t) lo = m; else hi = m;
  }
  // cells without query blocks share their offset with the next cell, so
  // the last cell whose offset is <= t is the one that owns block t
  QBlock b;
  b.A = (uint32_t)lo;
  uint32_t qa, qe;
  cell_query_slots(lo, cell_start, qlist, nq, &qa, &qe);
  b.q0 = qa + (uint32_t)(t - qb_off[lo]) * tq;
  b.q1 = min(b.q0 + tq, qe);
  if (per_block) {  // the block's own runs (SORTIDU ranges), already cut at q0
    b.r0 = run_off[t];
    b.r1 = run_off[t + 1];
    b.skip = 0u;
    b.L = run_total[t];
    return b;
  }
  b.r0 = run_off[lo];
  b.r1 = run_off[lo + 1];
  // a symmetric block starts at its first query's position (in list mode
  // the list holds whole cells, so that position is qlist[q0])
  b.skip = sym ? ((qlist ? qlist[b.q0] : b.q0) - runs[b.r0].x) : 0u;
  b.L = run_total[lo] - b.skip;
  return b;
}

__global__ __launch_bounds__(kBlock) void k_wu_count(
    uint64_t nqb_total, int sym, uint64_t ncell, uint32_t tq, uint32_t tc,
    const uint32_t *__restrict__ cell_start, const uint32_t *__restrict__ qlist, uint64_t nq,
    const uint32_t *__restrict__ qb_off, const uint32_t *__restrict__ run_off,
    const uint2 *__restrict__ runs, const uint64_t *__restrict__ run_total,
    uint32_t *__restrict__ units, uint64_t *__restrict__ eval, int per_block) {
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nqb_total) return;
  const QBlock b = query_block(t, sym, ncell, tq, cell_start, qlist, nq, qb_off, run_off, runs,
                               run_total, per_block);
  units[t] = (uint32_t)((b.L + tc - 1) / tc);
  eval[t] = (uint64_t)(b.q1 - b.q0) * b.L;
}

__global__ __launch_bounds__(kBlock) void k_wu_fill(
    uint64_t nqb_total, int sym, uint64_t ncell, uint32_t tq, uint32_t tc,
    const uint32_t *__restrict__ cell_start, const uint32_t *__restrict__ qlist, uint64_t nq,
    const uint32_t *__restrict__ qb_off, const uint32_t *__restrict__ run_off,
    const uint2 *__restrict__ runs, const uint64_t *__restrict__ run_total,
    const uint32_t *__restrict__ unit_off, WorkUnit *__restrict__ wu,
    uint64_t *__restrict__ order_key, int per_block) {
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nqb_total) return;
  const QBlock b = query_block(t, sym, ncell, tq, cell_start, qlist, nq, qb_off, run_off, runs,
                               run_total, per_block);
  if (b.L == 0) return;
  const uint32_t nu = (uint32_t)((b.L + tc - 1) / tc);
  const uint32_t r1 = b.r1;
  uint32_t r = b.r0;
  uint32_t c = runs[r].x + b.skip;
  uint32_t w = unit_off[t];
  for (uint32_t u = 0; u < nu; ++u) {
    WorkUnit x;
    x.q0 = b.q0;
    x.q1 = b.q1;
    x.cell = b.A;
    x.pad = 0;
    x.run_first = r;
    x.c_begin = c;
    uint32_t need = tc;
    for (;;) {
      const uint32_t avail = runs[r].y - c;
      if (avail > need) { c += need; break; }
      need -= avail;
      if (r + 1 == r1 || need == 0) { c = runs[r].y; break; }
      ++r;
      c = runs[r].x;
    }
    x.run_last = r;
    x.c_end = c;
    // optional order key: stretch index within the block, then unit index
    if (order_key) order_key[w] = ((uint64_t)u << 32) | w;
    wu[w++] = x;
    if (c == runs[r].y && r + 1 < r1) { ++r; c = runs[r].x; }
  }
}

// SORTIDU for blocks of queries (see launch_qb_ranges).  The window around
// the block's u-range [umin, umax] is widened by eps (1 + 2^-16) plus a
// relative 2^-40: a candidate outside it is farther than eps (1 + 2^-16)
// from every query of the block along u alone, so its canonical FP64 sum
// exceeds eps^2 and no pair is lost.  The window is quantised like the sort
// key, so the search runs over the sorted keys of each adjacent cell.
__device__ __forceinline__ uint32_t quantise_u(double v, const USearch &us) {
  double q = (v - us.org) * us.scale;
  q = q < 0.0 ? 0.0 : q;
  q = q > (double)us.fmax ? (double)us.fmax : q;
  return (uint32_t)q;
}

__global__ __launch_bounds__(kBlock) void k_qb_ranges(
    int pass, int sym, uint64_t nqb_total, uint64_t ncell, uint32_t tq,
    const uint32_t *__restrict__ cell_start, const uint32_t *__restrict__ qb_off,
    const uint32_t *__restrict__ nbr_off, const uint32_t *__restrict__ nbr_cell,
    const uint32_t *__restrict__ ecell_start, const uint64_t *__restrict__ ekey,
    const float *__restrict__ Xq, USearch us, uint32_t *__restrict__ rcount,
    uint64_t *__restrict__ rlen, const uint32_t *__restrict__ roff, uint2 *__restrict__ ranges) {
  const uint32_t l = lane_id();
  const uint64_t nw = (uint64_t)gridDim.x * kWavesPerBlock;
  for (uint64_t t = (uint64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; t < nqb_total;
       t += nw) {
    // the block: its cell A (last cell with qb_off[A] <= t) and slots
    uint64_t lo = 0, hi = ncell;
    while (hi - lo > 1) {
      const uint64_t m = (lo + hi) >> 1;
      if (qb_off[m] <= t) lo = m; else hi = m;
    }
    const uint32_t A = (uint32_t)lo;
    const uint32_t q0 = cell_start[A] + (uint32_t)(t - qb_off[A]) * tq;
    const uint32_t q1 = min(q0 + tq, cell_start[A + 1]);
    // the queries' u-range
    float umin = __builtin_inff(), umax = -__builtin_inff();
    for (uint32_t q = q0 + l; q < q1; q += kWave) {
      const float u = Xq[(uint64_t)q * us.dp + us.ur];
      umin = fminf(umin, u);
      umax = fmaxf(umax, u);
    }
    for (int off = 32; off > 0; off >>= 1) {
      umin = fminf(umin, __shfl_xor(umin, off));
      umax = fmaxf(umax, __shfl_xor(umax, off));
    }
    const double dl = (double)umin, dh = (double)umax;
    const double wl = us.eps * (1.0 + 0x1p-16) + (__builtin_fabs(dl) + us.eps) * 0x1p-40;
    const double wh = us.eps * (1.0 + 0x1p-16) + (__builtin_fabs(dh) + us.eps) * 0x1p-40;
    const uint64_t flo = quantise_u(dl - wl, us), fhi = quantise_u(dh + wh, us);
    // adjacent cells, 64 at a time: each lane searches one cell, then the
    // wave merges the lanes' ranges in cell order
    const uint32_t b0 = nbr_off[A], b1 = nbr_off[A + 1];
    uint32_t cnt = 0, oc0 = 0, oc1 = 0;
    uint64_t len = 0;
    bool open = false;
    const uint32_t wbase = pass ? roff[t] : 0u;
    for (uint32_t base = b0; base < b1; base += kWave) {
      const uint32_t i = base + l;
      uint32_t c0 = 0, c1 = 0;
      if (i < b1) {
        const uint32_t B = nbr_cell[i];
        if (!(sym && B < A)) {
          const uint32_t cs = ecell_start[B], ce = ecell_start[B + 1];
          uint32_t a = cs, b = ce;  // first position with u-part >= flo
          while (a < b) {
            const uint32_t m = (a + b) >> 1;
            if ((ekey[m] & us.fmask) < flo) a = m + 1; else b = m;
          }
          c0 = a;
          b = ce;  // first position with u-part > fhi
          while (a < b) {
            const uint32_t m = (a + b) >> 1;
            if ((ekey[m] & us.fmask) <= fhi) a = m + 1; else b = m;
          }
          c1 = a;
          if (sym && B == A && c0 < q0) c0 = q0;
        }
      }
      const uint32_t nl = min((uint32_t)kWave, b1 - base);
      for (uint32_t j = 0; j < nl; ++j) {
        const uint32_t x0 = (uint32_t)__builtin_amdgcn_readlane((int)c0, (int)j);
        const uint32_t x1 = (uint32_t)__builtin_amdgcn_readlane((int)c1, (int)j);
        if (x1 <= x0) continue;
        if (open && x0 == oc1) {
          oc1 = x1;
          continue;
        }
        if (open) {
          if (pass && l == 0) ranges[wbase + cnt] = make_uint2(oc0, oc1);
          len += oc1 - oc0;
          ++cnt;
        }
        open = true;
        oc0 = x0;
        oc1 = x1;
      }
    }
    if (open) {
      if (pass && l == 0) ranges[wbase + cnt] = make_uint2(oc0, oc1);
      len += oc1 - oc0;
      ++cnt;
    }
    if (!pass && l == 0) {
      rcount[t] = cnt;
      rlen[t] = len;
    }
  }
}

// dst[i] = src[low 32 bits of keys[i]]
__global__ __launch_bounds__(kBlock) void k_gather_wu(const WorkUnit *__restrict__ src,
                                                      const uint64_t *__restrict__ keys,
                                                      uint64_t n, WorkUnit *__restrict__ dst) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  dst[i] = src[(uint32_t)keys[i]];
}

// out[A] = (query slots of cell A's units of tq queries) * cand_sum[A]: the
// lane work of A's units, idle slots included
__global__ void k_cell_slot_work(uint64_t ncell, const uint32_t *__restrict__ cell_start,
                                 const uint64_t *__restrict__ cand_sum, uint32_t tq,
                                 uint64_t *__restrict__ out) {
  const uint64_t A = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (A >= ncell) return;
  const uint64_t m = cell_start[A + 1] - cell_start[A];
  out[A] = (m + tq - 1) / tq * tq * cand_sum[A];
}

__global__ void k_cell_products(uint64_t ncell, const uint32_t *__restrict__ cell_start,
                                const uint64_t *__restrict__ cand_sum, uint64_t *__restrict__ out) {
  const uint64_t A = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (A >= ncell) return;
  out[A] = (uint64_t)(cell_start[A + 1] - cell_start[A]) * cand_sum[A];
}

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }
// Workgroups of a grid-stride launch over n elements: one element per
// thread up to 2^20 workgroups (a dispatch holds at most 2^32 work-items).
inline uint32_t stride_blocks(uint64_t n) {
  return (uint32_t)std::min<uint64_t>((n + kBlock - 1) / kBlock, 1u << 20);
}

// Pairs per row of sorted keys (row = key >> 32): counts[i] += the number
// of keys of row i.  Each wave adds one count per row it holds: the lane
// that starts a run of equal rows inside the wave adds the run's length.
// Grid-stride over 64-key segments, one per wave and step (count may exceed
// the 2^32 work-items of one dispatch).
__global__ __launch_bounds__(kBlock) void k_row_counts(const uint64_t *__restrict__ keys,
                                                       uint64_t count,
                                                       unsigned long long *__restrict__ counts) {
  const uint32_t l = lane_id();
  const uint64_t step = (uint64_t)gridDim.x * kBlock;
  for (uint64_t e0 = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~(uint32_t)(kWave - 1));
       e0 < count; e0 += step) {
    const uint64_t e = e0 + l;
    const bool live = e < count;
    const uint64_t row = live ? keys[e] >> 32 : 0;
    const bool head = live && (l == 0 || (keys[e - 1] >> 32) != row);
    const uint64_t heads = ballot(head);
    const uint64_t lives = ballot(live);
    if (head) {
      // the run ends at the next head above this lane, or at the last live lane
      const uint64_t above = heads & ~((2ull << l) - 1ull);
      const uint32_t end = above ? (uint32_t)__builtin_ctzll(above)
                                 : (uint32_t)(64 - __builtin_clzll(lives));
      atomicAdd(&counts[row], (unsigned long long)(end - l));
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
void launch_minmax(const float *P, uint64_t n, uint32_t d, uint32_t *gmin, uint32_t *gmax,
                   uint32_t *bad, hipStream_t s) {
  hipLaunchKernelGGL(k_init_minmax, dim3(1), dim3(kBlock), 0, s, gmin, gmax, bad, d);
  SJ_HIP(hipGetLastError());
  const uint64_t total = n * d;
  if (total == 0) return;
  uint32_t grid = (uint32_t)std::min<uint64_t>((total + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_minmax, dim3(grid), dim3(kBlock), 0, s, P, total, d, gmin, gmax, bad);
  SJ_HIP(hipGetLastError());
}

void launch_variance(const float *P, uint32_t d, uint64_t stride, uint64_t m, double *var,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_variance, dim3(d), dim3(kBlock), 0, s, P, d, stride, m, var);
  SJ_HIP(hipGetLastError());
}

void launch_cellkey(const float *P, uint64_t n, uint32_t d, const KeyParams &kp, uint64_t *keys,
                    uint32_t *ids, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_cellkey, dim3(blocks_for(n)), dim3(kBlock), 0, s, P, n, d, kp, keys, ids);
  SJ_HIP(hipGetLastError());
}

void launch_query_keys(const float *Q, uint64_t m, uint32_t d, const KeyParams &kp,
                       const double *lo, const double *hi, uint64_t far_key, uint64_t *keys,
                       uint32_t *ids, unsigned long long *n_far, hipStream_t s) {
  if (!m) return;
  hipLaunchKernelGGL(k_query_keys, dim3(blocks_for(m)), dim3(kBlock), 0, s, Q, m, d, kp, lo, hi,
                     far_key, keys, ids, n_far);
  SJ_HIP(hipGetLastError());
}

void launch_gather(const float *P, uint64_t n, uint32_t d, uint32_t dp, const uint32_t *perm,
                   const uint32_t *sorted_ids, float *X, uint32_t *orig_id, uint32_t *pos_of,
                   hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_gather, dim3(stride_blocks(n * dp)), dim3(kBlock), 0, s, P, n, d, dp, perm,
                     sorted_ids, X, orig_id, pos_of);
  SJ_HIP(hipGetLastError());
}

void launch_compact(const uint64_t *keys, uint64_t n, uint32_t fine_shift, uint32_t *flag_tmp,
                    uint32_t *d_ncell, uint64_t *cell_key, uint32_t *cell_start, void *scan_tmp,
                    hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_cell_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, keys, n, fine_shift,
                     flag_tmp);
  SJ_HIP(hipGetLastError());
  exclusive_scan_u32(flag_tmp, flag_tmp, n, d_ncell, scan_tmp, s);
  hipLaunchKernelGGL(k_cell_write, dim3(blocks_for(n)), dim3(kBlock), 0, s, keys, n, fine_shift,
                     flag_tmp, cell_key, cell_start);
  SJ_HIP(hipGetLastError());
}

void launch_neighbors(int pass, const uint64_t *qkey, uint64_t nq, const uint64_t *cell_key,
                      const uint32_t *cell_start, uint64_t ncell, const NbrParams &np,
                      uint32_t *nbr_count, uint64_t *cand_sum, const uint32_t *nbr_off,
                      uint32_t *nbr_cell, hipStream_t s) {
  if (!nq || !ncell) return;
  const uint64_t waves = nq;
  uint32_t grid = (uint32_t)std::min<uint64_t>((waves + kNbrWaves - 1) / kNbrWaves, 1024);
  hipLaunchKernelGGL(k_neighbors, dim3(grid), dim3(kNbrBlock), 0, s, pass, qkey, nq, cell_key,
                     cell_start, ncell, np, nbr_count, cand_sum, nbr_off, nbr_cell);
  SJ_HIP(hipGetLastError());
}

void launch_runs(int pass, int sym, uint64_t ncell, const uint32_t *cell_start,
                 const uint32_t *nbr_off, const uint32_t *nbr_cell, uint32_t *run_count,
                 const uint32_t *run_off, uint2 *runs, hipStream_t s) {
  if (!ncell) return;
  hipLaunchKernelGGL(k_runs, dim3(blocks_for(ncell)), dim3(kBlock), 0, s, pass, sym, ncell,
                     cell_start, nbr_off, nbr_cell, run_count, run_off, runs);
  SJ_HIP(hipGetLastError());
}

void launch_group_runs(int pass, uint64_t ngroup, const uint32_t *gfirst, const uint32_t *run_off,
                       const uint2 *runs, uint32_t *gcount, const uint32_t *goff, uint2 *gruns,
                       hipStream_t s) {
  if (!ngroup) return;
  hipLaunchKernelGGL(k_group_runs, dim3(blocks_for(ngroup)), dim3(kBlock), 0, s, pass, ngroup,
                     gfirst, run_off, runs, gcount, goff, gruns);
  SJ_HIP(hipGetLastError());
}

void launch_wu_cells(uint64_t ncell, uint32_t tq, const uint32_t *cell_start,
                     const uint32_t *qlist, uint64_t nq, const uint32_t *run_off,
                     const uint2 *runs, uint32_t *nqb, uint64_t *run_total, hipStream_t s) {
  if (!ncell) return;
  hipLaunchKernelGGL(k_wu_cells, dim3(blocks_for(ncell)), dim3(kBlock), 0, s, ncell, tq,
                     cell_start, qlist, nq, run_off, runs, nqb, run_total);
  SJ_HIP(hipGetLastError());
}

void launch_wu_count(uint64_t nqb_total, int sym, uint64_t ncell, uint32_t tq, uint32_t tc,
                     const uint32_t *cell_start, const uint32_t *qlist, uint64_t nq,
                     const uint32_t *qb_off, const uint32_t *run_off, const uint2 *runs,
                     const uint64_t *run_total, uint32_t *units, uint64_t *eval, hipStream_t s,
                     int per_block) {
  if (!nqb_total) return;
  hipLaunchKernelGGL(k_wu_count, dim3(blocks_for(nqb_total)), dim3(kBlock), 0, s, nqb_total, sym,
                     ncell, tq, tc, cell_start, qlist, nq, qb_off, run_off, runs, run_total, units,
                     eval, per_block);
  SJ_HIP(hipGetLastError());
}

void launch_wu_fill(uint64_t nqb_total, int sym, uint64_t ncell, uint32_t tq, uint32_t tc,
                    const uint32_t *cell_start, const uint32_t *qlist, uint64_t nq,
                    const uint32_t *qb_off, const uint32_t *run_off, const uint2 *runs,
                    const uint64_t *run_total, const uint32_t *unit_off, WorkUnit *wu,
                    uint64_t *order_key, hipStream_t s, int per_block) {
  if (!nqb_total) return;
  hipLaunchKernelGGL(k_wu_fill, dim3(blocks_for(nqb_total)), dim3(kBlock), 0, s, nqb_total, sym,
                     ncell, tq, tc, cell_start, qlist, nq, qb_off, run_off, runs, run_total,
                     unit_off, wu, order_key, per_block);
  SJ_HIP(hipGetLastError());
}

void launch_qb_ranges(int pass, int sym, uint64_t nqb_total, uint64_t ncell, uint32_t tq,
                      const uint32_t *cell_start, const uint32_t *qb_off,
                      const uint32_t *nbr_off, const uint32_t *nbr_cell,
                      const uint32_t *ecell_start, const uint64_t *ekey, const float *Xq,
                      const USearch &us, uint32_t *rcount, uint64_t *rlen,
                      const uint32_t *roff, uint2 *ranges, hipStream_t s) {
  if (!nqb_total) return;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((nqb_total + kWavesPerBlock - 1) /
                                                     kWavesPerBlock, 1u << 16);
  hipLaunchKernelGGL(k_qb_ranges, dim3(grid), dim3(kBlock), 0, s, pass, sym, nqb_total, ncell,
                     tq, cell_start, qb_off, nbr_off, nbr_cell, ecell_start, ekey, Xq, us,
                     rcount, rlen, roff, ranges);
  SJ_HIP(hipGetLastError());
}

void launch_gather_wu(const WorkUnit *src, const uint64_t *keys, uint64_t n, WorkUnit *dst,
                      hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_gather_wu, dim3(blocks_for(n)), dim3(kBlock), 0, s, src, keys, n, dst);
  SJ_HIP(hipGetLastError());
}

void launch_cell_products(uint64_t ncell, const uint32_t *cell_start, const uint64_t *cand_sum,
                          uint64_t *out, hipStream_t s) {
  if (!ncell) return;
  hipLaunchKernelGGL(k_cell_products, dim3(blocks_for(ncell)), dim3(kBlock), 0, s, ncell,
                     cell_start, cand_sum, out);
  SJ_HIP(hipGetLastError());
}

void launch_cell_slot_work(uint64_t ncell, const uint32_t *cell_start, const uint64_t *cand_sum,
                           uint32_t tq, uint64_t *out, hipStream_t s) {
  if (!ncell) return;
  hipLaunchKernelGGL(k_cell_slot_work, dim3(blocks_for(ncell)), dim3(kBlock), 0, s, ncell,
                     cell_start, cand_sum, tq, out);
  SJ_HIP(hipGetLastError());
}

void launch_row_counts(const uint64_t *keys, uint64_t count, unsigned long long *counts,
                       hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_row_counts, dim3(stride_blocks(count)), dim3(kBlock), 0, s, keys, count,
                     counts);
  SJ_HIP(hipGetLastError());
}

}  // namespace sj
