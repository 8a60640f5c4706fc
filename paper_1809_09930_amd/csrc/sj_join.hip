// Distance filter of the self-join (Algorithm 1, SelfJoinKernel with
// calcDistancePts; Section 4.4 short-circuit), FP32 difference form on the
// vector ALUs of gfx950.
//
// Mapping.  Each wave processes one work unit: up to 64*RQ query points of
// one cell (RQ per lane, coordinates held in VGPRs) against a stretch of
// candidate positions.  The candidate index is wave-uniform, so candidate
// coordinates arrive through scalar loads into SGPRs and feed every lane's
// subtraction directly: no LDS traffic and no shuffles on the hot loop.
//
// Short-circuit.  The squared distance grows monotonically as dimensions are
// added (round-to-nearest addition of a non-negative term never decreases
// the sum), so once every lane of a query group has a partial sum above the
// reject threshold `hi`, the rest of that candidate is skipped for the group.
// The test is wave-uniform; its schedule is SJ_SHORTC_FIRST / SJ_SHORTC_STEP.
// Points inside a cell are ordered along a Morton curve, so the 64 queries of
// a group are neighbours and their partial sums rise together.
//
// Exactness.  `hi` and `lo` bound the FP32 rounding error of the sum against
// the canonical FP64 predicate: s > hi proves rejection, s <= lo proves
// acceptance, anything between goes to the FP64 recheck below, which
// evaluates the canonical predicate itself (caller's dimension order,
// separately rounded binary64 operations).
//
// Emission.  Accepted pairs are compacted per wave with ballot + mbcnt into
// a wave-private LDS stage; a full stage is flushed with one atomic on the
// global cursor and coalesced stores.  Pairs past `capacity` are counted
// but not stored (the host then grows the buffer and reruns).
#include "sj_internal.hpp"

namespace sj {

namespace {

constexpr int kStage = 512;  // u64 keys staged per wave

// Short-circuit schedule: first test after SJ_SHORTC_FIRST dimensions, then
// every SJ_SHORTC_STEP (padded dimension above 24); the _SMALL pair applies
// up to 24.
#ifndef SJ_SHORTC_FIRST_SMALL
#define SJ_SHORTC_FIRST_SMALL 8
#endif
#ifndef SJ_SHORTC_STEP_SMALL
#define SJ_SHORTC_STEP_SMALL 8
#endif
#ifndef SJ_SHORTC_FIRST
#define SJ_SHORTC_FIRST 24
#endif
#ifndef SJ_SHORTC_STEP
#define SJ_SHORTC_STEP 8
#endif
// Query points per lane by padded dimension (register blocking).
#ifndef SJ_FP32_RQ_SMALL
#define SJ_FP32_RQ_SMALL 2  // dp <= 24
#endif
#ifndef SJ_FP32_RQ_MID
#define SJ_FP32_RQ_MID 1    // dp <= 64
#endif

// Canonical predicate on positions a, b of the cell-ordered rows.
__device__ __noinline__ bool canonical_within(const float *__restrict__ X, uint32_t a, uint32_t b,
                                              const uint16_t *__restrict__ inv_perm, uint32_t d,
                                              uint32_t dp, double eps2) {
#pragma clang fp contract(off)
  const float *pa = X + (uint64_t)a * dp;
  const float *pb = X + (uint64_t)b * dp;
  double acc = 0.0;
  for (uint32_t t = 0; t < d; ++t) {
    const uint32_t r = inv_perm[t];
    const double diff = (double)pa[r] - (double)pb[r];
    const double sq = diff * diff;
    acc = acc + sq;
  }
  return acc <= eps2;
}

struct WaveStage {
  uint64_t *buf;  // this wave's LDS slice
  uint32_t cnt;   // wave-uniform fill level
};

__device__ __forceinline__ void stage_flush(WaveStage &st, uint64_t *__restrict__ out,
                                            uint64_t capacity,
                                            unsigned long long *__restrict__ cursor) {
  if (st.cnt == 0) return;
  __builtin_amdgcn_wave_barrier();
  unsigned long long base = 0;
  if (lane_id() == 0) base = atomicAdd(cursor, (unsigned long long)st.cnt);
  base = uniform_u64(__shfl(base, 0));
  for (uint32_t i = lane_id(); i < st.cnt; i += kWave) {
    const uint64_t pos = base + i;
    if (pos < capacity) out[pos] = st.buf[i];
  }
  __builtin_amdgcn_wave_barrier();
  st.cnt = 0;
}

template <int DP, int RQ>
struct Lanes {
  float q[RQ][DP];
  uint32_t pos[RQ];  // cell-order position of each query (0xffffffff: empty slot)
  uint32_t id[RQ];   // caller index of each query
  float init[RQ];    // 0 for a live slot, +inf for an empty one
};

template <int DP, int RQ, bool kFilter, bool kCount>
__device__ __forceinline__ void eval_candidate(
    const Lanes<DP, RQ> &L, uint32_t c, const float *__restrict__ X,
    const uint32_t *__restrict__ orig_id, const uint16_t *__restrict__ inv_perm, uint32_t d,
    float lo, float hi, double eps2, bool symmetric, bool shortc,
    WaveStage &st, uint64_t *__restrict__ out, uint64_t capacity,
    unsigned long long *__restrict__ cursor, uint64_t &n_recheck, uint64_t &n_count) {
  constexpr int kFirst0 = DP <= 24 ? SJ_SHORTC_FIRST_SMALL : SJ_SHORTC_FIRST;
  constexpr int kFirst = DP < kFirst0 ? DP : kFirst0;
  constexpr int kStep = DP <= 24 ? SJ_SHORTC_STEP_SMALL : SJ_SHORTC_STEP;
  const float *__restrict__ crow = X + (uint64_t)c * DP;
  float s[RQ];
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    s[r] = L.init[r];
    if (kFilter) s[r] = (L.pos[r] <= c) ? s[r] : __builtin_inff();
  }
  uint32_t alive = (1u << RQ) - 1u;

  // dimensions [0, kFirst) for every group
  {
    float cv[kFirst];
#pragma unroll
    for (int t = 0; t < kFirst; ++t) cv[t] = crow[t];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
#pragma unroll
      for (int t = 0; t < kFirst; ++t) {
        const float diff = L.q[r][t] - cv[t];
        s[r] = __builtin_fmaf(diff, diff, s[r]);
      }
    }
  }
  // remaining dimensions in steps of kStep, each preceded by the test
#pragma unroll
  for (int t0 = kFirst; t0 < DP; t0 += kStep) {
    if (shortc) {
#pragma unroll
      for (int r = 0; r < RQ; ++r)
        if ((alive >> r) & 1u)
          if (ballot(s[r] <= hi) == 0) alive &= ~(1u << r);
      if (alive == 0) return;
    }
    // the last step is shorter when kStep does not divide DP (the bounds
    // are compile-time constants once the loops are unrolled)
    float cv[kStep];
#pragma unroll
    for (int t = 0; t < kStep; ++t)
      if (t0 + t < DP) cv[t] = crow[t0 + t];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      if ((alive >> r) & 1u) {
#pragma unroll
        for (int t = 0; t < kStep; ++t) {
          if (t0 + t < DP) {
            const float diff = L.q[r][t0 + t] - cv[t];
            s[r] = __builtin_fmaf(diff, diff, s[r]);
          }
        }
      }
    }
  }

  // classification: s > hi rejects, s <= lo accepts, the band is rechecked
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    if (!((alive >> r) & 1u)) continue;
    const uint64_t m = ballot(s[r] <= hi);
    if (m == 0) continue;
    if (kCount) {
      n_count += (uint64_t)__builtin_popcountll(m);
      continue;
    }
    uint64_t acc = m & ballot(s[r] <= lo);
    const uint64_t band = m & ~acc;
    if (band) {
      bool ok = false;
      if ((band >> lane_id()) & 1ull)
        ok = canonical_within(X, L.pos[r], c, inv_perm, d, DP, eps2);
      acc |= ballot(ok);
      n_recheck += (uint64_t)__builtin_popcountll(band);
    }
    if (acc == 0) continue;
    // emit (query, candidate), and (candidate, query) too in symmetric mode
    const uint32_t cid = orig_id[c];
    const bool e1 = (acc >> lane_id()) & 1ull;
    const bool e2 = e1 && symmetric && L.pos[r] != c;
    const uint64_t m2 = ballot(e2);
    const uint32_t total = (uint32_t)(__builtin_popcountll(acc) + __builtin_popcountll(m2));
    if (st.cnt + total > (uint32_t)kStage) stage_flush(st, out, capacity, cursor);
    const uint32_t off = st.cnt + lanes_below(acc) + lanes_below(m2);
    if (e1) {
      st.buf[off] = ((uint64_t)L.id[r] << 32) | cid;
      if (e2) st.buf[off + 1] = ((uint64_t)cid << 32) | L.id[r];
    }
    st.cnt += total;
  }
}

// One wave = one work unit.  kCount: count the pairs the filter cannot
// reject (s <= hi) instead of emitting them.
template <int DP, int RQ, bool kCount>
__device__ __forceinline__ void join_body(
    const float *__restrict__ X, const uint32_t *__restrict__ orig_id,
    const uint16_t *__restrict__ inv_perm, const WorkUnit *__restrict__ wus, uint64_t n_wu,
    const uint2 *__restrict__ runs, const uint32_t *__restrict__ qlist, uint32_t d, float lo,
    float hi, double eps2, int symmetric, int shortc, uint64_t *__restrict__ out,
    uint64_t capacity, unsigned long long *__restrict__ cursor,
    unsigned long long *__restrict__ rechecks, uint64_t (*stage_mem)[kStage]) {
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  const uint64_t u = (uint64_t)blockIdx.x * kWavesPerBlock + w;
  if (u >= n_wu) return;  // whole wave leaves; no workgroup barrier follows
  const WorkUnit wu = wus[u];
  const uint32_t l = lane_id();

  Lanes<DP, RQ> L;
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const uint32_t slot = wu.q0 + (uint32_t)r * kWave + l;
    const bool live = slot < wu.q1;
    const uint32_t p = live ? (qlist ? qlist[slot] : slot) : 0u;
    L.pos[r] = live ? p : 0xffffffffu;
    L.id[r] = live ? orig_id[p] : 0u;
    L.init[r] = live ? 0.0f : __builtin_inff();
    const float4 *row = reinterpret_cast<const float4 *>(X + (uint64_t)p * DP);
#pragma unroll
    for (int t = 0; t < DP / 4; ++t) {
      const float4 v = row[t];
      L.q[r][4 * t + 0] = v.x;
      L.q[r][4 * t + 1] = v.y;
      L.q[r][4 * t + 2] = v.z;
      L.q[r][4 * t + 3] = v.w;
    }
  }
  // in symmetric contiguous mode candidates below q1 need the per-lane
  // "query position <= candidate position" filter; beyond it all pass
  const uint32_t filt_end = (symmetric && !qlist) ? wu.q1 : 0u;

  WaveStage st{kCount ? nullptr : &stage_mem[w][0], 0u};
  uint64_t n_recheck = 0, n_count = 0;
  const bool sym = symmetric != 0, sc = shortc != 0;

  for (uint32_t r = wu.run_first; r <= wu.run_last; ++r) {
    const uint2 run = runs[r];
    const uint32_t cb = (r == wu.run_first) ? wu.c_begin : run.x;
    const uint32_t ce = (r == wu.run_last) ? wu.c_end : run.y;
    const uint32_t mid = cb < filt_end ? (ce < filt_end ? ce : filt_end) : cb;
    for (uint32_t c = cb; c < mid; ++c)
      eval_candidate<DP, RQ, true, kCount>(L, c, X, orig_id, inv_perm, d, lo, hi, eps2, sym, sc,
                                           st, out, capacity, cursor, n_recheck, n_count);
    for (uint32_t c = mid; c < ce; ++c)
      eval_candidate<DP, RQ, false, kCount>(L, c, X, orig_id, inv_perm, d, lo, hi, eps2, sym, sc,
                                            st, out, capacity, cursor, n_recheck, n_count);
  }
  stage_flush(st, out, capacity, cursor);
  if (l == 0) {
    if (n_recheck) atomicAdd(rechecks, (unsigned long long)n_recheck);
    if (n_count) atomicAdd(cursor, (unsigned long long)n_count);
  }
}

#define SJ_JOIN_PARAMS                                                                          \
  const float *__restrict__ X, const uint32_t *__restrict__ orig_id,                            \
      const uint16_t *__restrict__ inv_perm, const WorkUnit *__restrict__ wus, uint64_t n_wu,   \
      const uint2 *__restrict__ runs, const uint32_t *__restrict__ qlist, uint32_t d, float lo, \
      float hi, double eps2, int symmetric, int shortc, uint64_t *__restrict__ out,             \
      uint64_t capacity, unsigned long long *__restrict__ cursor,                               \
      unsigned long long *__restrict__ rechecks

// The self-join distance kernel: emits result pairs.
template <int DP, int RQ>
__global__ __launch_bounds__(kBlock) void k_join_fp32(SJ_JOIN_PARAMS) {
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  join_body<DP, RQ, false>(X, orig_id, inv_perm, wus, n_wu, runs, qlist, d, lo, hi, eps2,
                           symmetric, shortc, out, capacity, cursor, rechecks, stage_mem);
}

// The estimation kernel (count only) used to size result buffers.
template <int DP, int RQ>
__global__ __launch_bounds__(kBlock) void k_count_fp32(SJ_JOIN_PARAMS) {
  join_body<DP, RQ, true>(X, orig_id, inv_perm, wus, n_wu, runs, qlist, d, lo, hi, eps2,
                          symmetric, shortc, out, capacity, cursor, rechecks, nullptr);
}

__global__ __launch_bounds__(kBlock) void k_unpack(const uint64_t *__restrict__ keys,
                                                   uint64_t count, uint32_t *__restrict__ out_i,
                                                   uint32_t *__restrict__ out_j,
                                                   float *__restrict__ out_dist,
                                                   const float *__restrict__ X,
                                                   const uint32_t *__restrict__ pos_of,
                                                   const uint16_t *__restrict__ inv_perm,
                                                   uint32_t d, uint32_t dp, uint32_t ishift) {
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= count) return;
  const uint64_t key = keys[e];
  const uint64_t mask = (1ull << ishift) - 1ull;
  const uint32_t i = (uint32_t)((key >> ishift) & mask), j = (uint32_t)(key & mask);
  if (out_i) out_i[e] = i;
  if (out_j) out_j[e] = j;
  if (out_dist) {
    const float *a = X + (uint64_t)pos_of[i] * dp;
    const float *b = X + (uint64_t)pos_of[j] * dp;
    float s = 0.0f;
    for (uint32_t t = 0; t < d; ++t) {
      const uint32_t r = inv_perm[t];
      const float diff = a[r] - b[r];
      s = __builtin_fmaf(diff, diff, s);
    }
    out_dist[e] = __builtin_sqrtf(s);
  }
}

template <int DP>
void launch_dp(const JoinLaunch &a, hipStream_t s) {
  const uint32_t grid = (uint32_t)((a.n_wu + kWavesPerBlock - 1) / kWavesPerBlock);
  if (grid == 0) return;
  constexpr int kRq = DP <= 24 ? SJ_FP32_RQ_SMALL : (DP <= 64 ? SJ_FP32_RQ_MID : 1);
  if (a.count_only)
    hipLaunchKernelGGL((k_count_fp32<DP, kRq>), dim3(grid), dim3(kBlock), 0, s, a.X, a.orig_id,
                       a.inv_perm, a.wu, a.n_wu, a.runs, a.qlist, a.d, a.lo, a.hi, a.eps2,
                       a.symmetric, a.shortc, a.out, a.capacity, a.cursor, a.rechecks);
  else
    hipLaunchKernelGGL((k_join_fp32<DP, kRq>), dim3(grid), dim3(kBlock), 0, s, a.X, a.orig_id,
                       a.inv_perm, a.wu, a.n_wu, a.runs, a.qlist, a.d, a.lo, a.hi, a.eps2,
                       a.symmetric, a.shortc, a.out, a.capacity, a.cursor, a.rechecks);
  SJ_HIP(hipGetLastError());
}

}  // namespace

uint32_t padded_dim(uint32_t d) {
  if (d == 0 || d > SJ_MAX_DIM) return 0;
  if (d <= 32) return (d + 7) / 8 * 8;
  return (d + 15) / 16 * 16;
}

int fp32_rq_for(uint32_t dp) { return dp <= 24 ? SJ_FP32_RQ_SMALL : (dp <= 64 ? SJ_FP32_RQ_MID : 1); }

void launch_join_fp32(const JoinLaunch &a, hipStream_t s) {
  switch (a.dp) {
    case 8: launch_dp<8>(a, s); break;
    case 16: launch_dp<16>(a, s); break;
    case 24: launch_dp<24>(a, s); break;
    case 32: launch_dp<32>(a, s); break;
    case 48: launch_dp<48>(a, s); break;
    case 64: launch_dp<64>(a, s); break;
    case 80: launch_dp<80>(a, s); break;
    case 96: launch_dp<96>(a, s); break;
    case 112: launch_dp<112>(a, s); break;
    case 128: launch_dp<128>(a, s); break;
    default: fail(SJ_ERR_INVALID_ARG, "unsupported padded dimension");
  }
}

void launch_unpack(const uint64_t *keys, uint64_t count, uint32_t *out_i, uint32_t *out_j,
                   float *out_dist, const float *X, const uint32_t *pos_of,
                   const uint16_t *inv_perm, uint32_t d, uint32_t dp, hipStream_t s,
                   uint32_t ishift) {
  if (!count) return;
  const uint32_t grid = (uint32_t)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_unpack, dim3(grid), dim3(kBlock), 0, s, keys, count, out_i, out_j,
                     out_dist, X, pos_of, inv_perm, d, dp, ishift);
  SJ_HIP(hipGetLastError());
}

}  // namespace sj
