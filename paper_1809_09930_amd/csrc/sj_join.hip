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
#include <type_traits>

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
// Dimension counts after which the short-circuit test runs (the last one is
// DP itself); the norm form keeps prefix norms at exactly these counts.
constexpr int shortc_first(int dp) {
  return dp < (dp <= 24 ? SJ_SHORTC_FIRST_SMALL : SJ_SHORTC_FIRST)
             ? dp
             : (dp <= 24 ? SJ_SHORTC_FIRST_SMALL : SJ_SHORTC_FIRST);
}
constexpr int shortc_step(int dp) { return dp <= 24 ? SJ_SHORTC_STEP_SMALL : SJ_SHORTC_STEP; }
constexpr int n_checkpoints(int dp) {
  return 1 + (dp - shortc_first(dp) + shortc_step(dp) - 1) / shortc_step(dp);
}
constexpr int checkpoint_dim(int dp, int k) {
  return shortc_first(dp) + k * shortc_step(dp) < dp ? shortc_first(dp) + k * shortc_step(dp)
                                                     : dp;
}
// floats per point in the norm form's two tables (checkpoints + 1, padded)
constexpr int norm_row(int dp) {
  return n_checkpoints(dp) + 1 <= 2   ? 2
         : n_checkpoints(dp) + 1 <= 4 ? 4
         : n_checkpoints(dp) + 1 <= 8 ? 8
                                      : 16;
}
static_assert(n_checkpoints(128) + 1 <= 16, "norm table rows hold at most 16 floats");

// Query points per lane by padded dimension (register blocking).
#ifndef SJ_FP32_RQ_SMALL
#define SJ_FP32_RQ_SMALL 2  // dp <= 24
#endif
#ifndef SJ_FP32_RQ_MID
#define SJ_FP32_RQ_MID 1    // dp <= 64
#endif
// Query-box prefilter up to 24 padded dimensions: candidates are first
// tested in batches of 64 (one per lane) against the bounding box of the
// wave's queries over the first kBoxDims dimensions, and only those whose
// lower bound on the squared distance to the box passes `hi` are evaluated
// query by query.  Above 24 dimensions the first 8 hold too little of the
// distance to reject enough (32-D exponential set 44 % slower with the test,
// 2M x 64 and 515k x 90 5 and 14 %), so candidates are swept one by one.
#ifndef SJ_BOX_FILTER
#define SJ_BOX_FILTER 1
#endif
template <int DP>
constexpr bool kBoxOn = SJ_BOX_FILTER && DP <= 24;
// the same for the norm form
#ifndef SJ_NORM_RQ_SMALL
#define SJ_NORM_RQ_SMALL 4
#endif
#ifndef SJ_NORM_RQ_MID
#define SJ_NORM_RQ_MID 1
#endif

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

// dimensions of the query box (the first ones in the variance order)
#ifndef SJ_BOX_DIMS
#define SJ_BOX_DIMS 8
#endif
template <int DP>
constexpr int kBoxDims = DP < SJ_BOX_DIMS ? DP : SJ_BOX_DIMS;

template <int DP, int RQ>
struct Lanes {
  float q[RQ][DP];   // difference form: the query; norm form: -2 x the query
  uint32_t pos[RQ];  // cell-order position of each query (0xffffffff: empty slot)
  uint32_t id[RQ];   // caller index of each query
  float init[RQ];    // difference form: 0 for a live slot, +inf for an empty one
};

template <int DP, int RQ, bool kNorm>
struct NormLanes {  // norm form: the query's increments of its accumulator
  float qa[RQ][n_checkpoints(DP) + 1];
};
template <int DP, int RQ>
struct NormLanes<DP, RQ, false> {};

// The candidate values the first test needs (its first coordinates, and the
// first table value in the norm form), loaded one candidate ahead so the
// scalar loads overlap the previous candidate's arithmetic.  The arrays
// hold one row more than there are points, so the look-ahead past the last
// candidate of a run stays inside them.
template <int DP, bool kNorm>
struct Head {
  float cv[shortc_first(DP)];
  float ct0;
};
template <int DP, bool kNorm>
__device__ __forceinline__ Head<DP, kNorm> load_head(const float *__restrict__ crow,
                                                     const float *__restrict__ ccr) {
  Head<DP, kNorm> h;
#pragma unroll
  for (int t = 0; t < shortc_first(DP); ++t) h.cv[t] = crow[t];
  h.ct0 = kNorm ? ccr[0] : 0.0f;
  return h;
}

// Final decision for query group r of a wave against candidate c: m = lanes
// not rejected, lo_m = lanes proven accepted; the rest of m is rechecked with
// the canonical FP64 predicate.  Accepted pairs are staged (both orders in
// symmetric mode), or only counted.
template <int DP, int RQ, bool kCount>
__device__ __forceinline__ void classify_emit(
    const Lanes<DP, RQ> &L, int r, uint32_t c, uint64_t m, uint64_t lo_m,
    const float *__restrict__ Xq, const float *__restrict__ X, const uint32_t *__restrict__ orig_id,
    const uint16_t *__restrict__ inv_perm, uint32_t d, double eps2, bool symmetric,
    WaveStage &st, uint64_t *__restrict__ out, uint64_t capacity,
    unsigned long long *__restrict__ cursor, uint64_t &n_recheck, uint64_t &n_count) {
  if (m == 0) return;
  if (kCount) {
    n_count += (uint64_t)__builtin_popcountll(m);
    return;
  }
  uint64_t acc = m & lo_m;
  const uint64_t band = m & ~acc;
  if (band) {
    bool ok = false;
    if ((band >> lane_id()) & 1ull)
      ok = canonical_within(Xq, L.pos[r], X, c, inv_perm, d, DP, eps2);
    acc |= ballot(ok);
    n_recheck += (uint64_t)__builtin_popcountll(band);
  }
  if (acc == 0) return;
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

template <int DP, int RQ, bool kFilter, bool kCount, bool kSC>
__device__ __forceinline__ void eval_candidate(
    const Lanes<DP, RQ> &L, const Head<DP, false> &hd, uint32_t c,
    const float *__restrict__ crow, const float *__restrict__ Xq, const float *__restrict__ X,
    const uint32_t *__restrict__ orig_id, const uint16_t *__restrict__ inv_perm, uint32_t d,
    float lo, float hi, double eps2, bool symmetric, WaveStage &st, uint64_t *__restrict__ out,
    uint64_t capacity, unsigned long long *__restrict__ cursor, uint64_t &n_recheck,
    uint64_t &n_count) {
  constexpr int kFirst = shortc_first(DP);
  constexpr int kStep = shortc_step(DP);
  float s[RQ];
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    s[r] = L.init[r];
    if (kFilter) s[r] = (L.pos[r] <= c) ? s[r] : __builtin_inff();
  }
  // dimensions [0, kFirst) for every group
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
#pragma unroll
    for (int t = 0; t < kFirst; ++t) {
      const float diff = L.q[r][t] - hd.cv[t];
      s[r] = __builtin_fmaf(diff, diff, s[r]);
    }
  }
  // remaining dimensions in steps of kStep, each preceded by the test; the
  // wave leaves the candidate once no lane of any group is below hi
#pragma unroll
  for (int t0 = kFirst; t0 < DP; t0 += kStep) {
    if (kSC) {
      // one compare on the lanes' minimum: no scalar mask arithmetic
      float mn = s[0];
#pragma unroll
      for (int r = 1; r < RQ; ++r) mn = __builtin_fminf(mn, s[r]);
      if (ballot(mn <= hi) == 0) return;
    }
    // the last step is shorter when kStep does not divide DP (the bounds
    // are compile-time constants once the loops are unrolled)
    float cv[kStep];
#pragma unroll
    for (int t = 0; t < kStep; ++t)
      if (t0 + t < DP) cv[t] = crow[t0 + t];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
#pragma unroll
      for (int t = 0; t < kStep; ++t) {
        if (t0 + t < DP) {
          const float diff = L.q[r][t0 + t] - cv[t];
          s[r] = __builtin_fmaf(diff, diff, s[r]);
        }
      }
    }
  }
  // classification: s > hi rejects, s <= lo accepts, the band is rechecked
  {
    float mn = s[0];
#pragma unroll
    for (int r = 1; r < RQ; ++r) mn = __builtin_fminf(mn, s[r]);
    if (ballot(mn <= hi) == 0) return;
  }
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const uint64_t m = ballot(s[r] <= hi);
    if (m == 0) continue;
    classify_emit<DP, RQ, kCount>(L, r, c, m, ballot(s[r] <= lo), Xq, X, orig_id, inv_perm, d,
                                  eps2, symmetric, st, out, capacity, cursor, n_recheck, n_count);
  }
}

// Norm form of the same filter.  Each lane's accumulator starts from its
// query's first table value and takes one fused multiply-add per dimension
// with -2 x the query coordinate; at checkpoint k it holds (up to a bounded
// FP32 error) |q|^2_k - 2 q.c_k - s_hi - mu_q,k, and the pair is rejected once
// it exceeds the candidate's table value -|c|^2_k + mu_c,k, i.e. once the
// exact partial sum of squares provably exceeds s_hi.  Between checkpoints
// the accumulator moves to the next reference by one addition; the final
// test against the candidate's lower value proves acceptance.  The tables
// and the margins mu come from k_norm_tables.
template <int DP, int RQ, bool kFilter, bool kCount, bool kSC>
__device__ __forceinline__ void eval_candidate_norm(
    const Lanes<DP, RQ> &L, const NormLanes<DP, RQ, true> &N, const Head<DP, true> &hd,
    uint32_t c, const float *__restrict__ crow, const float *__restrict__ cr,
    const float *__restrict__ Xq, const float *__restrict__ X, const uint32_t *__restrict__ orig_id,
    const uint16_t *__restrict__ inv_perm, uint32_t d, double eps2, bool symmetric,
    WaveStage &st, uint64_t *__restrict__ out, uint64_t capacity,
    unsigned long long *__restrict__ cursor, uint64_t &n_recheck, uint64_t &n_count) {
  constexpr int K = n_checkpoints(DP);
  float a[RQ];
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    a[r] = N.qa[r][0];
    if (kFilter) a[r] = (L.pos[r] <= c) ? a[r] : __builtin_inff();
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int t0 = k == 0 ? 0 : checkpoint_dim(DP, k - 1);
    const int t1 = checkpoint_dim(DP, k);
    float cv[DP];  // the candidate's coordinates [t0, t1)
#pragma unroll
    for (int t = 0; t < DP; ++t)
      if (t >= t0 && t < t1) cv[t] = k == 0 ? hd.cv[t < shortc_first(DP) ? t : 0] : crow[t];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      if (k > 0) a[r] += N.qa[r][k];
#pragma unroll
      for (int t = 0; t < DP; ++t)
        if (t >= t0 && t < t1) a[r] = __builtin_fmaf(L.q[r][t], cv[t], a[r]);
    }
    if (kSC && k + 1 < K) {
      const float ctk = k == 0 ? hd.ct0 : cr[k];
      float mn = a[0];
#pragma unroll
      for (int r = 1; r < RQ; ++r) mn = __builtin_fminf(mn, a[r]);
      if (ballot(mn <= ctk) == 0) return;
    }
  }
  const float rej = K == 1 ? hd.ct0 : cr[K - 1];
  const float acc_t = cr[K];
  {
    float mn = a[0];
#pragma unroll
    for (int r = 1; r < RQ; ++r) mn = __builtin_fminf(mn, a[r]);
    if (ballot(mn <= rej) == 0) return;
  }
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const uint64_t m = ballot(a[r] <= rej);
    if (m == 0) continue;
    classify_emit<DP, RQ, kCount>(L, r, c, m, ballot(a[r] + N.qa[r][K] <= acc_t), Xq, X, orig_id,
                                  inv_perm, d, eps2, symmetric, st, out, capacity, cursor,
                                  n_recheck, n_count);
  }
}

// One wave = one work unit.  kCount: count the pairs the filter cannot
// reject (s <= hi) instead of emitting them.
template <int DP, int RQ, bool kCount, bool kNorm, bool kSC>
__device__ __forceinline__ void join_body(
    const float *__restrict__ X, const uint32_t *__restrict__ orig_id,
    const float *__restrict__ Xq, const uint32_t *__restrict__ qid,
    const uint16_t *__restrict__ inv_perm, const WorkUnit *__restrict__ wus, uint64_t n_wu,
    const uint2 *__restrict__ runs, const uint32_t *__restrict__ qlist, uint32_t d, float lo,
    float hi, double eps2, int symmetric, uint64_t *__restrict__ out,
    uint64_t capacity, unsigned long long *__restrict__ cursor,
    unsigned long long *__restrict__ rechecks, uint64_t (*stage_mem)[kStage],
    const float *__restrict__ QA, const float *__restrict__ CR, uint32_t skip_below,
    unsigned long long *__restrict__ skipped) {
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  const uint64_t u = (uint64_t)blockIdx.x * kWavesPerBlock + w;
  if (u >= n_wu) return;  // whole wave leaves; no workgroup barrier follows
  const WorkUnit wu = wus[u];
  const uint32_t l = lane_id();

  Lanes<DP, RQ> L;
  NormLanes<DP, RQ, kNorm> NL;
  constexpr int NB = kBoxDims<DP>;
  float blo[NB], bhi[NB];  // this lane's part of the query box
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    blo[t] = __builtin_inff();
    bhi[t] = -__builtin_inff();
  }
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const uint32_t slot = wu.q0 + (uint32_t)r * kWave + l;
    const bool live = slot < wu.q1;
    const uint32_t p = live ? (qlist ? qlist[slot] : slot) : 0u;
    L.pos[r] = live ? p : 0xffffffffu;
    L.id[r] = live ? qid[p] : 0u;
    L.init[r] = live ? 0.0f : __builtin_inff();
    const float4 *row = reinterpret_cast<const float4 *>(Xq + (uint64_t)p * DP);
    const float sc = kNorm ? -2.0f : 1.0f;  // exact scaling
#pragma unroll
    for (int t = 0; t < DP / 4; ++t) {
      const float4 v = row[t];
      L.q[r][4 * t + 0] = sc * v.x;
      L.q[r][4 * t + 1] = sc * v.y;
      L.q[r][4 * t + 2] = sc * v.z;
      L.q[r][4 * t + 3] = sc * v.w;
      const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (4 * t + i < NB && live) {
          blo[4 * t + i] = __builtin_fminf(blo[4 * t + i], vv[i]);
          bhi[4 * t + i] = __builtin_fmaxf(bhi[4 * t + i], vv[i]);
        }
      }
    }
    if constexpr (kNorm) {
      const float *qa = QA + (uint64_t)p * norm_row(DP);
#pragma unroll
      for (int k = 0; k <= n_checkpoints(DP); ++k) NL.qa[r][k] = live ? qa[k] : 0.0f;
      if (!live) NL.qa[r][0] = __builtin_inff();
    }
  }
  // the box of the wave's live queries, made wave-uniform (scalar registers)
#pragma unroll
  for (int t = 0; t < (kBoxOn<DP> ? NB : 0); ++t) {
    float a = blo[t], b = bhi[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a = __builtin_fminf(a, __shfl_xor(a, off));
      b = __builtin_fmaxf(b, __shfl_xor(b, off));
    }
    blo[t] = __builtin_bit_cast(float, uniform_u32(__builtin_bit_cast(uint32_t, a)));
    bhi[t] = __builtin_bit_cast(float, uniform_u32(__builtin_bit_cast(uint32_t, b)));
  }
  // in symmetric contiguous mode candidates below q1 need the per-lane
  // "query position <= candidate position" filter; beyond it all pass
  const uint32_t filt_end = (symmetric && !qlist) ? wu.q1 : 0u;

  WaveStage st{kCount ? nullptr : &stage_mem[w][0], 0u};
  uint64_t n_recheck = 0, n_count = 0, n_skip = 0;
  const bool sym = symmetric != 0;
  // live queries of the wave (counted per skipped candidate)
  const uint32_t n_live = uniform_u32(wu.q1 - wu.q0 < (uint32_t)(RQ * kWave)
                                          ? wu.q1 - wu.q0
                                          : (uint32_t)(RQ * kWave));

  for (uint32_t r = wu.run_first; r <= wu.run_last; ++r) {
    const uint2 run = runs[r];
    const uint32_t cb = (r == wu.run_first) ? wu.c_begin : run.x;
    const uint32_t ce = (r == wu.run_last) ? wu.c_end : run.y;
    const uint32_t mid = cb < filt_end ? (ce < filt_end ? ce : filt_end) : cb;
    // candidates [from, to) with the per-lane filter or without; the head
    // of candidate c + 1 is loaded before candidate c is evaluated
    auto sweep = [&](uint32_t from, uint32_t to, auto filter) __attribute__((always_inline)) {
      constexpr bool kF = decltype(filter)::value;
      constexpr int NR = norm_row(DP);
      if (from >= to) return;
      const float *crow = X + (uint64_t)from * DP;
      const float *ccr = kNorm ? CR + (uint64_t)from * NR : nullptr;
      auto eval = [&](const Head<DP, kNorm> &h, uint32_t c) __attribute__((always_inline)) {
        if constexpr (kNorm)
          eval_candidate_norm<DP, RQ, kF, kCount, kSC>(L, NL, h, c, crow, ccr, Xq, X, orig_id,
                                                       inv_perm, d, eps2, sym, st, out, capacity,
                                                       cursor, n_recheck, n_count);
        else
          eval_candidate<DP, RQ, kF, kCount, kSC>(L, h, c, crow, Xq, X, orig_id, inv_perm, d, lo,
                                                  hi, eps2, sym, st, out, capacity, cursor,
                                                  n_recheck, n_count);
      };
      auto next = [&]() __attribute__((always_inline)) {
        crow += DP;
        if (kNorm) ccr += NR;
      };
      if constexpr (kBoxOn<DP>) {
        // batches of 64 candidates: lane l bounds the squared distance from
        // candidate b0 + l to the query box over the first NB dimensions.
        // Every query of the box is at least that far (in FP32 the bound is a
        // sum of at most DP rounded squares, within the error `hi` already
        // allows for), so a candidate with bound > hi is rejected for all of
        // them; the others are evaluated in order, the head of the next one
        // loaded ahead.
        for (uint32_t b0 = from; b0 < to; b0 += kWave) {
          const uint32_t cl = b0 + l < to ? b0 + l : b0;
          const float4 *brow = reinterpret_cast<const float4 *>(X + (uint64_t)cl * DP);
          float lb = 0.0f;
#pragma unroll
          for (int t4 = 0; t4 < NB / 4; ++t4) {
            const float4 v = brow[t4];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float g = __builtin_fmaxf(
                  __builtin_fmaxf(blo[4 * t4 + i] - vv[i], vv[i] - bhi[4 * t4 + i]), 0.0f);
              lb = __builtin_fmaf(g, g, lb);
            }
          }
          bool pass = b0 + l < to && lb <= hi;
          if (skip_below) {
            // candidates of earlier result batches: their pairs were taken there
            const bool early = b0 + l < to && orig_id[cl] < skip_below;
            n_skip += (uint64_t)__builtin_popcountll(ballot(early)) * n_live;
            pass = pass && !early;
          }
          uint64_t keep = ballot(pass);
          if (keep == 0) continue;
          uint32_t c = b0 + (uint32_t)__builtin_ctzll(keep);
          keep &= keep - 1;
          crow = X + (uint64_t)c * DP;
          if (kNorm) ccr = CR + (uint64_t)c * NR;
          Head<DP, kNorm> h = load_head<DP, kNorm>(crow, ccr);
          for (;;) {
            const bool more = keep != 0;
            const uint32_t cn = more ? b0 + (uint32_t)__builtin_ctzll(keep) : c;
            Head<DP, kNorm> hn = h;
            if (more)
              hn = load_head<DP, kNorm>(X + (uint64_t)cn * DP,
                                        kNorm ? CR + (uint64_t)cn * NR : nullptr);
            eval(h, c);
            if (!more) break;
            keep &= keep - 1;
            c = cn;
            h = hn;
            crow = X + (uint64_t)c * DP;
            if (kNorm) ccr = CR + (uint64_t)c * NR;
          }
        }
      } else {
        // one loop without the skip test (every run but the symmetric
        // batches) and one with it
        auto walk = [&](auto skip) __attribute__((always_inline)) {
          Head<DP, kNorm> h = load_head<DP, kNorm>(crow, ccr);
          for (uint32_t c = from; c < to; ++c) {
            const Head<DP, kNorm> hn =
                load_head<DP, kNorm>(crow + DP, kNorm ? ccr + NR : nullptr);
            if (decltype(skip)::value && orig_id[c] < skip_below)
              n_skip += n_live;  // a pair of an earlier result batch
            else
              eval(h, c);
            h = hn;
            next();
          }
        };
        if (skip_below)
          walk(std::true_type{});
        else
          walk(std::false_type{});
      }
    };
    sweep(cb, mid, std::true_type{});
    sweep(mid, ce, std::false_type{});
  }
  stage_flush(st, out, capacity, cursor);
  if (l == 0) {
    if (n_recheck) atomicAdd(rechecks, (unsigned long long)n_recheck);
    if (n_count) atomicAdd(cursor, (unsigned long long)n_count);
    if (n_skip) atomicAdd(skipped, (unsigned long long)n_skip);
  }
}

#define SJ_JOIN_PARAMS                                                                          \
  const float *__restrict__ X, const uint32_t *__restrict__ orig_id,                            \
      const float *__restrict__ Xq, const uint32_t *__restrict__ qid,                           \
      const uint16_t *__restrict__ inv_perm, const WorkUnit *__restrict__ wus, uint64_t n_wu,   \
      const uint2 *__restrict__ runs, const uint32_t *__restrict__ qlist, uint32_t d, float lo, \
      float hi, double eps2, int symmetric, uint64_t *__restrict__ out,                         \
      uint64_t capacity, unsigned long long *__restrict__ cursor,                               \
      unsigned long long *__restrict__ rechecks, const float *__restrict__ QA,                  \
      const float *__restrict__ CR, uint32_t skip_below, unsigned long long *__restrict__ skipped

// The distance kernel (queries Xq against candidates X; Xq = X in a
// self-join): emits result pairs.
template <int DP, int RQ, bool kNorm, bool kSC>
__global__ __launch_bounds__(kBlock) void k_join_fp32(SJ_JOIN_PARAMS) {
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  join_body<DP, RQ, false, kNorm, kSC>(X, orig_id, Xq, qid, inv_perm, wus, n_wu, runs, qlist, d,
                                       lo, hi, eps2, symmetric, out, capacity, cursor, rechecks,
                                       stage_mem, QA, CR, skip_below, skipped);
}

// The estimation kernel (count only) used to size result buffers.
template <int DP, int RQ, bool kNorm, bool kSC>
__global__ __launch_bounds__(kBlock) void k_count_fp32(SJ_JOIN_PARAMS) {
  join_body<DP, RQ, true, kNorm, kSC>(X, orig_id, Xq, qid, inv_perm, wus, n_wu, runs, qlist, d,
                                      lo, hi, eps2, symmetric, out, capacity, cursor, rechecks,
                                      nullptr, QA, CR, skip_below, skipped);
}

// Tables of the norm form, one row of norm_row(DP) floats per point p (the
// remaining entries are 0).  With N_k = sum over the first checkpoint_dim(k)
// coordinates of x^2 (FP64), s_hi / s_lo the bounds on the exact squared
// distance implied by canonical acceptance / rejection, and margins
// mu_q = kappa (4 N_k + 2 s_hi), mu_c = 2 kappa N_k:
//   QA[p][0]   = rd(N_0 - s_hi - mu_q,0)             the accumulator's start
//   QA[p][k]   = rd(T_k - sum of QA[p][0..k-1])       step to reference k
//               (T_k = N_k - s_hi - mu_q,k)
//   QA[p][K]   = ru(N_K-1 - s_lo + mu_q,K-1 - T_K-1')  shift to the accept test
//   CR[p][k]   = ru(-N_k + mu_c,k)                     reject above this
//   CR[p][K]   = rd(-N_K-1 - mu_c,K-1)                  accept at or below this
// (rd / ru: rounding to FP32 towards -inf / +inf).  The accumulated FP32
// error of the accumulator at checkpoint k is at most
// gamma(|start| + sum |steps| + 2 sum |q_t c_t|) <= gamma (4 N_q + 2 s_hi +
// 2 mu + N_c) since the references increase with k; kappa = 4 gamma_{DP+16}
// (2^-24) covers it on both sides, and every rounding above is directed so
// that it only makes a rejection or an acceptance harder.  *nsum collects
// the sum over points of N_K-1 (the caller's choice of form uses the mean).
__device__ __forceinline__ float rd_f32(double v) {
  float f = (float)v;
  if ((double)f > v) {
    const uint32_t b = __builtin_bit_cast(uint32_t, f);  // one step towards -inf
    f = __builtin_bit_cast(float, f > 0.0f ? b - 1u : (f == 0.0f ? 0x80000001u : b + 1u));
  }
  return f;
}
__device__ __forceinline__ float ru_f32(double v) { return -rd_f32(-v); }

template <int DP>
__global__ __launch_bounds__(kBlock) void k_norm_tables(const float *__restrict__ X, uint64_t n,
                                                        double s_hi, double s_lo, double kappa,
                                                        float *__restrict__ QA,
                                                        float *__restrict__ CR,
                                                        double *__restrict__ nsum) {
  constexpr int K = n_checkpoints(DP);
  constexpr int NR = norm_row(DP);
  const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  double N = 0.0;
  if (p < n) {
    const float *row = X + p * DP;
    float *qa = QA + p * NR;
    float *cr = CR + p * NR;
    double running = 0.0;
    int k = 0;
#pragma unroll
    for (int t = 0; t < DP; ++t) {
      const double x = (double)row[t];
      N += x * x;
      if (t + 1 == checkpoint_dim(DP, k)) {
        // the absolute term covers flushed subnormal results
        const double tiny = (double)(DP + 16) * 0x1p-124;
        const double mq = kappa * (4.0 * N + 2.0 * s_hi) + tiny;
        const double mc = 2.0 * kappa * N + tiny;
        const double T = N - s_hi - mq;
        const float step = rd_f32(T - running);
        qa[k] = step;
        running += (double)step;
        cr[k] = ru_f32(-N + mc);
        if (k == K - 1) {
          qa[K] = ru_f32(N - s_lo + mq - running);
          cr[K] = rd_f32(-N - mc);
        }
        ++k;
      }
    }
#pragma unroll
    for (int j = K + 1; j < NR; ++j) {
      qa[j] = 0.0f;
      cr[j] = 0.0f;
    }
  }
  // block sum of N for the mean
  for (int off = 32; off > 0; off >>= 1) N += __shfl_xor(N, off);
  if (lane_id() == 0 && N != 0.0) atomicAdd(nsum, N);
}

__global__ __launch_bounds__(kBlock) void k_unpack(const uint64_t *__restrict__ keys,
                                                   uint64_t count, uint32_t *__restrict__ out_i,
                                                   uint32_t *__restrict__ out_j,
                                                   float *__restrict__ out_dist,
                                                   const float *__restrict__ Xq,
                                                   const uint32_t *__restrict__ qpos_of,
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
    const float *a = Xq + (uint64_t)qpos_of[i] * dp;
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

template <int DP, int kRq, bool kNorm, bool kSC>
void launch_rq(const JoinLaunch &a, uint32_t grid, hipStream_t s) {
  if (a.count_only)
    hipLaunchKernelGGL((k_count_fp32<DP, kRq, kNorm, kSC>), dim3(grid), dim3(kBlock), 0, s, a.X,
                       a.orig_id, a.Xq, a.qid, a.inv_perm, a.wu, a.n_wu, a.runs, a.qlist, a.d,
                       a.lo, a.hi, a.eps2, a.symmetric, a.out, a.capacity, a.cursor, a.rechecks,
                       a.QA, a.CR, a.skip_below, a.skipped);
  else
    hipLaunchKernelGGL((k_join_fp32<DP, kRq, kNorm, kSC>), dim3(grid), dim3(kBlock), 0, s, a.X,
                       a.orig_id, a.Xq, a.qid, a.inv_perm, a.wu, a.n_wu, a.runs, a.qlist, a.d,
                       a.lo, a.hi, a.eps2, a.symmetric, a.out, a.capacity, a.cursor, a.rechecks,
                       a.QA, a.CR, a.skip_below, a.skipped);
  SJ_HIP(hipGetLastError());
}

// Queries per lane: the class default, or one when the cells are small
// (a.rq == 1: a cell's queries would leave most lanes of a wider unit idle).
template <int DP, bool kNorm, bool kSC>
void launch_form(const JoinLaunch &a, hipStream_t s) {
  const uint32_t grid = (uint32_t)((a.n_wu + kWavesPerBlock - 1) / kWavesPerBlock);
  if (grid == 0) return;
  constexpr int kRq = kNorm ? (DP <= 24 ? SJ_NORM_RQ_SMALL : (DP <= 64 ? SJ_NORM_RQ_MID : 1))
                            : (DP <= 24 ? SJ_FP32_RQ_SMALL : (DP <= 64 ? SJ_FP32_RQ_MID : 1));
  if (kRq != 1 && a.rq == 1)
    launch_rq<DP, 1, kNorm, kSC>(a, grid, s);
  else
    launch_rq<DP, kRq, kNorm, kSC>(a, grid, s);
}

template <int DP>
void launch_dp(const JoinLaunch &a, hipStream_t s) {
  if (a.norm) {
    if (a.shortc) launch_form<DP, true, true>(a, s);
    else launch_form<DP, true, false>(a, s);
  } else {
    if (a.shortc) launch_form<DP, false, true>(a, s);
    else launch_form<DP, false, false>(a, s);
  }
}

template <int DP>
void launch_tables_dp(const float *X, uint64_t n, double s_hi, double s_lo, double kappa,
                      float *QA, float *CR, double *nsum, hipStream_t s) {
  const uint32_t grid = (uint32_t)((n + kBlock - 1) / kBlock);
  if (!grid) return;
  hipLaunchKernelGGL(k_norm_tables<DP>, dim3(grid), dim3(kBlock), 0, s, X, n, s_hi, s_lo, kappa,
                     QA, CR, nsum);
  SJ_HIP(hipGetLastError());
}

}  // namespace

uint32_t padded_dim(uint32_t d) {
  if (d == 0 || d > SJ_MAX_DIM) return 0;
  if (d <= 32) return (d + 7) / 8 * 8;
  return (d + 15) / 16 * 16;
}

int fp32_rq_for(uint32_t dp, bool norm, bool small_cells) {
  if (small_cells) return 1;
  if (norm) return dp <= 24 ? SJ_NORM_RQ_SMALL : (dp <= 64 ? SJ_NORM_RQ_MID : 1);
  return dp <= 24 ? SJ_FP32_RQ_SMALL : (dp <= 64 ? SJ_FP32_RQ_MID : 1);
}

int norm_table_row(uint32_t dp) {
  switch (dp) {
    case 8: return norm_row(8);
    case 16: return norm_row(16);
    case 24: return norm_row(24);
    case 32: return norm_row(32);
    case 48: return norm_row(48);
    case 64: return norm_row(64);
    case 80: return norm_row(80);
    case 96: return norm_row(96);
    case 112: return norm_row(112);
    case 128: return norm_row(128);
    default: return 0;
  }
}

void launch_norm_tables(const float *X, uint64_t n, uint32_t dp, double s_hi, double s_lo,
                        double kappa, float *QA, float *CR, double *nsum, hipStream_t s) {
  switch (dp) {
    case 8: launch_tables_dp<8>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 16: launch_tables_dp<16>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 24: launch_tables_dp<24>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 32: launch_tables_dp<32>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 48: launch_tables_dp<48>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 64: launch_tables_dp<64>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 80: launch_tables_dp<80>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 96: launch_tables_dp<96>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 112: launch_tables_dp<112>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    case 128: launch_tables_dp<128>(X, n, s_hi, s_lo, kappa, QA, CR, nsum, s); break;
    default: fail(SJ_ERR_INVALID_ARG, "unsupported padded dimension");
  }
}

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
                   float *out_dist, const float *Xq, const uint32_t *qpos_of, const float *X,
                   const uint32_t *pos_of, const uint16_t *inv_perm, uint32_t d, uint32_t dp,
                   hipStream_t s, uint32_t ishift) {
  if (!count) return;
  const uint32_t grid = (uint32_t)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_unpack, dim3(grid), dim3(kBlock), 0, s, keys, count, out_i, out_j,
                     out_dist, Xq, qpos_of, X, pos_of, inv_perm, d, dp, ishift);
  SJ_HIP(hipGetLastError());
}

}  // namespace sj
