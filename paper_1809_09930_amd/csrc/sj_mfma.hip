// Matrix-core distance filter of the self-join on gfx950: 16-bit operands,
// FP32 accumulation, rigorous error band, FP64 recheck of the band.
//
// Form.  With a fixed centre c, every point is stored as x~ = Q(x - c) in
// FP16 or BF16 (Q = round to nearest; magnitudes below the format's
// smallest normal are flushed to 0).  For a candidate row a and a query
// column b one 32x32 MFMA tile computes
//     D = fl32(n_a) - 2 a~ . b~        (n_a = |a~|^2 in FP64)
// with fl32(n_a) as the tile's initial accumulator, so that D + n_b is the
// squared distance of the quantised points up to the FP32 accumulation
// error and the rounding of n_a (the fold residual |n_a - fl32(n_a)|), both
// inside the band.  The operands are laid out K-contiguous and zero-padded
// to K: A rows [a~ | 0], B columns [-2 b~ | 0]; scaling by -2 is exact.
//
// Band.  Per query b the FP64 preparation below gives thresholds
// Thi(b) >= D for every candidate the canonical predicate accepts, and
// Tlo(b) such that D <= Tlo(b) proves acceptance (derivation in
// k_mfma_thresholds).  D > Thi rejects, D <= Tlo accepts, the rest is
// rechecked with the canonical FP64 predicate, so the pair set is exact.
//
// Tiles.  Rows = 32 consecutive candidate positions, columns = 32 queries;
// a wave holds QB query blocks (B operands and thresholds in registers) and
// streams candidate blocks (A operands) from memory.  Each lane's 16
// accumulators share one query column, so "any pair of this lane below its
// threshold" is one min over 16 values (v_min3) and one compare; only tiles
// with a hit enter the per-element path.
#include "sj_internal.hpp"
#include "sj_mfma.hpp"

#include <algorithm>
#include <cfloat>

namespace sj {

namespace {

constexpr int kStage = 512;

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));
typedef float float4v __attribute__((ext_vector_type(4)));

template <int FMT>
struct Fmt;
template <>
struct Fmt<kFmtF16> {
  typedef _Float16 T;
  typedef half8 V8;
  __device__ static T inf() { return (T)__builtin_inff(); }
  __device__ static float16v mfma(V8 a, V8 b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Fmt<kFmtBF16> {
  typedef __bf16 T;
  typedef bf16x8 V8;
  __device__ static T inf() { return (T)__builtin_inff(); }
  __device__ static float16v mfma(V8 a, V8 b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// Round to the 16-bit format, flushing magnitudes below its smallest
// normal to zero (the error bound budgets for that flush).
template <int FMT>
__device__ __forceinline__ typename Fmt<FMT>::T quantise(double v) {
  const double tiny = FMT == kFmtF16 ? 6.103515625e-05 /* 2^-14 */ : 1.1754943508222875e-38;
  if (__builtin_fabs(v) < tiny) return (typename Fmt<FMT>::T)0.0f;
  // double -> float is exact for the values used here (v is a float
  // difference or a residual of a float-sized sum); float -> 16 bit rounds
  return (typename Fmt<FMT>::T)(float)v;
}

// ---------------------------------------------------------------------------
// Preparation, pass 1: quantised rows, norms and the global maxima.
// ---------------------------------------------------------------------------
// One centred, quantised coordinate (the same value wherever it is needed).
template <int FMT>
__device__ __forceinline__ typename Fmt<FMT>::T prep_coord(float x, float c) {
  const float diff = x - c;  // rounded to FP32: budgeted
  return quantise<FMT>((double)diff);
}

// The operand rows: 8 consecutive K slots per thread, so that the 16-byte
// stores of XA and XB are contiguous across the lanes.  A rows [x~ | 0],
// B columns [-2 x~ | 0] (scaling by -2 is exact); padding rows are zero.
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_mfma_prep(
    const float *__restrict__ X, uint64_t n, uint64_t n_pad, uint32_t d, uint32_t dp,
    uint32_t kp, const float *__restrict__ centre, typename Fmt<FMT>::T *__restrict__ XA,
    typename Fmt<FMT>::T *__restrict__ XB) {
  typedef typename Fmt<FMT>::T T;
  typedef typename Fmt<FMT>::V8 V8;
  const uint32_t kv = kp / 8;  // vectors per row
  const uint64_t total = n_pad * kv;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint64_t p = e / kv;
    const uint32_t k0 = (uint32_t)(e - p * kv) * 8u;
    V8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t t = k0 + (uint32_t)j;
      const T q = p < n && t < d ? prep_coord<FMT>(X[p * dp + t], centre[t]) : (T)0.0f;
      a[j] = q;
      b[j] = (T)(-2.0f * (float)q);  // exact
    }
    reinterpret_cast<V8 *>(XA)[e] = a;
    reinterpret_cast<V8 *>(XB)[e] = b;
  }
}

// Per point, in dimension order: the quantised norm |x~|^2 and the distance
// from the centre, both in FP64.  The norm enters the MFMA as the
// candidate's initial accumulator, rounded to FP32; that rounding is the
// "fold" error of the bound.  Padding rows get the norm +inf (D = +inf for
// every query).  Each lane reads its own row as 16-byte vectors.
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_mfma_norms(
    const float *__restrict__ X, uint64_t n, uint64_t n_pad, uint32_t d, uint32_t dp,
    const float *__restrict__ centre, float *__restrict__ cn, double *__restrict__ norm2,
    double *__restrict__ dist_c, double *__restrict__ fold_err) {
  typedef typename Fmt<FMT>::T T;
  const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n_pad) return;
  if (p >= n) {
    cn[p] = __builtin_inff();
    return;
  }
  const float4 *x4 = reinterpret_cast<const float4 *>(X + p * dp);  // dp: a multiple of 8
  double nn = 0.0, dc = 0.0;
  for (uint32_t t0 = 0; t0 < d; t0 += 4) {
    const float4 v = x4[t0 / 4];
    const float xv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t t = t0 + (uint32_t)j;
      if (t < d) {
        const T q = prep_coord<FMT>(xv[j], centre[t]);
        const double qd = (double)(float)q;
        nn += qd * qd;
        const double e = (double)xv[j] - (double)centre[t];
        dc += e * e;
      }
    }
  }
  const float h = (float)nn;
  cn[p] = h;
  norm2[p] = nn;
  dist_c[p] = __builtin_sqrt(dc);
  fold_err[p] = __builtin_fabs(nn - (double)h);
}

// Maxima of |x - c|, |x~|, n and the fold residual over all points.
// Non-negative doubles compare like their bit patterns.
__global__ __launch_bounds__(kBlock) void k_mfma_maxima(uint64_t n, const double *__restrict__ norm2,
                                                        const double *__restrict__ dist_c,
                                                        const double *__restrict__ fold_err,
                                                        unsigned long long *__restrict__ maxima) {
  unsigned long long m[4] = {0, 0, 0, 0};
  for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * kBlock) {
    const double v[4] = {dist_c[p], __builtin_sqrt(norm2[p]), norm2[p], fold_err[p]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned long long b = __builtin_bit_cast(unsigned long long, v[i]);
      m[i] = b > m[i] ? b : m[i];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(m[i], off);
      m[i] = o > m[i] ? o : m[i];
    }
    if (lane_id() == 0) atomicMax(&maxima[i], m[i]);
  }
}

// ---------------------------------------------------------------------------
// Preparation, pass 2: per-query thresholds.
//
// Notation for a query b and any candidate a:
//   S    exact squared distance of the FP32 points, S64 its canonical FP64
//        value; canonical acceptance is S64 <= eps2, and
//        S64 <= eps2 implies S <= s_hi = eps2/(1-g64), while
//        S <= s_lo = eps2/(1+g64) implies S64 <= eps2 (g64 = gamma_{d+2}(2^-53)).
//   S_q  squared distance of the quantised points a~, b~.
//   Each coordinate error |x~ - (x-c)| <= u|x-c| + eta, u = (1+2^-24)(1+u16)-1
//   (u16 = 2^-11 FP16, 2^-8 BF16; eta = the flush threshold), hence by the
//   triangle inequality |sqrt(S_q) - sqrt(S)| <= Delta_b =
//   u (|b-c| + R) + 2 eta sqrt(d), R = max over points of |x-c|.
//   D = n_a - 2 a~.b~ up to E' = gamma_K(2^-23)(N + F + 2 |b~| Rq) + F + 2^-120
//   (the MFMA starts from fl32(n_a) and adds K exact products in FP32 in
//   any order, even with truncating adds; N, Rq, F = maxima of n_a, |a~|
//   and |n_a - fl32(n_a)|), and S_q = D_exact + n_b.
// Then
//   Thi(b) = (sqrt(s_hi) + Delta_b)^2 - n_b + E'   (canonical accept => D <= Thi)
//   Tlo(b) = (max(0, sqrt(s_lo) - Delta_b))^2 - n_b - E'   (D <= Tlo => accept)
// evaluated in FP64 with a relative margin and rounded outward to FP32.
// ---------------------------------------------------------------------------
// next float above a finite f (one ulp step on the bit pattern)
__device__ __forceinline__ float next_up(float f) {
  if (f == 0.0f) return __builtin_bit_cast(float, 1u);
  const uint32_t b = __builtin_bit_cast(uint32_t, f);
  return __builtin_bit_cast(float, f > 0.0f ? b + 1u : b - 1u);
}
__device__ __forceinline__ float round_up_f32(double v) {
  if (v != v || v == __builtin_inf()) return __builtin_inff();
  if (v == -__builtin_inf()) return -__builtin_inff();
  float f = (float)v;
  if ((double)f < v) f = next_up(f);
  return f;
}
__device__ __forceinline__ float round_down_f32(double v) {
  return -round_up_f32(-v);
}

__global__ __launch_bounds__(kBlock) void k_mfma_thresholds(
    uint64_t n, uint64_t n_pad, MfmaBand band, const double *__restrict__ norm2,
    const double *__restrict__ dist_c, const unsigned long long *__restrict__ maxima,
    float *__restrict__ thi, float *__restrict__ tlo) {
  const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n_pad) return;
  if (p >= n) {
    thi[p] = -__builtin_inff();
    tlo[p] = -__builtin_inff();
    return;
  }
  const double R = __builtin_bit_cast(double, (uint64_t)maxima[0]);
  const double Rq = __builtin_bit_cast(double, (uint64_t)maxima[1]);
  const double N = __builtin_bit_cast(double, (uint64_t)maxima[2]);
  const double F = __builtin_bit_cast(double, (uint64_t)maxima[3]);
  const double nb = norm2[p];
  const double bq = __builtin_sqrt(nb);
  const double delta = band.u * (dist_c[p] + R) + band.eta_term;
  const double E = band.gamma_acc * (N + F + 2.0 * bq * Rq) + F + 0x1p-120;
  const double m = 0x1p-45;
  const double hi_root = __builtin_sqrt(band.s_hi) * (1.0 + m) + delta;
  const double thi_v = (hi_root * hi_root - nb + E) + m * (hi_root * hi_root + nb + E);
  double lo_root = __builtin_sqrt(band.s_lo) * (1.0 - m) - delta;
  double tlo_v;
  if (lo_root <= 0.0) {
    tlo_v = -__builtin_inf();
  } else {
    tlo_v = (lo_root * lo_root - nb - E) - m * (lo_root * lo_root + nb + E);
  }
  thi[p] = round_up_f32(thi_v);
  tlo[p] = round_down_f32(tlo_v);
}

struct Stage {
  uint64_t *buf;
  uint32_t cnt;
};

__device__ __forceinline__ void flush(Stage &st, uint64_t *__restrict__ out, uint64_t capacity,
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

// Where the hit path sends band pairs: a per-wave LDS stage flushed to the
// deferred-recheck list, or (buf == null) nowhere: the pair is rechecked in
// place.
constexpr int kBandStage = 128;
struct BandSink {
  uint64_t *buf;
  uint64_t cap;
  unsigned long long *cursor;
  Stage st;
};

__device__ __forceinline__ float min16(const float16v &v) {
  float a = __builtin_fminf(__builtin_fminf(v[0], v[1]), v[2]);
  float b = __builtin_fminf(__builtin_fminf(v[3], v[4]), v[5]);
  float c = __builtin_fminf(__builtin_fminf(v[6], v[7]), v[8]);
  float e = __builtin_fminf(__builtin_fminf(v[9], v[10]), v[11]);
  float f = __builtin_fminf(__builtin_fminf(v[12], v[13]), v[14]);
  a = __builtin_fminf(__builtin_fminf(a, b), c);
  e = __builtin_fminf(__builtin_fminf(e, f), v[15]);
  return __builtin_fminf(a, e);
}

// Unroll factor of the element loop of the hit path.
#ifndef SJ_HIT_UNROLL
#define SJ_HIT_UNROLL 4
#endif
#define SJ_PRAGMA_(x) _Pragma(#x)
#define SJ_UNROLL_(n) SJ_PRAGMA_(unroll n)
#define SJ_UNROLL(n) SJ_UNROLL_(n)

// Initial accumulator of a 32-row block: element e of a lane belongs to row
// 8*(e/4) + 4*half + e%4, so the lane reads four aligned groups of four
// candidate norms.
__device__ __forceinline__ float16v norm_init(const float *__restrict__ nrm32, uint32_t half) {
  float16v c;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4v q = *reinterpret_cast<const float4v *>(nrm32 + 8 * g + 4 * half);
    c[4 * g + 0] = q[0];
    c[4 * g + 1] = q[1];
    c[4 * g + 2] = q[2];
    c[4 * g + 3] = q[3];
  }
  return c;
}

// Does any element of the QB tiles pass its query's upper threshold?
template <int QB>
__device__ __forceinline__ bool tiles_any(const float16v (&acc)[QB], const float (&th)[QB]) {
  bool any = false;
#pragma unroll
  for (int j = 0; j < QB; ++j) any |= (min16(acc[j]) <= th[j]);
  return any;
}

// Hit path for tiles where hits are common (clustered data: a few result or
// band pairs in most tiles).  No minimum over the tile first: the 16 element
// compares of a query block are the wave masks themselves, taken four
// elements at a time, and only elements with a hit do the row checks and
// the emission.  Rows are valid without a check when the whole 32-row block
// lies before cend.
template <int QB>
__device__ __forceinline__ void tiles_hits_scan(const float16v (&acc)[QB], const float (&th)[QB],
                                                const float (&tl)[QB],
                                                const uint32_t (&qpos)[QB], uint32_t c0,
                                                uint32_t cend, uint32_t half, const MfmaView &v,
                                                Stage &st, BandSink &bs,
                                                uint64_t *__restrict__ out, uint64_t capacity,
                                                unsigned long long *__restrict__ cursor,
                                                uint64_t &n_recheck) {
  const bool sym = v.symmetric != 0;
  const bool full = c0 + 32u <= cend;  // wave-uniform
  const uint32_t cbase = c0 + 4u * half;
#pragma unroll
  for (int j = 0; j < QB; ++j) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      uint64_t hm[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) hm[i] = ballot(acc[j][4 * g + i] <= th[j]);
      if ((hm[0] | hm[1] | hm[2] | hm[3]) == 0) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (hm[i] == 0) continue;
        const int e = 4 * g + i;
        const bool h = acc[j][e] <= th[j];
        const uint32_t cp = cbase + (uint32_t)(8 * g + i);
        const bool ok = h && (full || cp < cend) && (!sym || qpos[j] <= cp);
        bool acc_ok = ok && acc[j][e] <= tl[j];
        const bool band = ok && !acc_ok;
        const uint64_t bm = ballot(band);
        if (bm) {
          if (bs.buf) {  // deferred: the pair waits in the band list
            const uint32_t nb = (uint32_t)__builtin_popcountll(bm);
            if (bs.st.cnt + nb > (uint32_t)kBandStage) flush(bs.st, bs.buf, bs.cap, bs.cursor);
            if (band)
              bs.st.buf[bs.st.cnt + lanes_below(bm)] =
                  v.key_hi | ((uint64_t)qpos[j] << v.pshift) | cp;
            bs.st.cnt += nb;
          } else {
            if (band)
              acc_ok = canonical_within(v.Xq, qpos[j], v.X, cp, v.inv_perm, v.d, v.dp, v.eps2);
            n_recheck += (uint64_t)__builtin_popcountll(bm);
          }
        }
        const uint64_t am = ballot(acc_ok);
        if (am == 0) continue;
        const bool two = acc_ok && sym && qpos[j] != cp;
        const uint64_t m2 = ballot(two);
        const uint32_t total = (uint32_t)(__builtin_popcountll(am) + __builtin_popcountll(m2));
        if (st.cnt + total > (uint32_t)kStage) flush(st, out, capacity, cursor);
        const uint32_t off = st.cnt + lanes_below(am) + lanes_below(m2);
        if (acc_ok) {
          st.buf[off] = v.key_hi | ((uint64_t)qpos[j] << v.pshift) | cp;
          if (two) st.buf[off + 1] = v.key_hi | ((uint64_t)cp << v.pshift) | qpos[j];
        }
        st.cnt += total;
      }
    }
  }
}

// Hit modes of the single-join kernels: kHitsRare tests the minimum of each
// tile first and scans the elements only of tiles with a hit; kHitsFrequent
// goes straight to the element scan.
constexpr int kHitsRare = 0;
constexpr int kHitsFrequent = 1;

// Walks the 32-row candidate blocks of a work unit, run by run.
struct BlockIter {
  const uint2 *runs;
  uint32_t r, r_last, c, ce, c_end_last;
  __device__ __forceinline__ void init(const WorkUnit &wu, const uint2 *rs) {
    runs = rs;
    r = wu.run_first;
    r_last = wu.run_last;
    c_end_last = wu.c_end;
    c = wu.c_begin;
    ce = (r == r_last) ? c_end_last : runs[r].y;
    normalise();
  }
  __device__ __forceinline__ bool valid() const { return c < ce; }
  // move past exhausted runs; leaves c >= ce only when all runs are done
  __device__ __forceinline__ void normalise() {
    while (c >= ce && r < r_last) {
      ++r;
      c = runs[r].x;
      ce = (r == r_last) ? c_end_last : runs[r].y;
    }
  }
  __device__ __forceinline__ void advance() {
    c += 32;
    normalise();
  }
};

// One work unit of the matrix-core filter: QB query column blocks against
// the candidate blocks of the unit's runs.  Accepted pairs are staged as
// keys key_hi | pos_q << pshift | pos_c.
template <int KP, int FMT, int QB, int HM = kHitsRare>
__device__ __forceinline__ void mfma_unit(const MfmaView &v, const WorkUnit &wu, Stage &st,
                                          BandSink &bs, float *__restrict__ nrm,
                                          uint64_t *__restrict__ out, uint64_t capacity,
                                          unsigned long long *__restrict__ cursor,
                                          uint64_t &n_recheck) {
  typedef typename Fmt<FMT>::V8 V8;
  constexpr int KS = KP / 16;   // MFMA K steps
  constexpr int RV = KP / 8;    // 8-element vectors per row
  const V8 *__restrict__ XA = static_cast<const V8 *>(v.XA);
  const V8 *__restrict__ XB = static_cast<const V8 *>(v.XB);
  const uint32_t l = lane_id();
  const uint32_t half = l >> 5, col = l & 31;

  // query columns: B operands, both thresholds, positions
  V8 B[QB][KS];
  float th[QB], tl[QB];
  uint32_t qpos[QB];
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const uint32_t slot = wu.q0 + (uint32_t)j * 32 + col;
    const bool live = slot < wu.q1;
    const uint32_t p = live ? (v.qlist ? v.qlist[slot] : slot) : 0u;
    qpos[j] = live ? p : 0xffffffffu;
    th[j] = live ? v.thi[p] : -__builtin_inff();
    tl[j] = live ? v.tlo[p] : -__builtin_inff();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) B[j][ks] = XB[(uint64_t)p * RV + ks * 2 + half];
  }

  BlockIter it;
  it.init(wu, v.runs);
  if (!it.valid()) return;
  // candidate operands of the current block; the next block's are fetched
  // before the current block's MFMAs so their latency overlaps the math.
  // Rows past the end of the run (at most 31, inside the padded arrays)
  // are dropped in the hit path.
  // The block's candidate norms (the MFMA's initial accumulator) go
  // through the wave's 32-float LDS area, from one row per lane to the
  // accumulator layout.
  V8 A[KS];
  uint32_t c = it.c, ce = it.ce;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) A[ks] = XA[(uint64_t)(c + col) * RV + ks * 2 + half];
  float nc = v.cn[c + col];
  it.advance();
  for (;;) {
    const bool more = it.valid();
    V8 An[KS];
    float ncn = 0.0f;
    const uint32_t cnext = it.c, cen = it.ce;
    if (more) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) An[ks] = XA[(uint64_t)(cnext + col) * RV + ks * 2 + half];
      ncn = v.cn[cnext + col];
      it.advance();
    }
    if (half == 0) nrm[col] = nc;
    __builtin_amdgcn_wave_barrier();
    const float16v c0 = norm_init(nrm, half);
    __builtin_amdgcn_wave_barrier();
    float16v acc[QB];
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      acc[j] = Fmt<FMT>::mfma(A[0], B[j][0], c0);
#pragma unroll
      for (int ks = 1; ks < KS; ++ks) acc[j] = Fmt<FMT>::mfma(A[ks], B[j][ks], acc[j]);
    }
    if constexpr (HM == kHitsFrequent) {
      tiles_hits_scan<QB>(acc, th, tl, qpos, c, ce, half, v, st, bs, out, capacity, cursor,
                          n_recheck);
    } else if (ballot(tiles_any<QB>(acc, th))) {
      tiles_hits_scan<QB>(acc, th, tl, qpos, c, ce, half, v, st, bs, out, capacity, cursor,
                          n_recheck);
    }
    if (!more) break;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) A[ks] = An[ks];
    nc = ncn;
    c = cnext;
    ce = cen;
  }
}

// Per-wave form for indexes with small cells: every wave takes a work unit
// of its own (32 * SJ_WAVE_QB queries of one cell) and streams that unit's
// candidates itself, so cells much smaller than a workgroup's 256 queries do
// not leave most matrix columns empty.
#ifndef SJ_WAVE_QB
#define SJ_WAVE_QB 1
#endif
template <int KP, int FMT, int HM>
__global__ __launch_bounds__(kBlock) void k_join_mfma_wave(MfmaView v,
                                                           const WorkUnit *__restrict__ wus,
                                                           uint64_t n_wu, uint64_t *__restrict__ out,
                                                           uint64_t capacity,
                                                           unsigned long long *__restrict__ cursor,
                                                           unsigned long long *__restrict__ rechecks) {
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  __shared__ uint64_t band_mem[kWavesPerBlock][kBandStage];
  __shared__ __align__(16) float nrm_mem[kWavesPerBlock][32];
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  const uint64_t u = (uint64_t)blockIdx.x * kWavesPerBlock + w;
  if (u >= n_wu) return;  // whole wave leaves; no workgroup barrier follows
  const WorkUnit wu = wus[u];
  Stage st{&stage_mem[w][0], 0u};
  BandSink bs{v.band, v.band_cap, v.band_cursor, Stage{&band_mem[w][0], 0u}};
  uint64_t n_recheck = 0;
  mfma_unit<KP, FMT, SJ_WAVE_QB, HM>(v, wu, st, bs, &nrm_mem[w][0], out, capacity, cursor,
                                     n_recheck);
  flush(st, out, capacity, cursor);
  if (bs.buf) flush(bs.st, bs.buf, bs.cap, bs.cursor);
  if (lane_id() == 0 && n_recheck) atomicAdd(rechecks, (unsigned long long)n_recheck);
}

// Workgroup-cooperative form of the same filter for a single join: the 4
// waves of a workgroup own 4 x 32*QB query columns of one work unit and
// share every candidate chunk of kChunk rows, which is fetched from memory
// once into a double-buffered LDS stage (global -> registers during the
// MFMAs of the previous chunk -> LDS) instead of once per wave.
constexpr int kChunk = 64;  // candidate rows per LDS stage (2 MFMA row blocks)
// LDS row stride of a staged chunk, in 16-byte vectors.  Lanes read the
// same vector of 32 consecutive rows; with an odd stride (RV is even) the
// reads of 8 consecutive rows fall in different bank groups.  Measured: at
// K = 64 the FP16 join on 2M x 64 takes 246 / 284 ms with the padding and
// 288 / 319 without; at K = 16 (a 2-way conflict only) the padded form was
// slower where hits are frequent (207 against 169 ms), so K = 16 keeps the
// dense rows.
constexpr int lds_row_vectors(int rv) { return rv >= 4 ? rv + 1 : rv; }
// query column blocks per wave for K padding up to 64, and above
#ifndef SJ_WG_QB_SMALL
#define SJ_WG_QB_SMALL 2
#endif
#ifndef SJ_WG_QB_LARGE
#define SJ_WG_QB_LARGE 2
#endif
// 1: the MFMAs of a block are issued before the filter of the block before
// it (two accumulator sets); 0: one block at a time
#ifndef SJ_WG_PIPE
#define SJ_WG_PIPE 0
#endif
static_assert(kChunk == 64, "the workgroup kernel pipelines exactly two 32-row blocks per chunk");

template <int KP, int FMT, int QB, int HM>
__global__ __launch_bounds__(kBlock) void k_join_mfma_wg(MfmaView v,
                                                         const WorkUnit *__restrict__ wus,
                                                         uint64_t n_wu, uint64_t *__restrict__ out,
                                                         uint64_t capacity,
                                                         unsigned long long *__restrict__ cursor,
                                                         unsigned long long *__restrict__ rechecks) {
  typedef typename Fmt<FMT>::V8 V8;
  constexpr int KS = KP / 16;                     // MFMA K steps
  constexpr int RV = KP / 8;                      // 8-element vectors per row
  constexpr int CHUNK_VECS = kChunk * RV;         // vectors per LDS stage
  constexpr int PER_THREAD = (CHUNK_VECS + kBlock - 1) / kBlock;
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  constexpr int RS = lds_row_vectors(RV);
  __shared__ V8 tile[2][kChunk * RS];
  __shared__ __align__(16) float tile_n[2][kChunk];  // candidate norms of the chunk
  __shared__ uint64_t band_mem[kWavesPerBlock][kBandStage];
  const uint64_t u = blockIdx.x;
  if (u >= n_wu) return;  // whole workgroup leaves together
  const WorkUnit wu = wus[u];
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  const uint32_t l = lane_id();
  const uint32_t half = l >> 5, col = l & 31;
  const V8 *__restrict__ XA = static_cast<const V8 *>(v.XA);
  const V8 *__restrict__ XB = static_cast<const V8 *>(v.XB);

  // this wave's query columns
  V8 B[QB][KS];
  float th[QB], tl[QB];
  uint32_t qpos[QB];
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const uint32_t slot = wu.q0 + (w * QB + (uint32_t)j) * 32 + col;
    const bool live = slot < wu.q1;
    const uint32_t p = live ? (v.qlist ? v.qlist[slot] : slot) : 0u;
    qpos[j] = live ? p : 0xffffffffu;
    th[j] = live ? v.thi[p] : -__builtin_inff();
    tl[j] = live ? v.tlo[p] : -__builtin_inff();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) B[j][ks] = XB[(uint64_t)p * RV + ks * 2 + half];
  }
  Stage st{&stage_mem[w][0], 0u};
  BandSink bs{v.band, v.band_cap, v.band_cursor, Stage{&band_mem[w][0], 0u}};
  uint64_t n_recheck = 0;

  // chunk walk (uniform over the workgroup)
  uint32_t r = wu.run_first, c = wu.c_begin;
  uint32_t ce = (r == wu.run_last) ? wu.c_end : v.runs[r].y;
  auto normalise = [&]() {
    while (c >= ce && r < wu.run_last) {
      ++r;
      c = v.runs[r].x;
      ce = (r == wu.run_last) ? wu.c_end : v.runs[r].y;
    }
  };
  normalise();
  V8 pre[PER_THREAD];
  float pre_n = 0.0f;
  auto fetch = [&](uint32_t base) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const uint32_t e = threadIdx.x + (uint32_t)i * kBlock;
      if (e < (uint32_t)CHUNK_VECS) pre[i] = XA[(uint64_t)base * RV + e];
    }
    if (threadIdx.x < (uint32_t)kChunk) pre_n = v.cn[base + threadIdx.x];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const uint32_t e = threadIdx.x + (uint32_t)i * kBlock;
      if (e < (uint32_t)CHUNK_VECS) tile[buf][(e / RV) * RS + e % RV] = pre[i];
    }
    if (threadIdx.x < (uint32_t)kChunk) tile_n[buf][threadIdx.x] = pre_n;
  };
  // filter of one 32-row block whose MFMA results are in acc; rows from
  // c0, valid below cend
  auto epilogue = [&](const float16v(&acc)[QB], uint32_t c0,
                      uint32_t cend) __attribute__((always_inline)) {
    if constexpr (HM == kHitsFrequent) {
      tiles_hits_scan<QB>(acc, th, tl, qpos, c0, cend, half, v, st, bs, out, capacity, cursor,
                          n_recheck);
    } else if (ballot(tiles_any<QB>(acc, th))) {
      tiles_hits_scan<QB>(acc, th, tl, qpos, c0, cend, half, v, st, bs, out, capacity, cursor,
                          n_recheck);
    }
  };
  auto block_mfma = [&](int buf, int blk, float16v(&acc)[QB]) __attribute__((always_inline)) {
    V8 A[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) A[ks] = tile[buf][(blk * 32 + col) * RS + ks * 2 + half];
    const float16v c0 = norm_init(&tile_n[buf][blk * 32], half);
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      acc[j] = Fmt<FMT>::mfma(A[0], B[j][0], c0);
#pragma unroll
      for (int ks = 1; ks < KS; ++ks) acc[j] = Fmt<FMT>::mfma(A[ks], B[j][ks], acc[j]);
    }
  };

  if (c >= ce) return;  // empty unit (uniform)
  fetch(c);
  store(0);
  __syncthreads();
  int cur = 0;
  // Software pipeline over the two 32-row blocks of each chunk: the MFMAs
  // of a block are issued before the filter of the block before it, so the
  // matrix unit works while the vector ALU runs the filter.  accA holds the
  // first block of a chunk, accB the second (fixed registers, no copies).
  float16v accA[QB], accB[QB];
  uint32_t prev_c0 = 0, prev_end = 0;  // block held in accB
  bool have_prev = false;
  for (;;) {
    const uint32_t cc = c, cce = ce;
    c += kChunk;
    normalise();
    const bool more = c < ce;
    if (more) fetch(c);
#if SJ_WG_PIPE
    block_mfma(cur, 0, accA);
    if (have_prev) epilogue(accB, prev_c0, prev_end);
    block_mfma(cur, 1, accB);
    epilogue(accA, cc, cce);
    prev_c0 = cc + 32;
    prev_end = cce;
    have_prev = true;
#else
#pragma nounroll
    for (int blk = 0; blk < 2; ++blk) {
      block_mfma(cur, blk, accA);
      epilogue(accA, cc + 32u * (uint32_t)blk, cce);
    }
#endif
    if (!more) break;
    store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
#if SJ_WG_PIPE
  epilogue(accB, prev_c0, prev_end);
#else
  (void)accB;
  (void)prev_c0;
  (void)prev_end;
  (void)have_prev;
#endif
  if (bs.buf) flush(bs.st, bs.buf, bs.cap, bs.cursor);
  flush(st, out, capacity, cursor);
  if (l == 0 && n_recheck) atomicAdd(rechecks, (unsigned long long)n_recheck);
}

// Hit path of QB tiles whose 32 rows are the positions rows[0 .. nrows)
// (rows past nrows are padding with norm +inf): as tiles_hits_scan, with each
// hit's candidate position read from the row table.
template <int QB>
__device__ __forceinline__ void tiles_hits_rows(const float16v (&acc)[QB], const float (&th)[QB],
                                                const float (&tl)[QB],
                                                const uint32_t (&qpos)[QB],
                                                const uint32_t *__restrict__ rows, uint32_t nrows,
                                                uint32_t half, const MfmaView &v, Stage &st,
                                                BandSink &bs, uint64_t *__restrict__ out,
                                                uint64_t capacity,
                                                unsigned long long *__restrict__ cursor,
                                                uint64_t &n_recheck) {
  const bool sym = v.symmetric != 0;
#pragma unroll
  for (int j = 0; j < QB; ++j) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      uint64_t hm[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) hm[i] = ballot(acc[j][4 * g + i] <= th[j]);
      if ((hm[0] | hm[1] | hm[2] | hm[3]) == 0) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (hm[i] == 0) continue;
        const uint32_t ri = (uint32_t)(8 * g + i) + 4u * half;
        const bool live = ri < nrows;
        const uint32_t cp = rows[live ? ri : 0u];
        const bool ok = acc[j][4 * g + i] <= th[j] && live && (!sym || qpos[j] <= cp);
        bool acc_ok = ok && acc[j][4 * g + i] <= tl[j];
        const bool band = ok && !acc_ok;
        const uint64_t bm = ballot(band);
        if (bm) {
          if (bs.buf) {
            const uint32_t nb = (uint32_t)__builtin_popcountll(bm);
            if (bs.st.cnt + nb > (uint32_t)kBandStage) flush(bs.st, bs.buf, bs.cap, bs.cursor);
            if (band)
              bs.st.buf[bs.st.cnt + lanes_below(bm)] =
                  v.key_hi | ((uint64_t)qpos[j] << v.pshift) | cp;
            bs.st.cnt += nb;
          } else {
            if (band)
              acc_ok = canonical_within(v.Xq, qpos[j], v.X, cp, v.inv_perm, v.d, v.dp, v.eps2);
            n_recheck += (uint64_t)__builtin_popcountll(bm);
          }
        }
        const uint64_t am = ballot(acc_ok);
        if (am == 0) continue;
        const bool two = acc_ok && sym && qpos[j] != cp;
        const uint64_t m2 = ballot(two);
        const uint32_t total = (uint32_t)(__builtin_popcountll(am) + __builtin_popcountll(m2));
        if (st.cnt + total > (uint32_t)kStage) flush(st, out, capacity, cursor);
        const uint32_t off = st.cnt + lanes_below(am) + lanes_below(m2);
        if (acc_ok) {
          st.buf[off] = v.key_hi | ((uint64_t)qpos[j] << v.pshift) | cp;
          if (two) st.buf[off + 1] = v.key_hi | ((uint64_t)cp << v.pshift) | qpos[j];
        }
        st.cnt += total;
      }
    }
  }
}

// The workgroup kernel with the query-box prefilter.  The workgroup's
// queries span a box over the first kBoxDims dimensions (FP32 rows, the
// variance order).  The unit's candidate positions are tested 256 at a time
// (one per thread): the squared distance from a candidate to the box bounds
// its squared distance to every query of the workgroup from below, and in
// FP32 the bound is a sum of at most dp rounded squares, within the error
// the FP32 reject threshold `hi` allows for, so a candidate whose bound
// exceeds `hi` is rejected for all of them.  Survivors enter a ring of
// positions in LDS; each chunk of the matrix tiles takes the next 64 of
// them (gathered rows, positions kept beside the rows), so the tiles hold
// only candidates that can be within eps of some query.  The rows of the
// next chunk are fetched during the tiles of the current one, as in
// k_join_mfma_wg.
constexpr int kBoxDims = 8;
constexpr uint32_t kRing = 512;  // >= 127 pending + one window of 256

template <int KP, int FMT, int QB, int HM>
__global__ __launch_bounds__(kBlock) void k_join_mfma_wg_box(MfmaView v,
                                                             const WorkUnit *__restrict__ wus,
                                                             uint64_t n_wu,
                                                             uint64_t *__restrict__ out,
                                                             uint64_t capacity,
                                                             unsigned long long *__restrict__ cursor,
                                                             unsigned long long *__restrict__ rechecks) {
  typedef typename Fmt<FMT>::V8 V8;
  constexpr int KS = KP / 16;
  constexpr int RV = KP / 8;
  constexpr int CHUNK_VECS = kChunk * RV;
  constexpr int PER_THREAD = (CHUNK_VECS + kBlock - 1) / kBlock;
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  constexpr int RS = lds_row_vectors(RV);
  __shared__ V8 tile[2][kChunk * RS];
  __shared__ __align__(16) float tile_n[2][kChunk];
  __shared__ uint32_t tile_pos[2][kChunk];
  __shared__ uint64_t band_mem[kWavesPerBlock][kBandStage];
  __shared__ uint32_t ring[kRing];
  __shared__ float wbox[kWavesPerBlock][2 * kBoxDims];
  __shared__ uint32_t wcnt[kWavesPerBlock];
  const uint64_t u = blockIdx.x;
  if (u >= n_wu) return;  // whole workgroup leaves together
  const WorkUnit wu = wus[u];
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  const uint32_t l = lane_id();
  const uint32_t half = l >> 5, col = l & 31;
  const V8 *__restrict__ XA = static_cast<const V8 *>(v.XA);
  const V8 *__restrict__ XB = static_cast<const V8 *>(v.XB);

  // this wave's query columns, and their part of the box
  V8 B[QB][KS];
  float th[QB], tl[QB];
  uint32_t qpos[QB];
  float blo[kBoxDims], bhi[kBoxDims];
#pragma unroll
  for (int t = 0; t < kBoxDims; ++t) {
    blo[t] = __builtin_inff();
    bhi[t] = -__builtin_inff();
  }
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const uint32_t slot = wu.q0 + (w * QB + (uint32_t)j) * 32 + col;
    const bool live = slot < wu.q1;
    const uint32_t p = live ? (v.qlist ? v.qlist[slot] : slot) : 0u;
    qpos[j] = live ? p : 0xffffffffu;
    th[j] = live ? v.thi[p] : -__builtin_inff();
    tl[j] = live ? v.tlo[p] : -__builtin_inff();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) B[j][ks] = XB[(uint64_t)p * RV + ks * 2 + half];
    const float4 *qr = reinterpret_cast<const float4 *>(v.Xq + (uint64_t)p * v.dp);
#pragma unroll
    for (int t4 = 0; t4 < kBoxDims / 4; ++t4) {
      const float4 x = qr[t4];
      const float xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (live) {
          blo[4 * t4 + i] = __builtin_fminf(blo[4 * t4 + i], xv[i]);
          bhi[4 * t4 + i] = __builtin_fmaxf(bhi[4 * t4 + i], xv[i]);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kBoxDims; ++t) {
    float a = blo[t], b = bhi[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a = __builtin_fminf(a, __shfl_xor(a, off));
      b = __builtin_fmaxf(b, __shfl_xor(b, off));
    }
    if (l == 0) {
      wbox[w][t] = a;
      wbox[w][kBoxDims + t] = b;
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kBoxDims; ++t) {
    float a = wbox[0][t], b = wbox[0][kBoxDims + t];
#pragma unroll
    for (int i = 1; i < kWavesPerBlock; ++i) {
      a = __builtin_fminf(a, wbox[i][t]);
      b = __builtin_fmaxf(b, wbox[i][kBoxDims + t]);
    }
    blo[t] = __builtin_bit_cast(float, uniform_u32(__builtin_bit_cast(uint32_t, a)));
    bhi[t] = __builtin_bit_cast(float, uniform_u32(__builtin_bit_cast(uint32_t, b)));
  }
  const float hi = v.hi;
  Stage st{&stage_mem[w][0], 0u};
  BandSink bs{v.band, v.band_cap, v.band_cursor, Stage{&band_mem[w][0], 0u}};
  uint64_t n_recheck = 0;

  // candidate stream (uniform over the workgroup) and the ring of survivors
  uint32_t r = wu.run_first, c = wu.c_begin;
  uint32_t ce = (r == wu.run_last) ? wu.c_end : v.runs[r].y;
  auto normalise = [&]() {
    while (c >= ce && r < wu.run_last) {
      ++r;
      c = v.runs[r].x;
      ce = (r == wu.run_last) ? wu.c_end : v.runs[r].y;
    }
  };
  normalise();
  uint32_t head = 0, tail = 0;  // ring positions (uniform; differ by <= 383)
  // test windows until at least `want` survivors wait or the stream ends
  auto fill = [&](uint32_t want) __attribute__((always_inline)) {
    while (tail - head < want && c < ce) {
      const uint32_t wl = ce - c < (uint32_t)kBlock ? ce - c : (uint32_t)kBlock;
      const uint32_t p = c + threadIdx.x;
      const bool valid = threadIdx.x < wl;
      const float4 *xr = reinterpret_cast<const float4 *>(v.X + (uint64_t)(valid ? p : c) * v.dp);
      float lb = 0.0f;
#pragma unroll
      for (int t4 = 0; t4 < kBoxDims / 4; ++t4) {
        const float4 x = xr[t4];
        const float xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float g = __builtin_fmaxf(
              __builtin_fmaxf(blo[4 * t4 + i] - xv[i], xv[i] - bhi[4 * t4 + i]), 0.0f);
          lb = __builtin_fmaf(g, g, lb);
        }
      }
      const bool keep = valid && lb <= hi;
      const uint64_t km = ballot(keep);
      if (l == 0) wcnt[w] = (uint32_t)__builtin_popcountll(km);
      __syncthreads();
      uint32_t before = 0, total = 0;
#pragma unroll
      for (int i = 0; i < kWavesPerBlock; ++i) {
        const uint32_t ci = wcnt[i];
        before += (uint32_t)i < w ? ci : 0u;
        total += ci;
      }
      if (keep) ring[(tail + before + lanes_below(km)) % kRing] = p;
      __syncthreads();  // the ring is read and wcnt rewritten after this
      tail += total;
      c += wl;
      normalise();
    }
  };
  V8 pre[PER_THREAD];
  float pre_n = 0.0f;
  uint32_t pre_p = 0;
  // rows [head, head + nr) of the ring into registers (padding rows past nr)
  auto gather = [&](uint32_t nr) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const uint32_t e = threadIdx.x + (uint32_t)i * kBlock;
      if (e < (uint32_t)CHUNK_VECS) {
        const uint32_t rr = e / RV;
        const uint32_t pos = rr < nr ? ring[(head + rr) % kRing] : v.pad_row;
        pre[i] = XA[(uint64_t)pos * RV + e % RV];
      }
    }
    if (threadIdx.x < (uint32_t)kChunk) {
      const uint32_t rr = threadIdx.x;
      pre_p = rr < nr ? ring[(head + rr) % kRing] : v.pad_row;
      pre_n = v.cn[pre_p];
    }
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const uint32_t e = threadIdx.x + (uint32_t)i * kBlock;
      if (e < (uint32_t)CHUNK_VECS) tile[buf][(e / RV) * RS + e % RV] = pre[i];
    }
    if (threadIdx.x < (uint32_t)kChunk) {
      tile_n[buf][threadIdx.x] = pre_n;
      tile_pos[buf][threadIdx.x] = pre_p;
    }
  };
  auto block_mfma = [&](int buf, int blk, float16v(&acc)[QB]) __attribute__((always_inline)) {
    V8 A[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) A[ks] = tile[buf][(blk * 32 + col) * RS + ks * 2 + half];
    const float16v c0 = norm_init(&tile_n[buf][blk * 32], half);
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      acc[j] = Fmt<FMT>::mfma(A[0], B[j][0], c0);
#pragma unroll
      for (int ks = 1; ks < KS; ++ks) acc[j] = Fmt<FMT>::mfma(A[ks], B[j][ks], acc[j]);
    }
  };

  fill(kChunk);
  uint32_t ncur = tail - head < (uint32_t)kChunk ? tail - head : (uint32_t)kChunk;
  if (ncur == 0) return;  // every candidate rejected by the box (uniform)
  gather(ncur);
  store(0);
  head += ncur;
  __syncthreads();
  int cur = 0;
  for (;;) {
    fill(kChunk);
    const uint32_t nn = tail - head < (uint32_t)kChunk ? tail - head : (uint32_t)kChunk;
    if (nn) gather(nn);  // in flight during the tiles below
#pragma nounroll
    for (int blk = 0; blk < 2; ++blk) {
      const uint32_t nb = ncur > 32u * (uint32_t)blk ? ncur - 32u * (uint32_t)blk : 0u;
      if (nb == 0) break;
      float16v acc[QB];
      block_mfma(cur, blk, acc);
      bool any = true;
      if constexpr (HM != kHitsFrequent) any = ballot(tiles_any<QB>(acc, th)) != 0;
      if (any)
        tiles_hits_rows<QB>(acc, th, tl, qpos, &tile_pos[cur][blk * 32],
                            nb < 32u ? nb : 32u, half, v, st, bs, out, capacity, cursor,
                            n_recheck);
    }
    if (!nn) break;
    store(cur ^ 1);
    head += nn;
    __syncthreads();
    cur ^= 1;
    ncur = nn;
  }
  if (bs.buf) flush(bs.st, bs.buf, bs.cap, bs.cursor);
  flush(st, out, capacity, cursor);
  if (l == 0 && n_recheck) atomicAdd(rechecks, (unsigned long long)n_recheck);
}

// Deferred FP64 recheck of the band pairs of a launch: one pair per lane,
// all lanes busy, instead of the few band lanes of one tile element at a
// time.  Accepted pairs are staged and appended like the join's own.
constexpr int kRecheckUnroll = 8;
constexpr int kRecheckBlocksPerCu = 8;

// Appends the pairs of one batch of rechecks (lane: pair q, c, accepted or
// not; both orders in a symmetric join).
__device__ __forceinline__ void emit_rechecked(const MfmaView &v, bool ok, uint32_t q, uint32_t c,
                                               Stage &st, uint64_t *__restrict__ out,
                                               uint64_t capacity,
                                               unsigned long long *__restrict__ cursor) {
  const uint64_t am = ballot(ok);
  if (am == 0) return;
  const bool two = ok && v.symmetric != 0 && q != c;
  const uint64_t m2 = ballot(two);
  const uint32_t n = (uint32_t)(__builtin_popcountll(am) + __builtin_popcountll(m2));
  if (st.cnt + n > (uint32_t)kStage) flush(st, out, capacity, cursor);
  const uint32_t off = st.cnt + lanes_below(am) + lanes_below(m2);
  if (ok) {
    st.buf[off] = v.key_hi | ((uint64_t)q << v.pshift) | c;
    if (two) st.buf[off + 1] = v.key_hi | ((uint64_t)c << v.pshift) | q;
  }
  st.cnt += n;
}

// Rows of up to DPM padded dimensions, NP pairs per batch, one wave per
// workgroup.  The wave first copies the two rows of each of its pairs into
// LDS, 16 bytes per lane and whole row segments per instruction (a row costs
// a few cache-line requests instead of one per dimension and lane); each of
// the first NP lanes then evaluates its pair from LDS in the caller's
// dimension order.  Rows are DPM + 1 floats apart, so the lanes' reads of
// one dimension fall in different banks.  Above 64 padded dimensions a batch
// holds 32 pairs, so that four waves fit a CU's LDS.
template <int DPM, int NP>
__global__ __launch_bounds__(kWave) void k_band_recheck_staged(
    MfmaView v, const unsigned long long *__restrict__ band_count, uint64_t *__restrict__ out,
    uint64_t capacity, unsigned long long *__restrict__ cursor,
    unsigned long long *__restrict__ rechecks) {
  static_assert(NP == kWave || NP == kWave / 2, "one or half a pair per lane");
  constexpr int kRow = DPM + 1;
  constexpr int kVecs = 2 * NP * DPM / 4 / kWave;  // 16-byte loads per lane and batch
  __shared__ float rows[2][NP][kRow];
  __shared__ uint32_t pos[2][NP];
  __shared__ uint64_t stage_mem[kStage];
  __shared__ uint16_t perm[SJ_MAX_DIM];
  const uint32_t l = threadIdx.x;
  for (uint32_t t = l; t < v.d; t += kWave) perm[t] = v.inv_perm[t];
  Stage st{stage_mem, 0u};
  const uint64_t total = *band_count;
  const uint64_t count = total < v.band_cap ? total : v.band_cap;
  const uint32_t dv = v.dp / 4;  // 16-byte vectors per row (dp <= DPM, a multiple of 8)
  for (uint64_t base = (uint64_t)blockIdx.x * NP; base < count;
       base += (uint64_t)gridDim.x * NP) {
    const uint64_t i = base + l;
    const bool live = l < (uint32_t)NP && i < count;
    uint32_t q = 0, c = 0;  // slots past the end stage row 0 and drop it
    if (live) {
      const uint64_t key = v.band[i];
      q = (uint32_t)(key >> 32);
      c = (uint32_t)key;
    }
    if (l < (uint32_t)NP) {
      pos[0][l] = q;
      pos[1][l] = c;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kVecs; ++k) {
      // vector e of the batch's 2 x NP rows of DPM / 4 vectors
      const uint32_t e = (uint32_t)k * kWave + l;
      const uint32_t row = e / (DPM / 4), col = e % (DPM / 4);
      const uint32_t side = row / NP, slot = row % NP;
      if (col < dv) {
        const float *src = side ? v.X : v.Xq;
        const float4 x =
            *reinterpret_cast<const float4 *>(src + (uint64_t)pos[side][slot] * v.dp + col * 4);
        float *dst = &rows[side][slot][col * 4];
        dst[0] = x.x;
        dst[1] = x.y;
        dst[2] = x.z;
        dst[3] = x.w;
      }
    }
    __syncthreads();
    const uint32_t lr = l < (uint32_t)NP ? l : 0u;  // the row a lane evaluates
    const bool ok = live && canonical_within_body<kRecheckUnroll>(&rows[0][lr][0], 0,
                                                                 &rows[1][lr][0], 0, perm, v.d, 0,
                                                                 v.eps2);
    __syncthreads();  // the rows are overwritten by the next batch
    emit_rechecked(v, ok, q, c, st, out, capacity, cursor);
  }
  flush(st, out, capacity, cursor);
  if (blockIdx.x == 0 && l == 0 && count) atomicAdd(rechecks, (unsigned long long)count);
}

// query column blocks per wave of the persistent batched kernel
#ifndef SJ_BATCH_QB
#define SJ_BATCH_QB 1
#endif

// Many independent joins in one persistent launch.  Every wave takes
// `grab` work units at a time from a global queue shared by all jobs and
// runs each with the instantiation of its job's K padding and format.  A
// wave leaves once the queue is exhausted, so the grid drains by itself.
template <int KP, int FMT>
__device__ __forceinline__ void batched_dispatch(const MfmaView &v, const WorkUnit &wu, Stage &st,
                                                 BandSink &bs, float *__restrict__ nrm,
                                                 uint64_t *__restrict__ out, uint64_t capacity,
                                                 unsigned long long *__restrict__ cursor,
                                                 uint64_t &n_recheck) {
  mfma_unit<KP, FMT, SJ_BATCH_QB>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck);
}

__global__ __launch_bounds__(kBlock) void k_join_batched(
    const BatchJob *__restrict__ jobs, const WorkUnit *__restrict__ wus, uint64_t n_wu,
    uint32_t grab, unsigned int *__restrict__ queue, uint64_t *__restrict__ out,
    const unsigned long long *__restrict__ capacity_p, unsigned long long *__restrict__ cursor,
    unsigned long long *__restrict__ rechecks, uint64_t *__restrict__ band, uint64_t band_cap,
    unsigned long long *__restrict__ band_cursor) {
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  __shared__ uint64_t band_mem[kWavesPerBlock][kBandStage];
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  __shared__ __align__(16) float nrm_mem[kWavesPerBlock][32];
  float *nrm = &nrm_mem[w][0];
  Stage st{&stage_mem[w][0], 0u};
  BandSink bs{band, band_cap, band_cursor, Stage{&band_mem[w][0], 0u}};
  uint64_t n_recheck = 0;
  const uint64_t capacity = *capacity_p;
  for (;;) {
    unsigned int u0 = 0;
    if (lane_id() == 0) u0 = atomicAdd(queue, grab);
    u0 = uniform_u32(__shfl(u0, 0));
    if ((uint64_t)u0 >= n_wu) break;
    const uint64_t u1 = (uint64_t)u0 + grab < n_wu ? (uint64_t)u0 + grab : n_wu;
    for (uint64_t u = u0; u < u1; ++u) {
      const WorkUnit wu = wus[u];
      const uint32_t job = wu.pad;
      MfmaView v = jobs[job].view;
      v.key_hi = (uint64_t)job << 40;
      switch (jobs[job].variant) {
        case 0: batched_dispatch<16, kFmtF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 1: batched_dispatch<32, kFmtF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 2: batched_dispatch<48, kFmtF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 3: batched_dispatch<64, kFmtF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 4: batched_dispatch<80, kFmtF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 5: batched_dispatch<16, kFmtBF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 6: batched_dispatch<32, kFmtBF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 7: batched_dispatch<48, kFmtBF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 8: batched_dispatch<64, kFmtBF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        case 9: batched_dispatch<80, kFmtBF16>(v, wu, st, bs, nrm, out, capacity, cursor, n_recheck); break;
        default: break;
      }
    }
  }
  flush(st, out, capacity, cursor);
  if (bs.buf) flush(bs.st, bs.buf, bs.cap, bs.cursor);
  if (lane_id() == 0 && n_recheck) atomicAdd(rechecks, (unsigned long long)n_recheck);
}

// Deferred recheck of a batched launch's band pairs (job << 40 | pos_q << 20
// | pos_c), one per lane, each with its own job's rows.
__global__ __launch_bounds__(kBlock) void k_band_recheck_batched(
    const BatchJob *__restrict__ jobs, const uint64_t *__restrict__ band,
    const unsigned long long *__restrict__ band_count, uint64_t band_cap,
    uint64_t *__restrict__ out, const unsigned long long *__restrict__ capacity_p,
    unsigned long long *__restrict__ cursor, unsigned long long *__restrict__ rechecks) {
  __shared__ uint64_t stage_mem[kWavesPerBlock][kStage];
  const uint32_t w = uniform_u32(threadIdx.x / kWave);
  Stage st{&stage_mem[w][0], 0u};
  const uint64_t capacity = *capacity_p;
  const uint64_t total = *band_count;
  const uint64_t count = total < band_cap ? total : band_cap;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  constexpr uint64_t kMask = (1ull << 20) - 1ull;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + (uint64_t)w * kWave; base < count;
       base += stride) {
    const uint64_t i = base + lane_id();
    bool ok = false, two = false;
    uint64_t key = 0, rkey = 0;
    if (i < count) {
      key = band[i];
      const uint32_t job = (uint32_t)(key >> 40);
      const uint32_t q = (uint32_t)((key >> 20) & kMask), c = (uint32_t)(key & kMask);
      const MfmaView &v = jobs[job].view;
      ok = canonical_within_body<kRecheckUnroll>(v.Xq, q, v.X, c, v.inv_perm, v.d, v.dp, v.eps2);
      two = ok && v.symmetric && q != c;
      rkey = ((uint64_t)job << 40) | ((uint64_t)c << 20) | q;
    }
    const uint64_t am = ballot(ok);
    if (am == 0) continue;
    const uint64_t m2 = ballot(two);
    const uint32_t n = (uint32_t)(__builtin_popcountll(am) + __builtin_popcountll(m2));
    if (st.cnt + n > (uint32_t)kStage) flush(st, out, capacity, cursor);
    const uint32_t off = st.cnt + lanes_below(am) + lanes_below(m2);
    if (ok) {
      st.buf[off] = key;
      if (two) st.buf[off + 1] = rkey;
    }
    st.cnt += n;
  }
  flush(st, out, capacity, cursor);
  if (blockIdx.x == 0 && threadIdx.x == 0 && count) atomicAdd(rechecks, (unsigned long long)count);
}

// Batched keys job << 40 | pos_q << 20 | pos_c -> job << 40 | id_q << 20 | id_c,
// for the first min(*count, capacity) keys.
__global__ __launch_bounds__(kBlock) void k_pos_to_id_batched(
    uint64_t *__restrict__ keys, const unsigned long long *__restrict__ count,
    const unsigned long long *__restrict__ capacity_p, const BatchJob *__restrict__ jobs) {
  const unsigned long long cap = *capacity_p;
  const uint64_t total = *count < cap ? *count : cap;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint64_t k = keys[e];
    const uint32_t job = (uint32_t)(k >> 40);
    const uint32_t *oid = jobs[job].orig_id;
    const uint32_t q = (uint32_t)(k >> 20) & 0xfffffu, c = (uint32_t)k & 0xfffffu;
    keys[e] = ((uint64_t)job << 40) | ((uint64_t)oid[q] << 20) | oid[c];
  }
}

// First and last+1 slot of every job in the sorted batched keys.
__global__ __launch_bounds__(kBlock) void k_job_bounds(
    const uint64_t *__restrict__ keys, const unsigned long long *__restrict__ count,
    const unsigned long long *__restrict__ capacity_p, unsigned long long *__restrict__ first,
    unsigned long long *__restrict__ last) {
  const unsigned long long cap = *capacity_p;
  const uint64_t total = *count < cap ? *count : cap;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t job = (uint32_t)(keys[e] >> 40);
    if (e == 0 || (uint32_t)(keys[e - 1] >> 40) != job) first[job] = e;
    if (e + 1 == total || (uint32_t)(keys[e + 1] >> 40) != job) last[job] = e + 1;
  }
}

// Keys of cell-order positions (q << 32 | c) -> keys of caller indices
// (query positions through qid, candidate positions through orig_id).
__global__ __launch_bounds__(kBlock) void k_pos_to_id(uint64_t *__restrict__ keys, uint64_t count,
                                                      const uint32_t *__restrict__ qid,
                                                      const uint32_t *__restrict__ orig_id) {
  // grid-stride: count may exceed the 2^32 work-items of one dispatch
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < count;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint64_t k = keys[e];
    keys[e] = ((uint64_t)qid[(uint32_t)(k >> 32)] << 32) | orig_id[(uint32_t)k];
  }
}

// K padding up to which the workgroup kernel has the query-box form
constexpr int kBoxMaxKp = 32;

template <int KP, int FMT>
void launch_kp(const MfmaLaunch &a, hipStream_t s) {
  const uint32_t grid = (uint32_t)((a.n_wu + kWavesPerBlock - 1) / kWavesPerBlock);
  if (!grid) return;
  constexpr int QB = KP <= 64 ? SJ_WG_QB_SMALL : SJ_WG_QB_LARGE;
  MfmaView v = a.view;
  if (a.per_wave) {  // one wave per work unit
    if (a.hits_frequent)
      hipLaunchKernelGGL((k_join_mfma_wave<KP, FMT, kHitsFrequent>), dim3(grid), dim3(kBlock), 0,
                         s, v, a.wu, a.n_wu, a.out, a.capacity, a.cursor, a.rechecks);
    else
      hipLaunchKernelGGL((k_join_mfma_wave<KP, FMT, kHitsRare>), dim3(grid), dim3(kBlock), 0, s,
                         v, a.wu, a.n_wu, a.out, a.capacity, a.cursor, a.rechecks);
  } else if (KP <= kBoxMaxKp && a.box) {  // one workgroup per unit, query-box prefilter
    if constexpr (KP <= kBoxMaxKp) {
      if (a.hits_frequent)
        hipLaunchKernelGGL((k_join_mfma_wg_box<KP, FMT, QB, kHitsFrequent>),
                           dim3((uint32_t)a.n_wu), dim3(kBlock), 0, s, v, a.wu, a.n_wu, a.out,
                           a.capacity, a.cursor, a.rechecks);
      else
        hipLaunchKernelGGL((k_join_mfma_wg_box<KP, FMT, QB, kHitsRare>), dim3((uint32_t)a.n_wu),
                           dim3(kBlock), 0, s, v, a.wu, a.n_wu, a.out, a.capacity, a.cursor,
                           a.rechecks);
    }
  } else {  // one workgroup per work unit (4 waves x 32*QB queries)
    if (a.hits_frequent)
      hipLaunchKernelGGL((k_join_mfma_wg<KP, FMT, QB, kHitsFrequent>), dim3((uint32_t)a.n_wu),
                         dim3(kBlock), 0, s, v, a.wu, a.n_wu, a.out, a.capacity, a.cursor,
                         a.rechecks);
    else
      hipLaunchKernelGGL((k_join_mfma_wg<KP, FMT, QB, kHitsRare>), dim3((uint32_t)a.n_wu),
                         dim3(kBlock), 0, s, v, a.wu, a.n_wu, a.out, a.capacity, a.cursor,
                         a.rechecks);
  }
  SJ_HIP(hipGetLastError());
}

template <int FMT>
void launch_fmt(const MfmaLaunch &a, hipStream_t s) {
  switch (a.kp) {
    case 16: launch_kp<16, FMT>(a, s); break;
    case 32: launch_kp<32, FMT>(a, s); break;
    case 48: launch_kp<48, FMT>(a, s); break;
    case 64: launch_kp<64, FMT>(a, s); break;
    case 80: launch_kp<80, FMT>(a, s); break;
    case 96: launch_kp<96, FMT>(a, s); break;
    case 112: launch_kp<112, FMT>(a, s); break;
    case 128: launch_kp<128, FMT>(a, s); break;
    case 144: launch_kp<144, FMT>(a, s); break;
    default: fail(SJ_ERR_INVALID_ARG, "unsupported MFMA K padding");
  }
}

}  // namespace

uint32_t mfma_kp(uint32_t d) { return (d + 15) / 16 * 16; }

int mfma_qb(uint32_t) { return SJ_BATCH_QB; }

uint32_t mfma_wave_queries() { return 32u * SJ_WAVE_QB; }

uint32_t mfma_wg_queries(uint32_t kp) {
  return (uint32_t)(kWavesPerBlock * 32 * (kp <= 64 ? SJ_WG_QB_SMALL : SJ_WG_QB_LARGE));
}

void launch_mfma_prep(int fmt, const float *X, uint64_t n, uint64_t n_pad, uint32_t d, uint32_t dp,
                      uint32_t kp, const float *centre, void *XA, void *XB, float *cn,
                      double *norm2, double *dist_c, double *fold_err,
                      unsigned long long *maxima, hipStream_t s) {
  const uint32_t grid = (uint32_t)((n_pad + kBlock - 1) / kBlock);
  if (!grid) return;
  const uint32_t grid_rows =
      (uint32_t)std::min<uint64_t>((n_pad * (kp / 8) + kBlock - 1) / kBlock, 1u << 20);
  if (fmt == kFmtF16) {
    hipLaunchKernelGGL(k_mfma_prep<kFmtF16>, dim3(grid_rows), dim3(kBlock), 0, s, X, n, n_pad, d,
                       dp, kp, centre, (_Float16 *)XA, (_Float16 *)XB);
    hipLaunchKernelGGL(k_mfma_norms<kFmtF16>, dim3(grid), dim3(kBlock), 0, s, X, n, n_pad, d, dp,
                       centre, cn, norm2, dist_c, fold_err);
  } else {
    hipLaunchKernelGGL(k_mfma_prep<kFmtBF16>, dim3(grid_rows), dim3(kBlock), 0, s, X, n, n_pad,
                       d, dp, kp, centre, (__bf16 *)XA, (__bf16 *)XB);
    hipLaunchKernelGGL(k_mfma_norms<kFmtBF16>, dim3(grid), dim3(kBlock), 0, s, X, n, n_pad, d, dp,
                       centre, cn, norm2, dist_c, fold_err);
  }
  SJ_HIP(hipGetLastError());
  SJ_HIP(hipMemsetAsync(maxima, 0, 4 * sizeof(unsigned long long), s));
  const uint32_t g2 = (uint32_t)std::min<uint64_t>((n + kBlock - 1) / kBlock, 1024);
  if (g2) {
    hipLaunchKernelGGL(k_mfma_maxima, dim3(g2), dim3(kBlock), 0, s, n, norm2, dist_c, fold_err,
                       maxima);
    SJ_HIP(hipGetLastError());
  }
}

void launch_mfma_thresholds(uint64_t n, uint64_t n_pad, const MfmaBand &band, const double *norm2,
                            const double *dist_c, const unsigned long long *maxima, float *thi,
                            float *tlo, hipStream_t s) {
  const uint32_t grid = (uint32_t)((n_pad + kBlock - 1) / kBlock);
  if (!grid) return;
  hipLaunchKernelGGL(k_mfma_thresholds, dim3(grid), dim3(kBlock), 0, s, n, n_pad, band, norm2,
                     dist_c, maxima, thi, tlo);
  SJ_HIP(hipGetLastError());
}

void launch_pos_to_id(uint64_t *keys, uint64_t count, const uint32_t *qid,
                      const uint32_t *orig_id, hipStream_t s) {
  if (!count) return;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((count + kBlock - 1) / kBlock, 1u << 20);
  hipLaunchKernelGGL(k_pos_to_id, dim3(grid), dim3(kBlock), 0, s, keys, count, qid, orig_id);
  SJ_HIP(hipGetLastError());
}

int batched_variant(uint32_t kp, int fmt) {
  int base = fmt == kFmtF16 ? 0 : 5;
  switch (kp) {
    case 16: return base + 0;
    case 32: return base + 1;
    case 48: return base + 2;
    case 64: return base + 3;
    case 80: return base + 4;
    default: return -1;
  }
}

int batched_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_join_batched, kBlock, 0) !=
      hipSuccess) {
    (void)hipGetLastError();
    blocks = 2;
  }
  return blocks > 0 ? blocks : 1;
}

void launch_join_batched(const BatchJob *jobs, const WorkUnit *wus, uint64_t n_wu, uint32_t grab,
                         unsigned int *queue, uint64_t *out, const unsigned long long *capacity,
                         unsigned long long *cursor, unsigned long long *rechecks, uint32_t grid,
                         uint64_t *band, uint64_t band_cap, unsigned long long *band_cursor,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_join_batched, dim3(grid), dim3(kBlock), 0, s, jobs, wus, n_wu, grab, queue,
                     out, capacity, cursor, rechecks, band, band_cap, band_cursor);
  SJ_HIP(hipGetLastError());
}

void launch_band_recheck_batched(const BatchJob *jobs, const uint64_t *band,
                                 const unsigned long long *band_count, uint64_t band_cap,
                                 uint64_t *out, const unsigned long long *capacity,
                                 unsigned long long *cursor, unsigned long long *rechecks,
                                 uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_band_recheck_batched, dim3(grid), dim3(kBlock), 0, s, jobs, band,
                     band_count, band_cap, out, capacity, cursor, rechecks);
  SJ_HIP(hipGetLastError());
}

void launch_pos_to_id_batched(uint64_t *keys, const unsigned long long *count,
                              const unsigned long long *capacity, const BatchJob *jobs,
                              uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pos_to_id_batched, dim3(grid), dim3(kBlock), 0, s, keys, count, capacity,
                     jobs);
  SJ_HIP(hipGetLastError());
}

void launch_job_bounds(const uint64_t *keys, const unsigned long long *count,
                       const unsigned long long *capacity, unsigned long long *first,
                       unsigned long long *last, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_job_bounds, dim3(grid), dim3(kBlock), 0, s, keys, count, capacity, first,
                     last);
  SJ_HIP(hipGetLastError());
}

void launch_band_recheck(const MfmaView &v, uint64_t *out, uint64_t capacity,
                         unsigned long long *cursor, unsigned long long *rechecks, hipStream_t s) {
  int dev = 0, cus = 256;
  SJ_HIP(hipGetDevice(&dev));
  SJ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const dim3 grid((uint32_t)cus * kRecheckBlocksPerCu);
  if (v.dp <= 32)
    hipLaunchKernelGGL((k_band_recheck_staged<32, kWave>), grid, dim3(kWave), 0, s, v,
                       v.band_cursor, out, capacity, cursor, rechecks);
  else if (v.dp <= 64)
    hipLaunchKernelGGL((k_band_recheck_staged<64, kWave>), grid, dim3(kWave), 0, s, v,
                       v.band_cursor, out, capacity, cursor, rechecks);
  else  // 32 pairs per batch: 33 KB of rows, four waves per CU
    hipLaunchKernelGGL((k_band_recheck_staged<SJ_MAX_DIM, kWave / 2>), grid, dim3(kWave), 0, s, v,
                       v.band_cursor, out, capacity, cursor, rechecks);
  SJ_HIP(hipGetLastError());
}

void launch_join_mfma(const MfmaLaunch &a, hipStream_t s) {
  if (a.fmt == kFmtF16) launch_fmt<kFmtF16>(a, s);
  else launch_fmt<kFmtBF16>(a, s);
}

}  // namespace sj
