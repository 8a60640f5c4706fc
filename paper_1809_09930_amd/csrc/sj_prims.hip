// Device-wide primitives: exclusive prefix sum and stable LSD radix sort.
// Both are plain gfx950 kernels (wave64, 256-thread workgroups, LDS staging).
#include "sj_internal.hpp"

#include <algorithm>
#include <vector>

namespace sj {

namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // 2048 values per workgroup

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T u = __shfl_up(v, off);
    if (l >= (uint32_t)off) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread over the workgroup; *total gets
// the workgroup sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total) {
  __shared__ T wsum[kWavesPerBlock];
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_scan(v);
  if (lane_id() == kWave - 1) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T *__restrict__ in,
                                                        uint64_t n,
                                                        T *__restrict__ sums) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  T acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    if (idx < n) acc += in[idx];
  }
  T total;
  (void)block_exclusive_scan(acc, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of a 2048-value tile per workgroup, plus the workgroup's
// offset (offsets[blockIdx.x], or 0).  The last workgroup writes the grand
// total when `total` is non-null.  in == out is allowed.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_tile(const T *in, T *out, uint64_t n,
                                                      const T *__restrict__ offsets,
                                                      T *__restrict__ total) {
  __shared__ T tile[kScanTile];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    tile[i * kBlock + threadIdx.x] = idx < n ? in[idx] : T(0);
  }
  __syncthreads();
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    T t = tile[threadIdx.x * kScanItems + i];
    v[i] = s;
    s += t;
  }
  T btotal;
  T excl = block_exclusive_scan(s, &btotal);
  const T off = offsets ? offsets[blockIdx.x] : T(0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) tile[threadIdx.x * kScanItems + i] = v[i] + excl + off;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    if (idx < n) out[idx] = tile[i * kBlock + threadIdx.x];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + btotal;
}

template <typename T>
size_t scan_levels_bytes(uint64_t n) {
  size_t bytes = 0;
  while (n > (uint64_t)kScanTile) {
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    bytes += ((nb * sizeof(T) + 255) / 256) * 256;
    n = nb;
  }
  return bytes + 256;
}

template <typename T>
void scan_impl(const T *in, T *out, uint64_t n, T *d_total, char *tmp, hipStream_t s) {
  if (n == 0) {
    if (d_total) SJ_HIP(hipMemsetAsync(d_total, 0, sizeof(T), s));
    return;
  }
  if (n <= (uint64_t)kScanTile) {
    hipLaunchKernelGGL(k_scan_tile<T>, dim3(1), dim3(kBlock), 0, s, in, out, n,
                       (const T *)nullptr, d_total);
    SJ_HIP(hipGetLastError());
    return;
  }
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  T *sums = reinterpret_cast<T *>(tmp);
  char *rest = tmp + ((nb * sizeof(T) + 255) / 256) * 256;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)nb), dim3(kBlock), 0, s, in, n, sums);
  SJ_HIP(hipGetLastError());
  scan_impl<T>(sums, sums, nb, (T *)nullptr, rest, s);
  hipLaunchKernelGGL(k_scan_tile<T>, dim3((uint32_t)nb), dim3(kBlock), 0, s, in, out, n,
                     (const T *)sums, d_total);
  SJ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Radix sort: 8-bit digits, 4096 keys per workgroup (4 waves x 16 rounds of
// 64 consecutive keys).  Ranks inside a workgroup are found with the wave
// "multisplit": one ballot per digit bit gives each lane the mask of lanes
// holding the same digit, so equal digits keep their input order (stable).
// Digits are BITS <= 8 wide; narrower digits with the same number of passes
// give longer runs of equal digits per tile (better coalesced writes) and
// fewer ballots.
// ---------------------------------------------------------------------------
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRsRounds = 16;
constexpr int kRsTile = kBlock * kRsRounds;  // 4096 keys per workgroup with values
// rounds of a keys-only sort (no value array in LDS leaves room for a larger tile)
#ifndef SJ_RS_ROUNDS_KEYS
#define SJ_RS_ROUNDS_KEYS 16
#endif
constexpr int kRsRoundsKeys = SJ_RS_ROUNDS_KEYS;

// When d_count is non-null only the first min(*d_count, n) keys take part.
__device__ __forceinline__ uint64_t live_count(uint64_t n, const unsigned long long *d_count) {
  return d_count ? (*d_count < n ? (uint64_t)*d_count : n) : n;
}

template <int BITS, int R>
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                    uint64_t n_cap, int shift,
                                                    uint64_t *__restrict__ hist,
                                                    uint32_t nblocks,
                                                    const unsigned long long *__restrict__ d_count) {
  __shared__ uint32_t cnt[kWavesPerBlock][kRadixBins];
  const uint64_t n = live_count(n_cap, d_count);
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kWavesPerBlock * kRadixBins; i += kBlock)
    (&cnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * (kBlock * R);
#pragma unroll 4
  for (int r = 0; r < R; ++r) {
    uint64_t idx = base + (uint64_t)r * kBlock + threadIdx.x;
    if (idx < n) {
      uint32_t dg = (uint32_t)(keys[idx] >> shift) & ((1u << BITS) - 1u);
      atomicAdd(&cnt[w][dg], 1u);
    }
  }
  __syncthreads();
  for (int dg = threadIdx.x; dg < (1 << BITS); dg += kBlock) {
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) t += cnt[i][dg];
    hist[(uint64_t)dg * nblocks + blockIdx.x] = t;  // 64-bit: offsets may pass 2^32
  }
}

template <bool kVals, int BITS, int R>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint64_t n_cap, int shift,
    const uint64_t *__restrict__ offs, uint32_t nblocks,
    const unsigned long long *__restrict__ d_count) {
  __shared__ uint32_t cnt[kWavesPerBlock][kRadixBins];
  __shared__ uint32_t woff[kWavesPerBlock][kRadixBins];
  __shared__ uint32_t dbase[kRadixBins];   // first slot of each digit in the tile
  __shared__ uint64_t gbase[kRadixBins];   // first global slot of each digit
  constexpr int kTile = kBlock * R;
  __shared__ uint64_t tkey[kTile];
  __shared__ uint32_t tval[kVals ? kTile : 1];
  const int w = threadIdx.x / kWave;
  const uint32_t l = lane_id();
  for (int i = threadIdx.x; i < kWavesPerBlock * kRadixBins; i += kBlock)
    (&cnt[0][0])[i] = 0;
  __syncthreads();

  // 1. rank every key among equal digits of its wave, in input order
  const uint64_t n = live_count(n_cap, d_count);
  const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
  const uint64_t base = tile0 + (uint64_t)w * (kTile / kWavesPerBlock);
  uint64_t key[R];
  uint32_t val[R];
  uint32_t rank[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t idx = base + (uint64_t)r * kWave + l;
    const bool valid = idx < n;
    key[r] = valid ? kin[idx] : 0ull;
    if (kVals) val[r] = valid ? vin[idx] : 0u;
    const uint32_t dg = (uint32_t)(key[r] >> shift) & ((1u << BITS) - 1u);
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t below = lanes_below(peers);
    uint32_t before = 0;
    if (valid) before = cnt[w][dg];
    rank[r] = before + below;
    // all lanes of the wave have read the counter before its leader
    // (lowest lane of the digit group) updates it
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) cnt[w][dg] = before + (uint32_t)__builtin_popcountll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // 2. per digit: offsets of the waves' shares, the tile-local start and the
  //    global start (one digit per thread)
  {
    const uint32_t dg = threadIdx.x;
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
      woff[i][dg] = sum;
      sum += cnt[i][dg];
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<uint32_t>(sum, &total);
    dbase[dg] = ex;
    if (dg < (1u << BITS)) gbase[dg] = offs[(uint64_t)dg * nblocks + blockIdx.x];
  }
  __syncthreads();
  // 3. place the keys digit-major in LDS
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t idx = base + (uint64_t)r * kWave + l;
    if (idx < n) {
      const uint32_t dg = (uint32_t)(key[r] >> shift) & ((1u << BITS) - 1u);
      const uint32_t lp = dbase[dg] + woff[w][dg] + rank[r];
      tkey[lp] = key[r];
      if (kVals) tval[lp] = val[r];
    }
  }
  __syncthreads();
  // 4. write the tile out in digit order: consecutive threads write
  //    consecutive slots of each digit's run
  const uint32_t valid_keys =
      tile0 >= n ? 0u
                 : (uint32_t)((n - tile0) < (uint64_t)kTile ? (n - tile0) : (uint64_t)kTile);
  for (uint32_t i = threadIdx.x; i < valid_keys; i += kBlock) {
    const uint64_t k = tkey[i];
    const uint32_t dg = (uint32_t)(k >> shift) & ((1u << BITS) - 1u);
    const uint64_t pos = gbase[dg] + (i - dbase[dg]);
    kout[pos] = k;
    if (kVals) vout[pos] = tval[i];
  }
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t count, unsigned long long v) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = v;
}
__global__ void k_copy_u64(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint64_t n,
                           const unsigned long long *__restrict__ d_count) {
  const uint64_t m = live_count(n, d_count);
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * kBlock)
    out[i] = in[i];
}

__global__ void k_iota_strided(uint32_t *out, uint64_t count, uint64_t stride, uint32_t run) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) out[i] = (uint32_t)((i / run) * stride + i % run);
}
__global__ void k_widen(const uint32_t *__restrict__ in, uint64_t *__restrict__ out, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) out[i] = in[i];
}
__global__ void k_narrow(const uint64_t *__restrict__ in, uint32_t *__restrict__ out, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) out[i] = (uint32_t)in[i];
}

// Stream split of result keys: every entry gives up to two keys for `out`
// and one for `spill` (Classify returns them).  A block takes
// kSplitRounds * kBlock consecutive entries, each wave kSplitRounds rounds of
// 64; the block counts its outputs first, takes its slots with one atomic
// per stream, and writes every round's keys to consecutive slots.  Counts go
// on past the capacities; keys beyond them are dropped.
constexpr uint32_t kSplitRounds = 64;
constexpr uint32_t kSplitTile = kSplitRounds * kBlock;

struct SplitKeys {
  bool a1, a2, sp;        // out gets v1 / v2, spill gets vs
  uint64_t v1, v2, vs;
};

template <class Classify>
__device__ __forceinline__ void split_tile(const uint64_t *__restrict__ in, uint64_t n,
                                           Classify f, uint64_t *__restrict__ out,
                                           unsigned long long *__restrict__ out_cnt,
                                           uint64_t out_cap, uint64_t *__restrict__ spill,
                                           unsigned long long *__restrict__ spill_cnt,
                                           uint64_t spill_cap) {
  constexpr uint32_t kW = kBlock / kWave;
  __shared__ uint32_t w_out[kW], w_sp[kW];
  __shared__ unsigned long long b_out, b_sp;
  const uint32_t w = threadIdx.x / kWave, l = lane_id();
  const uint64_t base = (uint64_t)blockIdx.x * kSplitTile + (uint64_t)w * kSplitRounds * kWave;
  uint32_t c_out = 0, c_sp = 0;
  for (uint32_t r = 0; r < kSplitRounds; ++r) {
    const uint64_t e = base + (uint64_t)r * kWave + l;
    const bool valid = e < n;
    const SplitKeys k = f(valid, valid ? in[e] : 0ull);
    c_out += (uint32_t)(__builtin_popcountll(ballot(k.a1)) + __builtin_popcountll(ballot(k.a2)));
    c_sp += (uint32_t)__builtin_popcountll(ballot(k.sp));
  }
  if (l == 0) {
    w_out[w] = c_out;
    w_sp[w] = c_sp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t so = 0, ss = 0;
    for (uint32_t i = 0; i < kW; ++i) {
      const uint32_t to = w_out[i], ts = w_sp[i];
      w_out[i] = so;
      w_sp[i] = ss;
      so += to;
      ss += ts;
    }
    b_out = so ? atomicAdd(out_cnt, (unsigned long long)so) : 0ull;
    b_sp = ss ? atomicAdd(spill_cnt, (unsigned long long)ss) : 0ull;
  }
  __syncthreads();
  uint64_t po = b_out + w_out[w], ps = b_sp + w_sp[w];
  for (uint32_t r = 0; r < kSplitRounds; ++r) {
    const uint64_t e = base + (uint64_t)r * kWave + l;
    const bool valid = e < n;
    const SplitKeys k = f(valid, valid ? in[e] : 0ull);
    const uint64_t m1 = ballot(k.a1), m2 = ballot(k.a2), ms = ballot(k.sp);
    if (k.a1) {
      const uint64_t p = po + lanes_below(m1);
      if (p < out_cap) out[p] = k.v1;
    }
    po += (uint64_t)__builtin_popcountll(m1);
    if (k.a2) {
      const uint64_t p = po + lanes_below(m2);
      if (p < out_cap) out[p] = k.v2;
    }
    po += (uint64_t)__builtin_popcountll(m2);
    if (k.sp) {
      const uint64_t p = ps + lanes_below(ms);
      if (p < spill_cap) spill[p] = k.vs;
    }
    ps += (uint64_t)__builtin_popcountll(ms);
  }
}

__global__ __launch_bounds__(kBlock) void k_mirror_split(
    const uint64_t *__restrict__ in, uint64_t n, uint32_t i1, uint64_t *__restrict__ out,
    unsigned long long *__restrict__ out_cnt, uint64_t out_cap, uint64_t *__restrict__ spill,
    unsigned long long *__restrict__ spill_cnt, uint64_t spill_cap) {
  auto f = [i1](bool valid, uint64_t key) {
    const uint32_t i = (uint32_t)(key >> 32), j = (uint32_t)key;
    const bool keep = valid && j >= i;
    const bool mirror = keep && j > i;
    const uint64_t mk = ((uint64_t)j << 32) | i;
    return SplitKeys{keep, mirror && j < i1, mirror && j >= i1, key, mk, mk};
  };
  split_tile(in, n, f, out, out_cnt, out_cap, spill, spill_cnt, spill_cap);
}

__global__ __launch_bounds__(kBlock) void k_spill_take(
    const uint64_t *__restrict__ spill_in, uint64_t n, uint32_t i1, uint64_t *__restrict__ out,
    unsigned long long *__restrict__ out_cnt, uint64_t out_cap, uint64_t *__restrict__ spill_out,
    unsigned long long *__restrict__ spill_cnt, uint64_t spill_cap) {
  auto f = [i1](bool valid, uint64_t key) {
    const bool now = valid && (uint32_t)(key >> 32) < i1;
    return SplitKeys{now, false, valid && !now, key, key, key};
  };
  split_tile(spill_in, n, f, out, out_cnt, out_cap, spill_out, spill_cnt, spill_cap);
}

}  // namespace

void launch_mirror_split(const uint64_t *in, uint64_t n, uint32_t i1, uint64_t *out,
                         unsigned long long *out_cnt, uint64_t out_cap, uint64_t *spill,
                         unsigned long long *spill_cnt, uint64_t spill_cap, hipStream_t s) {
  if (!n) return;
  if ((n + kSplitTile - 1) / kSplitTile > 0x7fffffffull)
    fail(SJ_ERR_INVALID_ARG, "mirror split too large");
  hipLaunchKernelGGL(k_mirror_split, dim3((uint32_t)((n + kSplitTile - 1) / kSplitTile)),
                     dim3(kBlock), 0,
                     s, in, n, i1, out, out_cnt, out_cap, spill, spill_cnt, spill_cap);
  SJ_HIP(hipGetLastError());
}

void launch_spill_take(const uint64_t *spill_in, uint64_t n, uint32_t i1, uint64_t *out,
                       unsigned long long *out_cnt, uint64_t out_cap, uint64_t *spill_out,
                       unsigned long long *spill_cnt, uint64_t spill_cap, hipStream_t s) {
  if (!n) return;
  if ((n + kSplitTile - 1) / kSplitTile > 0x7fffffffull)
    fail(SJ_ERR_INVALID_ARG, "spill take too large");
  hipLaunchKernelGGL(k_spill_take, dim3((uint32_t)((n + kSplitTile - 1) / kSplitTile)),
                     dim3(kBlock), 0, s,
                     spill_in, n, i1, out, out_cnt, out_cap, spill_out, spill_cnt, spill_cap);
  SJ_HIP(hipGetLastError());
}

void launch_iota_strided(uint32_t *out, uint64_t count, uint64_t stride, uint32_t run,
                         hipStream_t s) {
  if (!count) return;
  if (run == 0 || (run > 1 && stride < run)) fail(SJ_ERR_INVALID_ARG, "iota runs overlap");
  hipLaunchKernelGGL(k_iota_strided, dim3((uint32_t)((count + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, out, count, stride, run);
  SJ_HIP(hipGetLastError());
}
void launch_widen(const uint32_t *in, uint64_t *out, uint64_t count, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_widen, dim3((uint32_t)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     in, out, count);
  SJ_HIP(hipGetLastError());
}
void launch_narrow(const uint64_t *in, uint32_t *out, uint64_t count, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_narrow, dim3((uint32_t)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     in, out, count);
  SJ_HIP(hipGetLastError());
}

size_t scan_tmp_bytes(uint64_t n) { return scan_levels_bytes<uint64_t>(n); }

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *d_total,
                        void *tmp, hipStream_t s) {
  scan_impl<uint32_t>(in, out, n, d_total, static_cast<char *>(tmp), s);
}

void exclusive_scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *d_total,
                        void *tmp, hipStream_t s) {
  scan_impl<uint64_t>(in, out, n, d_total, static_cast<char *>(tmp), s);
}

size_t radix_tmp_bytes(uint64_t n) {
  const uint64_t nb = (n + kRsTile - 1) / kRsTile;
  const uint64_t hist = (uint64_t)kRadixBins * (nb ? nb : 1);
  return ((hist * 8 + 255) / 256) * 256 + scan_levels_bytes<uint64_t>(hist);
}

void launch_fill_u64(unsigned long long *p, uint64_t count, unsigned long long v, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     p, count, v);
  SJ_HIP(hipGetLastError());
}

// One pass over the digit of BITS bits at shift sh: tiles of 16 rounds of
// 256 keys with values, kRsRoundsKeys rounds without.
template <int BITS>
void rs_pass(uint64_t *kin, uint32_t *vin, uint64_t *kout, uint32_t *vout, uint64_t n, int sh,
             uint64_t *hist, char *scan_tmp, hipStream_t s, const unsigned long long *d_count) {
  if (vin) {
    const uint32_t nb = (uint32_t)((n + kRsTile - 1) / kRsTile);
    hipLaunchKernelGGL((k_rs_hist<BITS, kRsRounds>), dim3(nb), dim3(kBlock), 0, s, kin, n, sh,
                       hist, nb, d_count);
    SJ_HIP(hipGetLastError());
    exclusive_scan_u64(hist, hist, (uint64_t)(1u << BITS) * nb, nullptr, scan_tmp, s);
    hipLaunchKernelGGL((k_rs_scatter<true, BITS, kRsRounds>), dim3(nb), dim3(kBlock), 0, s, kin,
                       vin, kout, vout, n, sh, hist, nb, d_count);
  } else {
    constexpr uint64_t kT = (uint64_t)kBlock * kRsRoundsKeys;
    const uint32_t nb = (uint32_t)((n + kT - 1) / kT);
    hipLaunchKernelGGL((k_rs_hist<BITS, kRsRoundsKeys>), dim3(nb), dim3(kBlock), 0, s, kin, n,
                       sh, hist, nb, d_count);
    SJ_HIP(hipGetLastError());
    exclusive_scan_u64(hist, hist, (uint64_t)(1u << BITS) * nb, nullptr, scan_tmp, s);
    hipLaunchKernelGGL((k_rs_scatter<false, BITS, kRsRoundsKeys>), dim3(nb), dim3(kBlock), 0, s,
                       kin, (const uint32_t *)nullptr, kout, (uint32_t *)nullptr, n, sh, hist,
                       nb, d_count);
  }
  SJ_HIP(hipGetLastError());
}

void radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], uint64_t n, const int *shifts,
                    int n_passes, void *tmp, hipStream_t s, const unsigned long long *d_count,
                    const int *widths) {
  if (n == 0 || (n == 1 && !d_count) || n_passes == 0) return;
  if ((n + kRsTile - 1) / kRsTile > 0x7fffffffull) fail(SJ_ERR_INVALID_ARG, "radix sort too large");
  const uint32_t nb = (uint32_t)((n + kRsTile - 1) / kRsTile);
  const uint64_t nhist = (uint64_t)kRadixBins * nb;
  uint64_t *hist = static_cast<uint64_t *>(tmp);
  char *scan_tmp = static_cast<char *>(tmp) + ((nhist * 8 + 255) / 256) * 256;
  int cur = 0;
  for (int p = 0; p < n_passes; ++p) {
    const int sh = shifts[p];
    const int w = widths ? widths[p] : kRadixBits;
    uint64_t *ki = keys[cur], *ko = keys[cur ^ 1];
    uint32_t *vi = vals ? vals[cur] : nullptr, *vo = vals ? vals[cur ^ 1] : nullptr;
    switch (w) {
      case 1: rs_pass<1>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 2: rs_pass<2>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 3: rs_pass<3>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 4: rs_pass<4>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 5: rs_pass<5>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 6: rs_pass<6>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 7: rs_pass<7>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      case 8: rs_pass<8>(ki, vi, ko, vo, n, sh, hist, scan_tmp, s, d_count); break;
      default: fail(SJ_ERR_INVALID_ARG, "radix digit width must be 1..8");
    }
    cur ^= 1;
  }
  if (cur == 1) {
    // odd number of passes: move the result into buffer 0
    if (d_count) {
      if (vals) fail(SJ_ERR_INVALID_ARG, "odd pass count with values and a device count");
      const uint32_t g = (uint32_t)std::min<uint64_t>((n + kBlock - 1) / kBlock, 65536);
      hipLaunchKernelGGL(k_copy_u64, dim3(g), dim3(kBlock), 0, s, keys[1], keys[0], n, d_count);
      SJ_HIP(hipGetLastError());
    } else {
      SJ_HIP(hipMemcpyAsync(keys[0], keys[1], n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
      if (vals)
        SJ_HIP(hipMemcpyAsync(vals[0], vals[1], n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
  }
}

}  // namespace sj
