// Host runtime and C ABI of libselfjoin (Algorithm 1, GPU-JOIN: reorder ->
// constructIndex -> computeNumBatches -> batch loop).  All device work runs
// on the caller's stream; results stay on the device when they fit the
// memory budget, else batches are streamed to pinned host memory.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include <unistd.h>

#include "sj_runtime.hpp"

namespace sj {

thread_local std::string g_last_error;

namespace {

constexpr int kCacheDevices = 64;

struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void *> blocks;  // capacity -> block
  size_t bytes = 0;                      // sum of the cached capacities
  size_t cap = 0;
  bool cap_known = false;
};

BlockCache g_cache[kCacheDevices];

// capacities are rounded so that nearby requests share blocks
size_t block_round(size_t b) {
  const size_t g = b < ((size_t)1 << 20) ? 4096 : ((size_t)2 << 20);
  return (b + g - 1) / g * g;
}

// cache limit of the current device, read once: SJ_CACHE_BYTES, else a
// quarter of the device's memory
size_t cache_cap(BlockCache &c) {
  if (!c.cap_known) {
    c.cap_known = true;
    const char *v = std::getenv("SJ_CACHE_BYTES");
    if (v && *v) {
      c.cap = (size_t)std::strtoull(v, nullptr, 10);
    } else {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        tot = 0;
      }
      c.cap = tot / 4;
    }
  }
  return c.cap;
}

void free_all_locked(BlockCache &c) {
  for (auto &kv : c.blocks) (void)hipFree(kv.second);
  c.blocks.clear();
  c.bytes = 0;
}

}  // namespace

void *dev_alloc(size_t bytes, size_t *got, int *dev) {
  int d = 0;
  SJ_HIP(hipGetDevice(&d));
  *dev = d;
  const size_t want = block_round(std::max<size_t>(bytes, 1));
  if (d >= 0 && d < kCacheDevices) {
    BlockCache &c = g_cache[d];
    std::lock_guard<std::mutex> lock(c.mu);
    // smallest cached block that holds the request and is at most about
    // twice its size
    auto it = c.blocks.lower_bound(want);
    if (it != c.blocks.end() && it->first <= std::max(2 * want, want + ((size_t)1 << 20))) {
      void *p = it->second;
      *got = it->first;
      c.bytes -= it->first;
      c.blocks.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess && d >= 0 && d < kCacheDevices) {
    (void)hipGetLastError();
    BlockCache &c = g_cache[d];
    {
      std::lock_guard<std::mutex> lock(c.mu);
      free_all_locked(c);
    }
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(SJ_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(want) + " bytes failed");
  }
  *got = want;
  return p;
}

void dev_free(void *p, size_t got, int dev, bool idle) {
  if (!p) return;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) {
    (void)hipGetLastError();
    cur = -1;
  }
  if (dev != cur || dev < 0 || dev >= kCacheDevices) {
    (void)hipFree(p);
    return;
  }
  BlockCache &c = g_cache[dev];
  auto fits = [&]() { return got <= cache_cap(c) - std::min(c.bytes, cache_cap(c)); };
  bool keep;
  {
    std::lock_guard<std::mutex> lock(c.mu);
    keep = fits();
  }
  // the block may still be read or written by queued work on any stream;
  // the next user may run on another stream.  The wait is not taken under
  // the cache's lock, so that other threads allocate meanwhile.
  if (keep && !idle && hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    keep = false;
  }
  if (keep) {
    std::lock_guard<std::mutex> lock(c.mu);
    if (fits()) {  // checked again: other blocks may have come in meanwhile
      c.blocks.emplace(got, p);
      c.bytes += got;
      return;
    }
  }
  (void)hipFree(p);
}

size_t dev_cached_bytes(int dev) {
  if (dev < 0 || dev >= kCacheDevices) return 0;
  std::lock_guard<std::mutex> lock(g_cache[dev].mu);
  return g_cache[dev].bytes;
}

void dev_cache_release(int dev) {
  if (dev < 0 || dev >= kCacheDevices) return;
  std::lock_guard<std::mutex> lock(g_cache[dev].mu);
  free_all_locked(g_cache[dev]);
}

namespace {

struct HostCache {
  std::mutex mu;
  std::multimap<size_t, void *> blocks;
  size_t bytes = 0;
  size_t cap = 0;
  bool cap_known = false;
};

HostCache g_host_cache;

size_t host_cap(HostCache &c) {
  if (!c.cap_known) {
    c.cap_known = true;
    const char *v = std::getenv("SJ_HOST_CACHE_BYTES");
    if (v && *v) {
      c.cap = (size_t)std::strtoull(v, nullptr, 10);
    } else {
      const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGE_SIZE);
      const size_t ram = pages > 0 && page > 0 ? (size_t)pages * (size_t)page : 0;
      c.cap = std::min<size_t>(ram / 8, (size_t)64 << 30);
    }
  }
  return c.cap;
}

}  // namespace

void *host_alloc(size_t bytes, size_t *got) {
  const size_t want = block_round(std::max<size_t>(bytes, 1));
  {
    std::lock_guard<std::mutex> lock(g_host_cache.mu);
    auto it = g_host_cache.blocks.lower_bound(want);
    if (it != g_host_cache.blocks.end() &&
        it->first <= std::max(2 * want, want + ((size_t)1 << 20))) {
      void *p = it->second;
      *got = it->first;
      g_host_cache.bytes -= it->first;
      g_host_cache.blocks.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    host_cache_release();
    e = hipHostMalloc(&p, want, hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(SJ_ERR_OUT_OF_MEMORY, "pinned host allocation of " + std::to_string(want) + " bytes failed");
  }
  *got = want;
  return p;
}

void host_free(void *p, size_t got) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_host_cache.mu);
  const size_t cap = host_cap(g_host_cache);
  if (got > cap - std::min(g_host_cache.bytes, cap)) {
    (void)hipHostFree(p);
    return;
  }
  g_host_cache.blocks.emplace(got, p);
  g_host_cache.bytes += got;
}

size_t host_cached_bytes() {
  std::lock_guard<std::mutex> lock(g_host_cache.mu);
  return g_host_cache.bytes;
}

void host_cache_release() {
  std::lock_guard<std::mutex> lock(g_host_cache.mu);
  for (auto &kv : g_host_cache.blocks) (void)hipHostFree(kv.second);
  g_host_cache.blocks.clear();
  g_host_cache.bytes = 0;
}

Scratch &thread_scratch() {
  thread_local Scratch s;
  return s;
}

void *Scratch::take(size_t bytes) {
  if (depth <= 0) fail(SJ_ERR_DEVICE, "internal: scratch taken outside a scope");
  const size_t b = std::max<size_t>(256, (bytes + 255) & ~(size_t)255);
  while (cur_ < chunks_.size()) {
    if (used_ + b <= chunks_[cur_].size) {
      void *p = static_cast<char *>(chunks_[cur_].p) + used_;
      used_ += b;
      return p;
    }
    ++cur_;
    used_ = 0;
  }
  size_t size = std::max<size_t>(b, (size_t)8 << 20);
  int dev = 0;
  void *p = dev_alloc(size, &size, &dev);
  chunks_.push_back({p, size, dev});
  cur_ = chunks_.size() - 1;
  used_ = b;
  return p;
}

void Scratch::release(bool error) {
  cur_ = 0;
  used_ = 0;
  size_t total = 0;
  for (const Chunk &c : chunks_) total += c.size;
  // after an error, work that used the temporaries may still be queued:
  // free everything and wait for the device; otherwise the scope's code has
  // synchronised every stream that used them
  const size_t keep = error ? 0 : keep_bytes;
  while (!chunks_.empty() && total > keep) {
    dev_free(chunks_.back().p, chunks_.back().size, chunks_.back().dev, !error);
    total -= chunks_.back().size;
    chunks_.pop_back();
  }
}

void Scratch::trim() {
  if (depth > 0) return;
  const size_t k = keep_bytes;
  keep_bytes = 0;
  release(false);
  keep_bytes = k;
}

// Kept chunks are freed by trim(); those still held when the thread ends
// belong to the process until it exits (the HIP runtime may already be gone
// when thread-local destructors run).
Scratch::~Scratch() = default;

ScratchScope::~ScratchScope() {
  Scratch &s = thread_scratch();
  if (--s.depth == 0) s.release(std::uncaught_exceptions() > uncaught);
}

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
                       ? SJ_ERR_OUT_OF_MEMORY
                       : SJ_ERR_DEVICE;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace sj

using namespace sj;


namespace sj {

constexpr double kWidthSlack = 1.0 + 1.0 / (1 << 20);  // cell side = eps * (1 + 2^-20)
#ifndef SJ_WU_BY_STRETCH
#define SJ_WU_BY_STRETCH 1
#endif
constexpr bool kWuByStretch = SJ_WU_BY_STRETCH != 0;  // join work units in stretch order

// Fine (Morton) ordering inside cells: dimensions and bits per dimension.
#ifndef SJ_FINE_DIMS
#define SJ_FINE_DIMS 8
#endif
#ifndef SJ_FINE_BITS
#define SJ_FINE_BITS 3
#endif

// Cost model for the automatic choice of k (Section 5.5 compares the memory
// operations of index searches with those of distance calculations): one
// unit per 3^k-offset lookup of each non-empty cell, one per evaluated pair.
#ifndef SJ_FP32_CELL_GROUPS
#define SJ_FP32_CELL_GROUPS 1
#endif

constexpr bool kFp32CellGroups = SJ_FP32_CELL_GROUPS != 0;
constexpr double kLookupsPerSec = 2.0e10;
constexpr double kPairsPerSec = 1.5e12;

bool make_geometry(const sj_index &ix, uint32_t k, Geometry &g) {
  g = Geometry{};
  g.k = k;
  g.kp.k = k;
  g.kp.w = ix.eps * kWidthSlack;
  g.np.k = k;
  unsigned __int128 prod = 1;
  uint64_t m[kKeyMaxDims];
  for (uint32_t r = 0; r < k; ++r) {
    const uint32_t t = ix.perm[r];
    g.kp.dim[r] = t;
    g.kp.org[r] = ix.dmin[t];
    // same arithmetic as the device: floor((x - org) / w) at x = max
    const double cm = std::floor((ix.dmax[t] - ix.dmin[t]) / g.kp.w);
    if (!(cm >= 0.0) || cm > 9.0e15) return false;
    g.kp.cmax[r] = (uint64_t)cm;
    m[r] = (uint64_t)cm + 1;
    prod *= m[r];
    if (prod > ((unsigned __int128)1 << 63)) return false;
  }
  uint64_t mult = 1;
  for (int r = (int)k - 1; r >= 0; --r) {
    g.kp.mult[r] = mult;
    g.np.mult[r] = mult;
    g.np.m[r] = m[r];
    mult *= m[r];
  }
  const uint32_t cell_bits = bits_for(mult - 1);
  // fine key: Morton code of up to SJ_FINE_DIMS reordered dimensions,
  // SJ_FINE_BITS bits each, as far as the 64-bit sort key allows; with
  // SORTIDU the quantised coordinate u of one un-indexed dimension instead
  // (the first one after the k indexed; reordered dimension 0 when k = d),
  // up to 24 bits, so every cell is sorted by u (Section 4.3)
  uint32_t fm = std::min<uint32_t>(ix.d, SJ_FINE_DIMS);
  uint32_t fb = SJ_FINE_BITS;
  uint32_t u_rank = 0;
  if (ix.opt.sortidu) {
    u_rank = k < ix.d ? k : 0;
    fm = 1;
    fb = std::min<uint32_t>(24, 63 - std::min<uint32_t>(cell_bits, 63));
  }
  while (fb > 0 && cell_bits + fm * fb > 63) --fb;
  g.kp.fm = fb ? fm : 0;
  g.kp.fb = fb;
  for (uint32_t r = 0; r < g.kp.fm; ++r) {
    const uint32_t t = ix.perm[ix.opt.sortidu ? u_rank : r];
    g.kp.fdim[r] = t;
    g.kp.forg[r] = ix.dmin[t];
    const double span = ix.dmax[t] - ix.dmin[t];
    g.kp.fscale[r] = span > 0.0 ? (double)(1u << fb) / span : 0.0;
  }
  g.fine_bits = g.kp.fm * g.kp.fb;
  g.key_bits = cell_bits + g.fine_bits;
  g.u_rank = u_rank;
  uint64_t noff = 1;
  for (uint32_t r = 0; r < k; ++r) noff *= 3;
  g.np.n_off = noff;
  return true;
}

// Temporary buffers of one build.
struct BuildTmp {  // temporaries of the grid builds (thread scratch)
  TmpBuf keys[2], ids[2], flag, radix, scan, small;
  TmpBuf nbr_count, cand_sum, prod;
};

uint64_t build_neighbors(sj_index &ix, const sj_index &E, NbrParams np, BuildTmp &t,
                         hipStream_t s, bool keep);

// Keys, sort, gather, compaction and neighbour counts for geometry g.
// Returns the candidate count C and fills ncell.
uint64_t build_grid(sj_index &ix, const float *P, const Geometry &g, BuildTmp &t, hipStream_t s,
                    bool keep) {
  const uint64_t n = ix.n;
  launch_cellkey(P, n, ix.d, g.kp, t.keys[0].as<uint64_t>(), t.ids[0].as<uint32_t>(), s);
  uint64_t *kb[2] = {t.keys[0].as<uint64_t>(), t.keys[1].as<uint64_t>()};
  uint32_t *vb[2] = {t.ids[0].as<uint32_t>(), t.ids[1].as<uint32_t>()};
  // a probe of k only counts candidates: the cell part of the keys, without
  // the point ids, is all it sorts
  std::vector<int> shifts;
  for (uint32_t b = keep ? 0u : g.fine_bits; b < g.key_bits; b += 8) shifts.push_back((int)b);
  radix_sort_u64(kb, keep ? vb : nullptr, n, shifts.data(), (int)shifts.size(), t.radix.p, s);
  if (keep) {
    launch_gather(P, n, ix.d, ix.dp, ix.perm_d.as<uint32_t>(), vb[0], ix.X.as<float>(),
                  ix.orig_id.as<uint32_t>(), ix.pos_of.as<uint32_t>(), s);
    if (ix.opt.sortidu) {  // the sorted keys: SORTIDU searches their u part
      ix.skey.alloc(n * 8);
      SJ_HIP(hipMemcpyAsync(ix.skey.p, kb[0], n * 8, hipMemcpyDeviceToDevice, s));
    }
  }
  uint32_t *d_ncell = t.small.as<uint32_t>();
  launch_compact(kb[0], n, g.fine_bits, t.flag.as<uint32_t>(), d_ncell,
                 ix.cell_key.as<uint64_t>(), ix.cell_start.as<uint32_t>(), t.scan.p, s);
  uint32_t h_ncell = 0;
  SJ_HIP(hipMemcpyAsync(&h_ncell, d_ncell, 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  ix.ncell = h_ncell;
  return build_neighbors(ix, ix, g.np, t, s, keep);
}

// Adjacent non-empty cells of ix's cells in E's cell table (E = ix in a
// self-join; np of E's grid).  Returns the candidate count C, the sum over
// ix's points of the sizes of their adjacent cells of E; with keep, fills
// ix.nbr_off / ix.nbr_cell.
uint64_t build_neighbors(sj_index &ix, const sj_index &E, NbrParams np, BuildTmp &t,
                         hipStream_t s, bool keep) {
  const uint64_t nc = ix.ncell;
  const uint64_t ne = E.ncell;
  const uint64_t kFence = 8192;
  uint64_t fs = 1;
  while ((ne + fs - 1) / fs > kFence) fs <<= 1;
  np.fstride = (uint32_t)fs;
  np.nfence = (uint32_t)((ne + fs - 1) / fs);
  SJ_HIP(hipMemsetAsync(t.nbr_count.p, 0, (nc + 1) * 4, s));
  SJ_HIP(hipMemsetAsync(t.cand_sum.p, 0, (nc + 1) * 8, s));
  launch_neighbors(0, ix.cell_key.as<uint64_t>(), nc, E.cell_key.as<uint64_t>(),
                   E.cell_start.as<uint32_t>(), ne, np, t.nbr_count.as<uint32_t>(),
                   t.cand_sum.as<uint64_t>(), nullptr, nullptr, s);
  launch_cell_products(nc, ix.cell_start.as<uint32_t>(), t.cand_sum.as<uint64_t>(),
                       t.prod.as<uint64_t>(), s);
  uint64_t *d_c = reinterpret_cast<uint64_t *>(t.small.as<char>() + 8);
  exclusive_scan_u64(t.prod.as<uint64_t>(), t.prod.as<uint64_t>(), nc, d_c, t.scan.p, s);
  uint64_t h_c = 0;
  SJ_HIP(hipMemcpyAsync(&h_c, d_c, 8, hipMemcpyDeviceToHost, s));
  if (keep) {
    // the adjacency lists use 32-bit offsets: their total, summed in 64 bits
    // (the C scan above no longer needs t.prod), must stay below 2^32
    launch_widen(t.nbr_count.as<uint32_t>(), t.prod.as<uint64_t>(), nc + 1, s);
    uint64_t *d_nn64 = reinterpret_cast<uint64_t *>(t.small.as<char>() + 24);
    exclusive_scan_u64(t.prod.as<uint64_t>(), t.prod.as<uint64_t>(), nc + 1, d_nn64, t.scan.p, s);
    uint64_t h_nn64 = 0;
    SJ_HIP(hipMemcpyAsync(&h_nn64, d_nn64, 8, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    if (h_nn64 > 0xffffffffull)
      fail(SJ_ERR_KEY_OVERFLOW, "the adjacency lists over k=" + std::to_string(ix.geom.k) +
                                    " dimensions hold " + std::to_string(h_nn64) +
                                    " cells, more than 2^32 - 1; use a smaller k");
    ix.nbr_off.alloc((nc + 1) * 4);
    uint32_t *d_nn = reinterpret_cast<uint32_t *>(t.small.as<char>() + 16);
    exclusive_scan_u32(t.nbr_count.as<uint32_t>(), ix.nbr_off.as<uint32_t>(), nc + 1, d_nn,
                       t.scan.p, s);
    uint32_t h_nn = 0;
    SJ_HIP(hipMemcpyAsync(&h_nn, d_nn, 4, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    ix.n_nbr = h_nn;
    ix.nbr_cell.alloc((uint64_t)h_nn * 4);
    launch_neighbors(1, ix.cell_key.as<uint64_t>(), nc, E.cell_key.as<uint64_t>(),
                     E.cell_start.as<uint32_t>(), ne, np, nullptr, nullptr,
                     ix.nbr_off.as<uint32_t>(), ix.nbr_cell.as<uint32_t>(), s);
  }
  SJ_HIP(hipStreamSynchronize(s));
  return h_c;
}

// Share of the lane work of the FP32 units of tq queries that falls on
// live query slots: candidates C over the sum, over the query cells, of the
// cell's slots (its query count rounded up to tq) times its candidates
// (cand_sum, per cell, from build_neighbors).  Low when much of the work is
// in cells holding far fewer queries than a unit has slots.
double live_slot_share(const sj_index &ix, const uint64_t *cand_sum, uint32_t tq, hipStream_t s) {
  const uint64_t nc = ix.ncell;
  if (!nc || !ix.candidates) return 1.0;
  ScratchScope scope;  // the read-back below synchronises the stream
  TmpBuf w, tot, scan;
  w.alloc(nc * 8);
  tot.alloc(64);
  scan.alloc(scan_tmp_bytes(nc) + 64);
  launch_cell_slot_work(nc, ix.cell_start.as<uint32_t>(), cand_sum, tq, w.as<uint64_t>(), s);
  exclusive_scan_u64(w.as<uint64_t>(), w.as<uint64_t>(), nc, tot.as<uint64_t>(), scan.p, s);
  uint64_t h = 0;
  SJ_HIP(hipMemcpyAsync(&h, tot.p, 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  return h ? (double)ix.candidates / (double)h : 1.0;
}
constexpr double kLiveSlotShareMin = 0.75;  // below it, units of one query per lane

// Candidate runs (sym: only cells B >= A) into off/runs.
uint64_t build_runs(sj_index &ix, int sym, DevBuf &off, DevBuf &runs, BuildTmp &t, hipStream_t s) {
  const uint64_t nc = ix.ncell;
  ScratchScope scope;
  TmpBuf cnt;
  cnt.alloc((nc + 1) * 4);
  SJ_HIP(hipMemsetAsync(cnt.p, 0, (nc + 1) * 4, s));
  const uint32_t *ecs = entries_of(ix).cell_start.as<uint32_t>();  // candidate cells
  launch_runs(0, sym, nc, ecs, ix.nbr_off.as<uint32_t>(), ix.nbr_cell.as<uint32_t>(),
              cnt.as<uint32_t>(), nullptr, nullptr, s);
  off.alloc((nc + 1) * 4);
  uint32_t *d_tot = t.small.as<uint32_t>() + 8;
  exclusive_scan_u32(cnt.as<uint32_t>(), off.as<uint32_t>(), nc + 1, d_tot, t.scan.p, s);
  uint32_t h_tot = 0;
  SJ_HIP(hipMemcpyAsync(&h_tot, d_tot, 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  runs.alloc((uint64_t)h_tot * sizeof(uint2));
  launch_runs(1, sym, nc, ecs, ix.nbr_off.as<uint32_t>(), ix.nbr_cell.as<uint32_t>(), nullptr,
              off.as<uint32_t>(), runs.as<uint2>(), s);
  return h_tot;
}

void build_cell_groups(sj_index &ix, uint32_t max_q, CellGroups &g, hipStream_t s) {
  const uint64_t nc = ix.ncell;
  std::vector<uint64_t> key(nc);
  std::vector<uint32_t> start(nc + 1);
  SJ_HIP(hipMemcpyAsync(key.data(), ix.cell_key.p, nc * 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipMemcpyAsync(start.data(), ix.cell_start.p, (nc + 1) * 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  // the last indexed dimension has stride 1 in the cell key: cells of one
  // row share key / m_last, and key + 1 is the next cell along it
  const uint64_t m_last = ix.geom.k ? std::max<uint64_t>(1, ix.geom.np.m[ix.geom.k - 1]) : 1;
  std::vector<uint32_t> first, gstart;
  first.reserve(nc + 1);
  gstart.reserve(nc + 1);
  for (uint64_t a = 0; a < nc;) {
    first.push_back((uint32_t)a);
    gstart.push_back(start[a]);
    uint64_t b = a + 1;
    while (b < nc && b - a < kGroupMaxCells && key[b] / m_last == key[a] / m_last &&
           key[b] - key[a] <= 2 && start[b + 1] - start[a] <= max_q)
      ++b;
    a = b;
  }
  first.push_back((uint32_t)nc);
  gstart.push_back(start[nc]);
  const uint64_t ng = first.size() - 1;
  ScratchScope scope;  // the read-back below synchronises the stream
  TmpBuf gfirst, cnt, tot, scan;
  gfirst.alloc((ng + 1) * 4);
  SJ_HIP(hipMemcpyAsync(gfirst.p, first.data(), (ng + 1) * 4, hipMemcpyHostToDevice, s));
  g.n = ng;
  g.start.alloc((ng + 1) * 4);
  SJ_HIP(hipMemcpyAsync(g.start.p, gstart.data(), (ng + 1) * 4, hipMemcpyHostToDevice, s));
  cnt.alloc((ng + 1) * 4);
  SJ_HIP(hipMemsetAsync(cnt.p, 0, (ng + 1) * 4, s));
  launch_group_runs(0, ng, gfirst.as<uint32_t>(), ix.run_off_sym.as<uint32_t>(),
                    ix.runs_sym.as<uint2>(), cnt.as<uint32_t>(), nullptr, nullptr, s);
  g.run_off.alloc((ng + 1) * 4);
  tot.alloc(64);
  scan.alloc(scan_tmp_bytes(ng + 1) + 64);
  exclusive_scan_u32(cnt.as<uint32_t>(), g.run_off.as<uint32_t>(), ng + 1, tot.as<uint32_t>(),
                     scan.p, s);
  uint32_t h_tot = 0;
  SJ_HIP(hipMemcpyAsync(&h_tot, tot.p, 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  g.runs.alloc(std::max<uint64_t>(h_tot, 1) * sizeof(uint2));
  launch_group_runs(1, ng, gfirst.as<uint32_t>(), ix.run_off_sym.as<uint32_t>(),
                    ix.runs_sym.as<uint2>(), nullptr, g.run_off.as<uint32_t>(),
                    g.runs.as<uint2>(), s);
  SJ_HIP(hipStreamSynchronize(s));
}

// Work units over the given runs; qlist == nullptr: contiguous queries.
// Returns the number of units; *eval receives the evaluated pair count.
// With by_stretch, the units are ordered by their stretch index within
// their query block, then by block: units that run at the same time then
// read overlapping candidate rows (shared in the caches) instead of every
// stretch of one block.
// SORTIDU search parameters of a handle (its sort keys' u part).
USearch usearch_of(const sj_index &ix) {
  const Geometry &g = ix.geom;
  USearch us{};
  us.ur = g.u_rank;
  us.dp = ix.dp;
  us.fmask = g.fine_bits ? ((1ull << g.fine_bits) - 1ull) : 0ull;
  us.org = g.kp.fm ? g.kp.forg[0] : 0.0;
  us.scale = g.kp.fm ? g.kp.fscale[0] : 0.0;
  us.fmax = g.kp.fb ? (1u << g.kp.fb) - 1u : 0u;
  us.eps = ix.eps;
  return us;
}

// With u_ranges (SORTIDU; contiguous queries only), every query block gets
// its own candidate ranges (launch_qb_ranges, into *u_ranges) and the units
// are cut from those instead of from the cells' runs.
uint64_t build_workunits(sj_index &ix, int sym, const uint32_t *qlist, uint64_t nq,
                         const DevBuf &run_off, const DevBuf &runs, uint32_t tq, uint32_t tc,
                         DevBuf &out, uint64_t *eval, hipStream_t s, bool by_stretch,
                         DevBuf *u_ranges, const CellGroups *groups) {
  // query blocks are cut from the cells, or from groups of consecutive cells
  const uint64_t nc = groups ? groups->n : ix.ncell;
  const uint32_t *cstart = groups ? groups->start.as<uint32_t>() : ix.cell_start.as<uint32_t>();
  ScratchScope scope;  // every temporary below is dead at the final synchronisation
  TmpBuf qb_off, run_total, scan, tot;
  qb_off.alloc((nc + 1) * 4);
  run_total.alloc(nc * 8);
  tot.alloc(64);
  SJ_HIP(hipMemsetAsync(qb_off.p, 0, (nc + 1) * 4, s));
  launch_wu_cells(nc, tq, cstart, qlist, nq, run_off.as<uint32_t>(),
                  runs.as<uint2>(), qb_off.as<uint32_t>(), run_total.as<uint64_t>(), s);
  scan.alloc(scan_tmp_bytes(std::max<uint64_t>(nc + 1, 1)) + 64);
  exclusive_scan_u32(qb_off.as<uint32_t>(), qb_off.as<uint32_t>(), nc + 1, tot.as<uint32_t>(),
                     scan.p, s);
  uint32_t h_nqb = 0;
  SJ_HIP(hipMemcpyAsync(&h_nqb, tot.p, 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  const uint64_t nqb = h_nqb;
  // the runs the units are cut from: the cells' (indexed by cell), or with
  // SORTIDU each block's own ranges (indexed by block)
  const uint32_t *r_off = run_off.as<uint32_t>();
  const uint2 *r_runs = runs.as<uint2>();
  const uint64_t *r_total = run_total.as<uint64_t>();
  int per_block = 0;
  TmpBuf rcount, rlen;
  if (u_ranges && !qlist && nqb) {
    const sj_index &E = entries_of(ix);
    const USearch us = usearch_of(E);
    rcount.alloc((nqb + 1) * 4);
    rlen.alloc(nqb * 8);
    SJ_HIP(hipMemsetAsync(rcount.p, 0, (nqb + 1) * 4, s));
    launch_qb_ranges(0, sym, nqb, nc, tq, ix.cell_start.as<uint32_t>(), qb_off.as<uint32_t>(),
                     ix.nbr_off.as<uint32_t>(), ix.nbr_cell.as<uint32_t>(),
                     E.cell_start.as<uint32_t>(), E.skey.as<uint64_t>(), ix.X.as<float>(), us,
                     rcount.as<uint32_t>(), rlen.as<uint64_t>(), nullptr, nullptr, s);
    scan.alloc(scan_tmp_bytes(nqb + 1) + 64);
    exclusive_scan_u32(rcount.as<uint32_t>(), rcount.as<uint32_t>(), nqb + 1, tot.as<uint32_t>(),
                       scan.p, s);
    uint32_t h_nr = 0;
    SJ_HIP(hipMemcpyAsync(&h_nr, tot.p, 4, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    u_ranges->alloc(std::max<uint64_t>(h_nr, 1) * sizeof(uint2));
    launch_qb_ranges(1, sym, nqb, nc, tq, ix.cell_start.as<uint32_t>(), qb_off.as<uint32_t>(),
                     ix.nbr_off.as<uint32_t>(), ix.nbr_cell.as<uint32_t>(),
                     E.cell_start.as<uint32_t>(), E.skey.as<uint64_t>(), ix.X.as<float>(), us,
                     nullptr, nullptr, rcount.as<uint32_t>(), u_ranges->as<uint2>(), s);
    r_off = rcount.as<uint32_t>();
    r_runs = u_ranges->as<uint2>();
    r_total = rlen.as<uint64_t>();
    per_block = 1;
  }
  TmpBuf units, ev;
  units.alloc((nqb + 1) * 4);
  ev.alloc((nqb + 1) * 8);
  SJ_HIP(hipMemsetAsync(units.p, 0, (nqb + 1) * 4, s));
  SJ_HIP(hipMemsetAsync(ev.p, 0, (nqb + 1) * 8, s));
  launch_wu_count(nqb, sym, nc, tq, tc, cstart, qlist, nq,
                  qb_off.as<uint32_t>(), r_off, r_runs, r_total, units.as<uint32_t>(),
                  ev.as<uint64_t>(), s, per_block);
  scan.alloc(scan_tmp_bytes(nqb + 1) + 64);
  exclusive_scan_u32(units.as<uint32_t>(), units.as<uint32_t>(), nqb + 1, tot.as<uint32_t>(),
                     scan.p, s);
  exclusive_scan_u64(ev.as<uint64_t>(), ev.as<uint64_t>(), nqb + 1, tot.as<uint64_t>() + 1,
                     scan.p, s);
  uint64_t h[2] = {0, 0};
  SJ_HIP(hipMemcpyAsync(h, tot.p, 16, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  const uint64_t n_wu = (uint32_t)h[0];
  *eval = h[1];
  out.ensure(n_wu * sizeof(WorkUnit));  // kept when it fits: no wait for the device
  if (by_stretch && n_wu > 1) {
    TmpBuf unordered, keys[2], rtmp;
    unordered.alloc(n_wu * sizeof(WorkUnit));
    keys[0].alloc(n_wu * 8);
    keys[1].alloc(n_wu * 8);
    launch_wu_fill(nqb, sym, nc, tq, tc, cstart, qlist, nq,
                   qb_off.as<uint32_t>(), r_off, r_runs, r_total, units.as<uint32_t>(),
                   unordered.as<WorkUnit>(), keys[0].as<uint64_t>(), s, per_block);
    // stable LSD sort on the stretch index (high word) keeps block order
    std::vector<int> sh;
    for (uint32_t b = 0; b < bits_for(n_wu - 1); b += 8) sh.push_back(32 + (int)b);
    rtmp.alloc(radix_tmp_bytes(n_wu));
    uint64_t *kb[2] = {keys[0].as<uint64_t>(), keys[1].as<uint64_t>()};
    radix_sort_u64(kb, nullptr, n_wu, sh.data(), (int)sh.size(), rtmp.p, s);
    launch_gather_wu(unordered.as<WorkUnit>(), kb[0], n_wu, out.as<WorkUnit>(), s);
  } else {
    launch_wu_fill(nqb, sym, nc, tq, tc, cstart, qlist, nq,
                   qb_off.as<uint32_t>(), r_off, r_runs, r_total, units.as<uint32_t>(),
                   out.as<WorkUnit>(), nullptr, s, per_block);
  }
  SJ_HIP(hipStreamSynchronize(s));
  return n_wu;
}

// Candidate block length so a launch has enough work units to fill the chip.
uint32_t choose_tc(uint64_t eval_pairs, uint32_t tq) {
  const double target_units = 256.0 * 32.0;  // CUs x waves in flight, roughly
  double tc = (double)eval_pairs / ((double)tq * target_units);
  tc = std::max(256.0, std::min(16384.0, tc));
  uint32_t t = 256;
  while (t < tc) t <<= 1;
  return t;
}

void compute_thresholds(sj_index &ix) {
  const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
  const double g32 = gamma_n((double)ix.dp + 2.0, u32);
  const double g64 = gamma_n((double)ix.d + 2.0, u64);
  const double tiny = 2.0 * ((double)ix.dp + 2.0) * std::ldexp(1.0, -126);
  const double margin = std::ldexp(1.0, -50);
  double hi = ix.eps2 * (1.0 + g32) / (1.0 - g64) * (1.0 + margin) + tiny;
  double lo = ix.eps2 * (1.0 - g32) / (1.0 + g64) * (1.0 - margin) - tiny;
  if (!(hi < (double)FLT_MAX / 4.0)) {
    ix.hi32 = __builtin_inff();
    ix.lo32 = -1.0f;
    return;
  }
  float h = (float)hi;
  if ((double)h < hi) h = std::nextafter(h, __builtin_inff());
  float l = (float)lo;
  if ((double)l > lo) l = std::nextafter(l, -__builtin_inff());
  if (lo <= 0.0) l = -1.0f;
  ix.hi32 = h;
  ix.lo32 = l;
}

// Operands and thresholds of the matrix-core filter (see sj_mfma.hip).
void mfma_prepare(sj_index &ix, hipStream_t s) {
  const uint32_t d = ix.d;
  // centre: the per-dimension sample mean (reordered order, like the rows
  // of X), clamped into the range.  Any centre gives a valid band; the
  // band's width grows with the distances of the points from the centre
  // (typical ones for the query, the largest for the candidates), so on
  // skewed data the mean beats the midrange
  std::vector<float> centre(d);
  double max_abs = 0.0, n_bound = 0.0;
  for (uint32_t r = 0; r < d; ++r) {
    const uint32_t t = ix.perm[r];
    centre[r] = (float)std::min(std::max(ix.dmean[t], ix.dmin[t]), ix.dmax[t]);
    const double h = std::max(std::fabs(ix.dmax[t] - (double)centre[r]),
                              std::fabs(ix.dmin[t] - (double)centre[r]));
    max_abs = std::max(max_abs, h);
    n_bound += h * h;
  }
  int fmt = ix.opt.precision == SJ_PREC_FP16 ? kFmtF16 : kFmtBF16;
  if (fmt == kFmtF16 && max_abs > 8192.0) fmt = kFmtBF16;  // -2 x~ must fit FP16
  if (fmt == kFmtBF16 && (max_abs > 1e15 || n_bound > 1e30))
    fail(SJ_ERR_INVALID_ARG, "coordinates too large for the 16-bit matrix path; use SJ_PREC_FP32");
  ix.fmt = fmt;
  ix.prec = fmt == kFmtF16 ? SJ_PREC_FP16 : SJ_PREC_BF16;
  ix.kp = mfma_kp(d);
  ix.n_pad = (ix.n + 31) / 32 * 32 + 64;  // chunks of 64 rows read past a run's end
  const uint64_t np = ix.n_pad;
  ix.XA.alloc(np * ix.kp * 2);
  ix.XB.alloc(np * ix.kp * 2);
  ix.cn.alloc(np * 4);
  ix.thi.alloc(np * 4);
  ix.tlo.alloc(np * 4);
  ScratchScope scope;  // ends after the final synchronisation below
  TmpBuf cdev, norm2, distc, fold;
  cdev.alloc(d * 4);
  norm2.alloc(np * 8);
  distc.alloc(np * 8);
  fold.alloc(np * 8);
  ix.mfma_max.alloc(64);  // kept: the thresholds of query handles use them
  DevBuf &maxima = ix.mfma_max;
  SJ_HIP(hipMemcpyAsync(cdev.p, centre.data(), d * 4, hipMemcpyHostToDevice, s));
  launch_mfma_prep(fmt, ix.X.as<float>(), ix.n, np, d, ix.dp, ix.kp, cdev.as<float>(), ix.XA.p,
                   ix.XB.p, ix.cn.as<float>(), norm2.as<double>(), distc.as<double>(),
                   fold.as<double>(), maxima.as<unsigned long long>(), s);
  MfmaBand band;
  const double u16 = fmt == kFmtF16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
  band.u = (1.0 + std::ldexp(1.0, -24)) * (1.0 + u16) - 1.0;
  band.u *= 1.0 + std::ldexp(1.0, -40);
  const double tiny = fmt == kFmtF16 ? std::ldexp(1.0, -14) : std::ldexp(1.0, -126);
  band.eta_term = 2.0 * tiny * 1.0001 * std::sqrt((double)d);
  band.gamma_acc = gamma_n((double)ix.kp + 1.0, std::ldexp(1.0, -23));
  const double g64 = gamma_n((double)d + 2.0, std::ldexp(1.0, -53));
  band.s_hi = ix.eps2 / (1.0 - g64);
  band.s_lo = ix.eps2 / (1.0 + g64);
  launch_mfma_thresholds(ix.n, np, band, norm2.as<double>(), distc.as<double>(),
                         maxima.as<unsigned long long>(), ix.thi.as<float>(), ix.tlo.as<float>(), s);
  ix.mfma_centre = centre;
  ix.mfma_band = band;
  SJ_HIP(hipStreamSynchronize(s));
}

// Form of the FP32 filter: the norm form when asked for, or (automatic) up
// to 16 padded dimensions when its error margin for a pair of mean squared
// norm stays below a small fraction of eps^2 (a wider band only sends more
// pairs to the FP64 recheck; either form gives the same result).  Above 16
// dimensions its extra checkpoint work made it slower than the difference
// form in every measured case.
constexpr double kNormBandMax = 0.005;
constexpr uint32_t kNormAutoMaxDp = 16;

// Bounds and margin factor of the norm-form tables (see k_norm_tables).
struct NormParams {
  double s_hi, s_lo, kappa;
};
NormParams norm_params(const sj_index &ix) {
  const double g64 = gamma_n((double)ix.d + 2.0, std::ldexp(1.0, -53));
  const double margin = std::ldexp(1.0, -50);
  NormParams p;
  p.s_hi = ix.eps2 / (1.0 - g64) * (1.0 + margin);
  p.s_lo = ix.eps2 / (1.0 + g64) * (1.0 - margin);
  p.kappa = 4.0 * gamma_n((double)ix.dp + 16.0, std::ldexp(1.0, -24));
  return p;
}

void choose_fp32_form(sj_index &ix, hipStream_t s) {
  ix.norm_form = false;
  ix.info.fp32_form = SJ_FP32_DIFFERENCE;
  if (ix.opt.fp32_form == SJ_FP32_DIFFERENCE || ix.n == 0) return;
  if (ix.opt.fp32_form == SJ_FP32_AUTO && ix.dp > kNormAutoMaxDp) return;
  const NormParams np = norm_params(ix);
  const double s_hi = np.s_hi, s_lo = np.s_lo, kappa = np.kappa;
  if (!(s_hi < 1e30)) return;  // keep the difference form for huge thresholds
  const uint64_t row = (uint64_t)norm_table_row(ix.dp);
  ix.norm_qa.alloc(ix.n * row * 4);
  ix.norm_cr.alloc((ix.n + 1) * row * 4);  // + one row the join kernel may read ahead
  ScratchScope scope;  // the read-back below synchronises the stream
  TmpBuf nsum;
  nsum.alloc(8);
  SJ_HIP(hipMemsetAsync(nsum.p, 0, 8, s));
  launch_norm_tables(ix.X.as<float>(), ix.n, ix.dp, s_hi, s_lo, kappa, ix.norm_qa.as<float>(),
                     ix.norm_cr.as<float>(), nsum.as<double>(), s);
  double h = 0.0;
  SJ_HIP(hipMemcpyAsync(&h, nsum.p, 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  const double mean = h / (double)ix.n;
  const bool narrow = kappa * (6.0 * mean + 2.0 * s_hi) <= kNormBandMax * ix.eps2;
  if (ix.opt.fp32_form == SJ_FP32_NORM || narrow) {
    ix.norm_form = true;
    ix.info.fp32_form = SJ_FP32_NORM;
  } else {
    ix.norm_qa.reset();
    ix.norm_cr.reset();
  }
}

void fill_defaults(sj_options *o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = SJ_PREC_FP32;
  o->struct_size = sizeof(sj_options);
  o->k = 0;
  o->k_min = 4;
  o->k_max = 8;
  o->reorder = 1;
  o->shortc = 1;
  o->precision = SJ_PREC_FP32;
}

void build(sj_index &ix, const float *points, hipStream_t s) {
  ScratchScope scope;  // temporaries live until the final event synchronisation
  Event ev0, ev1;
  SJ_HIP(hipEventRecord(ev0.e, s));
  const uint64_t n = ix.n;
  const uint32_t d = ix.d;
  ix.dp = padded_dim(d);
  ix.perm.resize(d);
  ix.inv_perm.resize(d);
  ix.dmin.assign(d, 0.0);
  ix.dmax.assign(d, 0.0);
  ix.counters.alloc(64);
  compute_thresholds(ix);
  if (n == 0) {
    std::iota(ix.perm.begin(), ix.perm.end(), 0u);
    for (uint32_t r = 0; r < d; ++r) ix.inv_perm[ix.perm[r]] = (uint16_t)r;
    ix.k = 0;
    SJ_HIP(hipEventRecord(ev1.e, s));
    SJ_HIP(hipEventSynchronize(ev1.e));
    ix.info.ms_build = elapsed_ms(ev0, ev1);
    return;
  }
  // input on the device (copy host input once)
  TmpBuf staged;
  const float *P = points;
  if (!is_device_pointer(points)) {
    staged.alloc(n * d * sizeof(float));
    SJ_HIP(hipMemcpyAsync(staged.p, points, n * d * sizeof(float), hipMemcpyHostToDevice, s));
    P = staged.as<float>();
  }
  // a1/a2: min/max, finiteness, sample variance
  TmpBuf stats;
  stats.alloc(d * 32 + 256);
  uint32_t *gmin = stats.as<uint32_t>();
  uint32_t *gmax = gmin + d;
  uint32_t *bad = gmax + d;
  double *var = reinterpret_cast<double *>(stats.as<char>() + ((d * 8 + 8 + 63) / 64) * 64);
  launch_minmax(P, n, d, gmin, gmax, bad, s);
  const uint64_t stride = n <= 10000 ? 1 : 100;
  const uint64_t m = (n + stride - 1) / stride;
  launch_variance(P, d, stride, m, var, s);
  std::vector<uint32_t> hmin(d), hmax(d);
  uint32_t hbad = 0;
  std::vector<double> hvar(2 * (size_t)d);  // variances, then means
  SJ_HIP(hipMemcpyAsync(hmin.data(), gmin, d * 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipMemcpyAsync(hmax.data(), gmax, d * 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipMemcpyAsync(hvar.data(), var, d * 16, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  if (hbad) fail(SJ_ERR_INVALID_ARG, "points contain NaN or Inf coordinates");
  ix.dmean.assign(hvar.begin() + d, hvar.end());
  for (uint32_t t = 0; t < d; ++t) {
    ix.dmin[t] = (double)ordered_to_float(hmin[t]);
    ix.dmax[t] = (double)ordered_to_float(hmax[t]);
  }
  std::iota(ix.perm.begin(), ix.perm.end(), 0u);
  if (ix.opt.reorder)
    std::stable_sort(ix.perm.begin(), ix.perm.end(),
                     [&](uint32_t a, uint32_t b) { return hvar[a] > hvar[b]; });
  for (uint32_t r = 0; r < d; ++r) ix.inv_perm[ix.perm[r]] = (uint16_t)r;
  ix.perm_d.alloc(d * 4);
  ix.inv_perm_d.alloc(d * 2);
  SJ_HIP(hipMemcpyAsync(ix.perm_d.p, ix.perm.data(), d * 4, hipMemcpyHostToDevice, s));
  SJ_HIP(hipMemcpyAsync(ix.inv_perm_d.p, ix.inv_perm.data(), d * 2, hipMemcpyHostToDevice, s));

  // buffers
  BuildTmp t;
  t.keys[0].alloc(n * 8);
  t.keys[1].alloc(n * 8);
  t.ids[0].alloc(n * 4);
  t.ids[1].alloc(n * 4);
  t.flag.alloc(n * 4);
  t.radix.alloc(radix_tmp_bytes(n));
  t.scan.alloc(scan_tmp_bytes(n + 1) + 256);
  t.small.alloc(256);
  t.nbr_count.alloc((n + 1) * 4);
  t.cand_sum.alloc((n + 1) * 8);
  t.prod.alloc((n + 1) * 8);
  ix.cell_key.alloc((n + 1) * 8);
  ix.cell_start.alloc((n + 1) * 4);
  ix.X.alloc((n + 1) * ix.dp * 4);  // + one row the join kernel may read ahead
  ix.orig_id.alloc(n * 4);
  ix.pos_of.alloc(n * 4);

  // k: explicit or chosen by the cost model over [k_min, k_max]
  const uint32_t kcap = std::min<uint32_t>(d, kKeyMaxDims);
  Geometry g;
  if (ix.opt.k > 0) {
    const uint32_t k = std::min<uint32_t>((uint32_t)ix.opt.k, kcap);
    if (!make_geometry(ix, k, g))
      fail(SJ_ERR_KEY_OVERFLOW, "the cell id over k=" + std::to_string(k) +
                                    " dimensions does not fit in 63 bits");
  } else {
    const uint32_t k0 = std::max<uint32_t>(1, std::min(ix.opt.k_min ? ix.opt.k_min : 4u, kcap));
    const uint32_t k1 = std::max(k0, std::min(ix.opt.k_max ? ix.opt.k_max : 8u, kcap));
    double best = 0.0;
    bool have = false;
    // With at most two cells along each of the first k1 reordered dimensions
    // every pair of cells is adjacent, so C(k) = n^2 for every k, while the
    // enumeration term grows with k: the model's choice is k0 without
    // building the other grids.
    bool all_adjacent = true;
    for (uint32_t r = 0; r < k1 && all_adjacent; ++r) {
      const uint32_t t = ix.perm[r];
      all_adjacent = std::floor((ix.dmax[t] - ix.dmin[t]) / (ix.eps * kWidthSlack)) <= 1.0;
    }
    if (all_adjacent && make_geometry(ix, k0, g)) have = true;
    for (uint32_t k = k0; k <= k1 && !all_adjacent; ++k) {
      Geometry gk;
      if (!make_geometry(ix, k, gk)) break;  // longer keys would overflow: stop
      const uint64_t C = build_grid(ix, P, gk, t, s, false);
      // adjacency lists that could pass 2^32 - 1 entries (at most 3^k, and
      // at most #G, per cell) rule out this k and every larger one
      const double nc_k = (double)ix.ncell;
      if (nc_k * std::min<double>((double)gk.np.n_off, nc_k) > 4294967295.0) break;
      const double cost = (double)C * 0.5 / kPairsPerSec +
                          (double)ix.ncell * (double)gk.np.n_off / kLookupsPerSec;
      if (!have || cost < best * (1.0 - 1e-9)) {
        best = cost;
        g = gk;
        have = true;
      } else if (cost > best * 1.02) {
        // C(k) never grows with k (one more indexed dimension only removes
        // candidates) while the lookups grow as 3^k: once the cost is past
        // the minimum, larger k are not built
        break;
      }
    }
    if (!have) {
      if (!make_geometry(ix, 1, g)) fail(SJ_ERR_KEY_OVERFLOW, "no usable k");
    }
  }
  ix.k = g.k;
  ix.geom = g;
  ix.candidates = build_grid(ix, P, g, t, s, true);
  ix.n_near = n;

  // candidate runs and the work units of the symmetric full join
  ix.n_runs_sym = build_runs(ix, 1, ix.run_off_sym, ix.runs_sym, t, s);
  ix.n_runs_full = build_runs(ix, 0, ix.run_off_full, ix.runs_full, t, s);
  if (ix.opt.precision == SJ_PREC_FP32) choose_fp32_form(ix, s);
  // one query per lane when units of the class's width would spend more
  // than a quarter of their lane work on idle query slots (many small cells)
  // (a job of the batched path runs on the matrix cores with its own units)
  ix.small_cells =
      !ix.batch_job &&
      live_slot_share(ix, t.cand_sum.as<uint64_t>(),
                      64u * (uint32_t)fp32_rq_for(ix.dp, ix.norm_form, false), s) <
          kLiveSlotShareMin;
  ix.tq = 64u * (uint32_t)fp32_rq_for(ix.dp, ix.norm_form, ix.small_cells);
  ix.info.units = ix.small_cells ? SJ_UNITS_SMALL_CELLS : SJ_UNITS_CELL;
  uint64_t ev = 0;
  DevBuf probe, probe_r;
  const bool su = ix.opt.sortidu != 0;  // units from per-block SORTIDU ranges
  if (ix.batch_job) {
    // a job of the batched path cuts its own units from runs_sym later; its
    // symmetric pair count is (C + n) / 2 up to the tiles' rounding
    ev = (ix.candidates + n) / 2;
  } else {
    build_workunits(ix, 1, nullptr, 0, ix.run_off_sym, ix.runs_sym, ix.tq, 16384, probe, &ev, s,
                    false, su ? &probe_r : nullptr);
    ix.tc = choose_tc(ev, ix.tq);
    // FP32 units of small cells from groups of neighbouring cells
    ix.wu_grouped = kFp32CellGroups && ix.small_cells && !su &&
                    ix.opt.precision == SJ_PREC_FP32;
    if (ix.wu_grouped) build_cell_groups(ix, ix.tq, ix.groups, s);
    const CellGroups *grp = ix.wu_grouped ? &ix.groups : nullptr;
    ix.n_wu = build_workunits(ix, 1, nullptr, 0, grp ? grp->run_off : ix.run_off_sym,
                              grp ? grp->runs : ix.runs_sym, ix.tq, ix.tc, ix.wu,
                              &ix.evaluated_sym, s, kWuByStretch, su ? &ix.uruns : nullptr, grp);
  }
  if (ix.opt.precision != SJ_PREC_FP32) {
    mfma_prepare(ix, s);
    ix.tq_m = 32u * (uint32_t)mfma_qb(ix.kp);         // per wave (batched kernel)
    ix.tc_m = choose_tc(ev, ix.tq_m);
    // single join: workgroup units, or per-wave units when more than a
    // quarter of the workgroup units' lane work would fall on idle query
    // slots (the work-weighted test of the FP32 join)
    const uint32_t tq_wg = mfma_wg_queries(ix.kp);
    // (also for a job of the batched path: its sampled count runs these units)
    ix.mfma_per_wave =
        live_slot_share(ix, t.cand_sum.as<uint64_t>(), tq_wg, s) < kLiveSlotShareMin;
    ix.info.units = ix.mfma_per_wave ? SJ_UNITS_SMALL_CELLS : SJ_UNITS_CELL;
    ix.tq_single = ix.mfma_per_wave ? mfma_wave_queries() : tq_wg;
    ix.tc_single = ix.mfma_per_wave ? choose_tc(ev, ix.tq_single)
                                    : std::max<uint32_t>(1024, choose_tc(ev, tq_wg) * 4);
    if (!ix.batch_job)
      ix.n_wu_m = build_workunits(ix, 1, nullptr, 0, ix.run_off_sym, ix.runs_sym, ix.tq_single,
                                  ix.tc_single, ix.wu_m, &ix.evaluated_sym_m, s, kWuByStretch,
                                  su ? &ix.uruns_m : nullptr);
  }

  SJ_HIP(hipEventRecord(ev1.e, s));
  SJ_HIP(hipEventSynchronize(ev1.e));
  ix.info.ms_build = elapsed_ms(ev0, ev1);
}

// The general join Q join_eps E (Section 3.1; the self-join is E join E):
// the queries are binned into E's grid (same k, cell side and origin, the
// dimension order of E's variance reorder), each query cell searches its
// 3^k adjacent cells in E's cell table, and the distance kernels compare
// query rows of q against candidate rows of E, one direction only.
void build_query(sj_index &q, const sj_index &E, const float *queries, hipStream_t s) {
  ScratchScope scope;  // temporaries live until the final event synchronisation
  Event ev0, ev1;
  SJ_HIP(hipEventRecord(ev0.e, s));
  const uint64_t m = q.n;
  const uint32_t d = E.d;
  q.entries = &E;
  q.d = d;
  q.dp = E.dp;
  q.eps = E.eps;
  q.eps2 = E.eps2;
  q.opt = E.opt;
  q.perm = E.perm;
  q.inv_perm = E.inv_perm;
  q.dmin = E.dmin;
  q.dmax = E.dmax;
  q.lo32 = E.lo32;
  q.hi32 = E.hi32;
  q.k = E.k;
  q.geom = E.geom;
  q.prec = E.prec;
  q.fmt = E.fmt;
  q.kp = E.kp;
  q.norm_form = E.norm_form;
  q.info.fp32_form = E.info.fp32_form;
  q.tq = E.tq;
  q.counters.alloc(64);
  q.perm_d.alloc(d * 4);
  q.inv_perm_d.alloc(d * 2);
  SJ_HIP(hipMemcpyAsync(q.perm_d.p, q.perm.data(), d * 4, hipMemcpyHostToDevice, s));
  SJ_HIP(hipMemcpyAsync(q.inv_perm_d.p, q.inv_perm.data(), d * 2, hipMemcpyHostToDevice, s));
  q.n_near = 0;
  q.ncell = 0;
  auto finish = [&] {
    SJ_HIP(hipEventRecord(ev1.e, s));
    SJ_HIP(hipEventSynchronize(ev1.e));
    q.info.ms_build = elapsed_ms(ev0, ev1);
  };
  if (m == 0) return finish();
  TmpBuf staged;
  const float *P = queries;
  if (!is_device_pointer(queries)) {
    staged.alloc(m * d * sizeof(float));
    SJ_HIP(hipMemcpyAsync(staged.p, queries, m * d * sizeof(float), hipMemcpyHostToDevice, s));
    P = staged.as<float>();
  }
  {  // finiteness of the queries
    TmpBuf st;
    st.alloc(d * 8 + 64);
    uint32_t *gmin = st.as<uint32_t>(), *gmax = gmin + d, *bad = gmax + d;
    launch_minmax(P, m, d, gmin, gmax, bad, s);
    uint32_t hbad = 0;
    SJ_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    if (hbad) fail(SJ_ERR_INVALID_ARG, "queries contain NaN or Inf coordinates");
  }
  if (E.n == 0) return finish();  // nothing to find
  const Geometry &g = E.geom;
  // queries more than two cell sides outside E's range in some dimension
  // have no neighbour (k_query_keys); the rest lie within that margin
  const double margin = 2.0 * g.kp.w;
  std::vector<double> bounds(2 * (size_t)d);
  for (uint32_t t = 0; t < d; ++t) {
    bounds[t] = E.dmin[t] - margin;
    bounds[d + t] = E.dmax[t] + margin;
  }
  if (E.prec != SJ_PREC_FP32 && E.fmt == kFmtF16) {
    // the near queries' centred coordinates stay below 16384, so -2 x~ fits FP16
    double reach = 0.0;
    for (uint32_t r = 0; r < d; ++r) {
      const uint32_t t = E.perm[r];
      const double c = (double)E.mfma_centre[r];
      reach = std::max(reach, std::max(std::fabs(bounds[d + t] - c), std::fabs(bounds[t] - c)));
    }
    if (!(reach * (1.0 + 1e-6) <= 16384.0))
      fail(SJ_ERR_INVALID_ARG,
           "epsilon is too large against the FP16 range of this index; build it with "
           "SJ_PREC_BF16 or SJ_PREC_FP32 for this query join");
  }
  BuildTmp t;
  t.keys[0].alloc(m * 8);
  t.keys[1].alloc(m * 8);
  t.ids[0].alloc(m * 4);
  t.ids[1].alloc(m * 4);
  t.flag.alloc(m * 4);
  t.radix.alloc(radix_tmp_bytes(m));
  t.scan.alloc(scan_tmp_bytes(m + 1) + 256);
  t.small.alloc(256);
  t.nbr_count.alloc((m + 1) * 4);
  t.cand_sum.alloc((m + 1) * 8);
  t.prod.alloc((m + 1) * 8);
  TmpBuf bd;
  bd.alloc(bounds.size() * 8);
  SJ_HIP(hipMemcpyAsync(bd.p, bounds.data(), bounds.size() * 8, hipMemcpyHostToDevice, s));
  unsigned long long *d_far = reinterpret_cast<unsigned long long *>(t.small.as<char>() + 64);
  SJ_HIP(hipMemsetAsync(d_far, 0, 8, s));
  const uint64_t far_key = 1ull << g.key_bits;  // above every key of key_bits bits
  launch_query_keys(P, m, d, g.kp, bd.as<double>(), bd.as<double>() + d, far_key,
                    t.keys[0].as<uint64_t>(), t.ids[0].as<uint32_t>(), d_far, s);
  uint64_t *kb[2] = {t.keys[0].as<uint64_t>(), t.keys[1].as<uint64_t>()};
  uint32_t *vb[2] = {t.ids[0].as<uint32_t>(), t.ids[1].as<uint32_t>()};
  std::vector<int> shifts;
  for (uint32_t b = 0; b <= g.key_bits; b += 8) shifts.push_back((int)b);
  radix_sort_u64(kb, vb, m, shifts.data(), (int)shifts.size(), t.radix.p, s);
  q.X.alloc((m + 1) * q.dp * 4);
  q.orig_id.alloc(m * 4);
  q.pos_of.alloc(m * 4);
  launch_gather(P, m, d, q.dp, q.perm_d.as<uint32_t>(), vb[0], q.X.as<float>(),
                q.orig_id.as<uint32_t>(), q.pos_of.as<uint32_t>(), s);
  unsigned long long h_far = 0;
  SJ_HIP(hipMemcpyAsync(&h_far, d_far, 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  q.n_near = m - h_far;  // far queries sort last: positions [n_near, m)
  q.cell_key.alloc((q.n_near + 1) * 8);
  q.cell_start.alloc((q.n_near + 1) * 4);
  if (q.n_near) {
    uint32_t *d_ncell = t.small.as<uint32_t>();
    launch_compact(kb[0], q.n_near, g.fine_bits, t.flag.as<uint32_t>(), d_ncell,
                   q.cell_key.as<uint64_t>(), q.cell_start.as<uint32_t>(), t.scan.p, s);
    uint32_t h_ncell = 0;
    SJ_HIP(hipMemcpyAsync(&h_ncell, d_ncell, 4, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    q.ncell = h_ncell;
  }
  if (q.ncell == 0) return finish();
  q.candidates = build_neighbors(q, E, g.np, t, s, true);
  q.small_cells =  // as for an index, over the query cells
      live_slot_share(q, t.cand_sum.as<uint64_t>(),
                      64u * (uint32_t)fp32_rq_for(q.dp, q.norm_form, false), s) <
      kLiveSlotShareMin;
  q.tq = 64u * (uint32_t)fp32_rq_for(q.dp, q.norm_form, q.small_cells);
  q.info.units = q.small_cells ? SJ_UNITS_SMALL_CELLS : SJ_UNITS_CELL;
  q.n_runs_full = build_runs(q, 0, q.run_off_full, q.runs_full, t, s);
  if (q.norm_form) {  // the queries' table of the norm form (E holds the candidates')
    const NormParams np = norm_params(q);
    const uint64_t row = (uint64_t)norm_table_row(q.dp);
    q.norm_qa.alloc(q.n_near * row * 4);
    TmpBuf cr, nsum;
    cr.alloc((q.n_near + 1) * row * 4);
    nsum.alloc(8);
    SJ_HIP(hipMemsetAsync(nsum.p, 0, 8, s));
    launch_norm_tables(q.X.as<float>(), q.n_near, q.dp, np.s_hi, np.s_lo, np.kappa,
                       q.norm_qa.as<float>(), cr.as<float>(), nsum.as<double>(), s);
  }
  uint64_t ev = 0;
  DevBuf probe, probe_r;
  const bool su = q.opt.sortidu != 0;  // units from per-block SORTIDU ranges
  build_workunits(q, 0, nullptr, 0, q.run_off_full, q.runs_full, q.tq, 16384, probe, &ev, s,
                  false, su ? &probe_r : nullptr);
  q.tc = choose_tc(ev, q.tq);
  if (q.prec == SJ_PREC_FP32) {
    q.n_wu = build_workunits(q, 0, nullptr, 0, q.run_off_full, q.runs_full, q.tq, q.tc, q.wu,
                             &q.evaluated_sym, s, kWuByStretch, su ? &q.uruns : nullptr);
  } else {
    // the queries' operands and thresholds against E's centring and maxima
    q.n_pad = (q.n_near + 31) / 32 * 32 + 64;
    const uint64_t np = q.n_pad;
    q.XB.alloc(np * q.kp * 2);
    q.thi.alloc(np * 4);
    q.tlo.alloc(np * 4);
    TmpBuf xa, cn, cdev, norm2, distc, fold, maxima;
    xa.alloc(np * q.kp * 2);
    cn.alloc(np * 4);
    cdev.alloc(d * 4);
    norm2.alloc(np * 8);
    distc.alloc(np * 8);
    fold.alloc(np * 8);
    maxima.alloc(64);
    SJ_HIP(hipMemcpyAsync(cdev.p, E.mfma_centre.data(), d * 4, hipMemcpyHostToDevice, s));
    launch_mfma_prep(q.fmt, q.X.as<float>(), q.n_near, np, d, q.dp, q.kp, cdev.as<float>(), xa.p,
                     q.XB.p, cn.as<float>(), norm2.as<double>(), distc.as<double>(),
                     fold.as<double>(), maxima.as<unsigned long long>(), s);
    launch_mfma_thresholds(q.n_near, np, E.mfma_band, norm2.as<double>(), distc.as<double>(),
                           E.mfma_max.as<unsigned long long>(), q.thi.as<float>(),
                           q.tlo.as<float>(), s);
    const uint32_t tq_wg = mfma_wg_queries(q.kp);
    q.mfma_per_wave =
        live_slot_share(q, t.cand_sum.as<uint64_t>(), tq_wg, s) < kLiveSlotShareMin;
    q.info.units = q.mfma_per_wave ? SJ_UNITS_SMALL_CELLS : SJ_UNITS_CELL;
    q.tq_single = q.mfma_per_wave ? mfma_wave_queries() : tq_wg;
    q.tc_single = q.mfma_per_wave ? choose_tc(ev, q.tq_single)
                                  : std::max<uint32_t>(1024, choose_tc(ev, tq_wg) * 4);
    q.n_wu_m = build_workunits(q, 0, nullptr, 0, q.run_off_full, q.runs_full, q.tq_single,
                               q.tc_single, q.wu_m, &q.evaluated_sym_m, s, kWuByStretch,
                               su ? &q.uruns_m : nullptr);
    q.evaluated_sym = q.evaluated_sym_m;
  }
  finish();
}

MfmaView mfma_view(const sj_index &ix, const uint2 *runs, const uint32_t *qlist, int sym) {
  const sj_index &E = entries_of(ix);  // candidates; ix holds the queries
  MfmaView v{};
  v.XA = E.XA.p;
  v.XB = ix.XB.p;
  v.cn = E.cn.as<float>();
  v.thi = ix.thi.as<float>();
  v.tlo = ix.tlo.as<float>();
  v.X = E.X.as<float>();
  v.Xq = ix.X.as<float>();
  v.inv_perm = ix.inv_perm_d.as<uint16_t>();
  v.runs = runs;
  v.qlist = qlist;
  v.d = ix.d;
  v.dp = ix.dp;
  v.eps2 = ix.eps2;
  v.symmetric = sym;
  v.pshift = 32;
  v.key_hi = 0;
  v.hi = ix.hi32;
  v.pad_row = (uint32_t)E.n;  // rows n .. n_pad-1: zero operands, norm +inf
  return v;
}

// One launch of the distance kernel over a set of work units.
bool debug_undersize();
int debug_hits_mode();
int debug_box_mode();
uint64_t read_counter(sj_index &ix, int which, hipStream_t s);
constexpr uint64_t kBandStart = 1u << 20;       // least band-list slots of a join
constexpr uint64_t kCountBandStart = 1u << 16;  // and of a sampled count
// result + band pairs per 32 x 32 tile above which the matrix-core kernels
// scan every tile's elements instead of testing each tile's minimum first
// (measured: 1.5 against the former 0.2 / 0.05 with a mask-building hit path
// took the 2M x 16 FP16 join at S_D 512 from 168 to 135 ms)
constexpr double kFrequentHits = 1.5;
constexpr uint32_t kBoxMaxDims = 24;  // dimensions up to which workgroup units use the box
constexpr double kBoxMaxHitsPerTile = 0.1;  // and hits per 32 x 32 tile below which

void join_launch(sj_index &ix, const DevBuf &wu, uint64_t n_wu, const DevBuf &runs,
                 const uint32_t *qlist, int sym, int count_only, uint64_t *out, uint64_t cap,
                 hipStream_t s, float *ms, uint32_t skip_below = 0) {
  const sj_index &E = entries_of(ix);  // candidates; ix holds the queries
  JoinLaunch a{};
  a.X = E.X.as<float>();
  a.orig_id = E.orig_id.as<uint32_t>();
  a.Xq = ix.X.as<float>();
  a.qid = ix.orig_id.as<uint32_t>();
  a.inv_perm = ix.inv_perm_d.as<uint16_t>();
  a.wu = wu.as<WorkUnit>();
  a.n_wu = n_wu;
  a.runs = runs.as<uint2>();
  a.qlist = qlist;
  a.d = ix.d;
  a.dp = ix.dp;
  a.lo = ix.lo32;
  a.hi = ix.hi32;
  a.eps2 = ix.eps2;
  a.symmetric = sym;
  a.count_only = count_only;
  a.shortc = ix.opt.shortc ? 1 : 0;
  a.out = out;
  a.capacity = cap;
  a.cursor = ix.counters.as<unsigned long long>();
  a.rechecks = ix.counters.as<unsigned long long>() + 1;
  a.rq = fp32_rq_for(ix.dp, ix.norm_form, ix.small_cells);
  a.norm = ix.norm_form ? 1 : 0;
  a.QA = ix.norm_qa.as<float>();
  a.CR = E.norm_cr.as<float>();
  a.skip_below = skip_below;
  a.skipped = ix.counters.as<unsigned long long>() + 3;
  Event e0, e1;
  SJ_HIP(hipEventRecord(e0.e, s));
  if (ix.prec != SJ_PREC_FP32) {
    MfmaLaunch m{};
    m.fmt = ix.fmt;
    m.kp = ix.kp;
    m.view = mfma_view(ix, a.runs, a.qlist, sym);
    m.wu = a.wu;
    m.n_wu = a.n_wu;
    m.out = count_only ? nullptr : out;
    m.capacity = count_only ? 0 : cap;
    m.cursor = a.cursor;
    m.rechecks = a.rechecks;
    m.per_wave = ix.mfma_per_wave ? 1 : 0;
    // hits common enough: scan the elements of every tile directly
    const double per_tile = ix.hit_density * 1024.0;
    m.hits_frequent = per_tile > kFrequentHits ? 1 : 0;
    if (const int forced = debug_hits_mode(); forced >= 0) m.hits_frequent = forced;
    // the query-box prefilter pays where 8 dimensions are a good part of
    // the distance (the bound uses the first 8 of the variance order) and
    // most candidates are far (measured: 2M x 16 uniform FP16 joins 25 % and
    // 13 % faster at 0.004 and 0.03 hits per tile, 15 % slower at 0.26)
    m.box = !m.per_wave && ix.d <= kBoxMaxDims && per_tile < kBoxMaxHitsPerTile ? 1 : 0;
    if (const int forced = debug_box_mode(); forced >= 0) m.box = m.per_wave ? 0 : forced;
    {
      // band pairs are collected during the join and rechecked afterwards,
      // one per lane; a band list that overflowed is grown and the join rerun
      // (a count-only pass counts the accepted band pairs the same way)
      unsigned long long *band_cursor = ix.counters.as<unsigned long long>() + 2;
      const uint64_t least = count_only ? kCountBandStart : kBandStart;
      const uint64_t want = debug_undersize() ? 16 : std::max(least, ix.band_hint);
      if (ix.band_cap < want) {
        ix.band_cap = want;
        ix.band.alloc(ix.band_cap * 8);
      }
      // result and recheck counts before this launch (a rerun starts from them)
      uint64_t base[2] = {0, 0};
      SJ_HIP(hipMemcpyAsync(base, ix.counters.p, 16, hipMemcpyDeviceToHost, s));
      SJ_HIP(hipStreamSynchronize(s));
      for (int attempt = 0;; ++attempt) {
        SJ_HIP(hipMemsetAsync(band_cursor, 0, 8, s));
        m.view.band = ix.band.as<uint64_t>();
        m.view.band_cap = ix.band_cap;
        m.view.band_cursor = band_cursor;
        launch_join_mfma(m, s);
        if (!count_only) ix.info.join_launches++;
        launch_band_recheck(m.view, m.out, m.capacity, a.cursor, a.rechecks, s);
        const uint64_t nb = read_counter(ix, 2, s);
        if (nb <= ix.band_cap) break;
        if (attempt == 2) fail(SJ_ERR_DEVICE, "band list size did not settle");
        ix.band_cap = nb + nb / 8;
        ix.band.alloc(ix.band_cap * 8);
        // the launch starts over
        SJ_HIP(hipMemcpyAsync(ix.counters.p, base, 16, hipMemcpyHostToDevice, s));
        SJ_HIP(hipStreamSynchronize(s));
      }
    }
  } else {
    launch_join_fp32(a, s);
    if (!count_only) ix.info.join_launches++;
  }
  SJ_HIP(hipEventRecord(e1.e, s));
  SJ_HIP(hipEventSynchronize(e1.e));
  *ms += elapsed_ms(e0, e1);
}

uint64_t read_counter(sj_index &ix, int which, hipStream_t s) {
  uint64_t v = 0;
  SJ_HIP(hipMemcpyAsync(&v, ix.counters.as<uint64_t>() + which, 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
  return v;
}

// Estimate |R| from a strided sample of query positions (Section 3.2.2:
// a count-only pass over a fraction of the points).  Counts pairs the FP32
// filter cannot reject, so it is an upper-bound estimate.  The sample is
// 1/64 of the queries, at least 1024 and at most 8192 of them, so it stays
// a small part of the join's work for small and mid-sized inputs too.  It
// takes runs of 8 consecutive positions (mostly of one cell): a wave then
// counts up to 8 sampled queries against a cell's candidates where single
// positions would leave it one, which matters when cells are small.
constexpr uint32_t kSampleRun = 8;

uint64_t estimate_pairs(sj_index &ix, hipStream_t s, float *ms) {
  const uint64_t n = ix.n_near;  // query positions in cells
  const uint64_t target = std::min<uint64_t>(8192, std::max<uint64_t>(1024, n / 64));
  uint64_t stride = 1, nq = n;
  uint32_t run = 1;
  if (n > target) {
    run = kSampleRun;
    const uint64_t nrun = target / run;  // >= 128
    stride = n / nrun;                   // >= run, as n > nrun * run
    nq = nrun * run;                     // last position (nrun-1) stride + run-1 < n
  }
  ScratchScope scope;  // the read-back of the count below synchronises the stream
  TmpBuf ql;
  DevBuf wu;
  ql.alloc(nq * 4);
  launch_iota_strided(ql.as<uint32_t>(), nq, stride, run, s);
  uint64_t ev = 0;
  // the matrix-core path counts with its own filter and its band list (no
  // keys are stored at capacity 0); the FP32 path has a count-only kernel
  const bool mf = ix.prec != SJ_PREC_FP32;
  // candidate chunks of at most 4096: the sample's few units are split
  // finely enough to spread over the chip
  const uint64_t nwu = build_workunits(ix, 0, ql.as<uint32_t>(), nq, ix.run_off_full,
                                       ix.runs_full, mf ? ix.tq_single : ix.tq,
                                       mf ? std::min<uint32_t>(ix.tc_single, 4096) : 4096, wu,
                                       &ev, s);
  SJ_HIP(hipMemsetAsync(ix.counters.p, 0, 16, s));
  // the sample's band list: at most one pair in 512 is expected in the band
  // (a larger band reruns the count with the list at its exact size)
  if (mf) ix.band_hint = ev / 512;
  join_launch(ix, wu, nwu, ix.runs_full, ql.as<uint32_t>(), 0, 1, nullptr, 0, s, ms);
  const uint64_t cnt = read_counter(ix, 0, s);
  const double scale = (double)n / (double)nq;
  if (mf) {
    // band pairs of the sample size the deferred recheck list of the join
    const double nband = (double)read_counter(ix, 1, s);
    ix.band_hint = (uint64_t)std::ceil(nband * scale * 1.25) + (1u << 16);
    ix.hit_density = ev ? ((double)cnt + nband) / (double)ev : 0.0;
  }
  return (uint64_t)std::ceil((double)cnt * scale);
}

uint64_t default_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return 1ull << 32;
  }
  int dev = 0;
  SJ_HIP(hipGetDevice(&dev));
  // blocks the library's cache holds are free for this run
  return (uint64_t)((double)(fr + dev_cached_bytes(dev)) * 0.7);
}

void sort_pairs(sj_index &ix, DevBuf &a, DevBuf &b, uint64_t cnt, hipStream_t s,
                DevBuf *keep_tmp = nullptr) {
  const uint64_t ne = entries_of(ix).n;
  const uint32_t ibits = bits_for(ix.n ? ix.n - 1 : 0), jbits = bits_for(ne ? ne - 1 : 0);
  std::vector<int> sh, wd;
  digit_plan(jbits, ibits, sh, wd);
  DevBuf own;
  DevBuf &tmp = keep_tmp ? *keep_tmp : own;  // a caller's buffer outlives the queued sort
  tmp.ensure(radix_tmp_bytes(cnt));
  uint64_t *kb[2] = {a.as<uint64_t>(), b.as<uint64_t>()};
  radix_sort_u64(kb, nullptr, cnt, sh.data(), (int)sh.size(), tmp.p, s, nullptr, wd.data());
}

// Single batch: symmetric join of all work units into device memory.
void run_single(sj_index &ix, uint64_t est, hipStream_t s) {
  uint64_t cap = est + est / 8 + (1u << 20);
  if (debug_undersize()) cap = std::max<uint64_t>(1, est / 16);
  float ms_join = 0.0f;
  DevBuf other;
  for (int attempt = 0; attempt < 3; ++attempt) {
    ix.pairs.alloc(cap * 8);
    SJ_HIP(hipMemsetAsync(ix.counters.p, 0, 16, s));
    const bool m = ix.prec != SJ_PREC_FP32;
    const bool self = !ix.entries;  // a self-join's units are symmetric
    const bool grouped = !m && ix.wu_grouped;
    const DevBuf &runs = ix.opt.sortidu ? (m ? ix.uruns_m : ix.uruns)
                         : grouped      ? ix.groups.runs
                                        : (self ? ix.runs_sym : ix.runs_full);
    join_launch(ix, m ? ix.wu_m : ix.wu, m ? ix.n_wu_m : ix.n_wu, runs, nullptr, self ? 1 : 0, 0,
                ix.pairs.as<uint64_t>(), cap, s, &ms_join);
    const uint64_t got = read_counter(ix, 0, s);
    if (got <= cap) {
      ix.total = got;
      break;
    }
    cap = got;  // exact now
    if (attempt == 2) fail(SJ_ERR_DEVICE, "result count did not settle");
  }
  ix.info.rechecks = read_counter(ix, 1, s);
  ix.info.ms_join += ms_join;
  Event e0, e1;
  SJ_HIP(hipEventRecord(e0.e, s));
  if (ix.prec != SJ_PREC_FP32)
    launch_pos_to_id(ix.pairs.as<uint64_t>(), ix.total, ix.orig_id.as<uint32_t>(),
                     entries_of(ix).orig_id.as<uint32_t>(), s);
  other.alloc(ix.total * 8);
  sort_pairs(ix, ix.pairs, other, ix.total, s);
  SJ_HIP(hipEventRecord(e1.e, s));
  SJ_HIP(hipEventSynchronize(e1.e));
  ix.info.ms_sort += elapsed_ms(e0, e1);
  ix.info.batches = 1;
  ix.info.evaluated = ix.prec != SJ_PREC_FP32 ? ix.evaluated_sym_m : ix.evaluated_sym;
  ix.on_host = false;
}

// The spill of a symmetric batched run overflowed: run one-directionally.
struct OneWayRetry {};

// Several batches over ranges of caller indices [i0, i1), each sorted and
// copied to pinned host memory while the next batch computes (Section 3.2.2,
// Figure 5), through three result slots.  An FP32 self-join takes each
// unordered pair once (sym): the batch of [i0, i1) skips candidates below i0
// (their pairs belong to an earlier batch, which took them), keeps (i, j)
// for j >= i and mirrors it to (j, i), into this batch when j < i1, else
// into a device spill that the batch holding j takes up.  Other runs
// (matrix cores, query joins) join a batch's queries against all their
// candidates.  Buffers live across batches, so that no free in the loop
// waits for the copies in flight.
void run_batched(sj_index &ix, uint64_t est, uint64_t per_batch, bool sym, hipStream_t s) {
  const uint64_t n = ix.n;
  uint64_t nb = std::max<uint64_t>(1, (est + per_batch - 1) / per_batch);
  nb = std::max<uint64_t>(nb, ix.opt.min_batches ? ix.opt.min_batches : 1);
  nb = std::min<uint64_t>(nb, n);
  constexpr int kSlots = 3;
  struct Slot {
    DevBuf keys, other, sort_tmp;
    Event done_copy;
    bool busy = false;
  } slots[kSlots];
  struct Copy {
    hipStream_t cs = nullptr;
    ~Copy() {
      if (cs) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamDestroy(cs);
      }
    }
  } copy;
  SJ_HIP(hipStreamCreateWithFlags(&copy.cs, hipStreamNonBlocking));
  ix.host_res.clear();
  ix.host_cnt.clear();
  ix.total = 0;
  ix.info.rechecks = 0;
  uint64_t evaluated = 0, skipped = 0;
  float ms_join = 0.0f;
  const bool mf = ix.prec != SJ_PREC_FP32;
  // spill of mirrored pairs for later batches: about a quarter of the
  // result at its peak when caller order is unrelated to position
  DevBuf spill[2], cnt2;
  uint64_t spill_n = 0, spill_cap = 0;
  int sc = 0;
  if (sym) {
    spill_cap = est / 4 + est / 8 + (1u << 16);
    if (debug_undersize()) spill_cap = 16;
    spill[0].alloc(spill_cap * 8);
    spill[1].alloc(spill_cap * 8);
    cnt2.alloc(64);
  }
  const uint32_t bits = bits_for(n - 1);
  std::vector<int> qsh;
  for (uint32_t b = 0; b < bits; b += 8) qsh.push_back((int)b);
  // every batch's query positions (caller indices [i0, i1), sorted on the
  // device) and work units, before the first join: the copies of finished
  // batches then overlap the next joins rather than the short launches and
  // read-backs of this preparation (the copies run as kernels that hold
  // the compute units)
  struct Prep {
    DevBuf p32, wu;
    uint64_t nwu = 0;
  };
  std::vector<std::unique_ptr<Prep>> prep(nb);
  {
    DevBuf qk[2], rt;
    const uint64_t nq_max = (n + nb - 1) / nb + 1;
    qk[0].ensure(nq_max * 8);
    qk[1].ensure(nq_max * 8);
    rt.ensure(radix_tmp_bytes(nq_max));
    for (uint64_t bi = 0; bi < nb; ++bi) {
      const uint64_t i0 = n * bi / nb, i1 = n * (bi + 1) / nb;
      prep[bi].reset(new Prep());
      if (i1 <= i0) continue;
      const uint64_t nq = i1 - i0;
      Prep &pb = *prep[bi];
      pb.p32.alloc(nq * 4);
      launch_widen(ix.pos_of.as<uint32_t>() + i0, qk[0].as<uint64_t>(), nq, s);
      uint64_t *kb[2] = {qk[0].as<uint64_t>(), qk[1].as<uint64_t>()};
      radix_sort_u64(kb, nullptr, nq, qsh.data(), (int)qsh.size(), rt.p, s);
      launch_narrow(kb[0], pb.p32.as<uint32_t>(), nq, s);
      uint64_t ev = 0;
      pb.nwu = build_workunits(ix, 0, pb.p32.as<uint32_t>(), nq, ix.run_off_full, ix.runs_full,
                               mf ? ix.tq_single : ix.tq, mf ? ix.tc_single : ix.tc, pb.wu, &ev,
                               s, kWuByStretch);
      evaluated += ev;
    }
    SJ_HIP(hipStreamSynchronize(s));
  }
  std::vector<std::unique_ptr<Event>> sort_ev;  // (start, end) of each sort, read at the end
  uint64_t slot = 0;
  for (uint64_t bi = 0; bi < nb; ++bi) {
    const uint64_t i0 = n * bi / nb, i1 = n * (bi + 1) / nb;
    if (i1 <= i0) continue;
    const DevBuf &p32 = prep[bi]->p32, &wu = prep[bi]->wu;
    const uint64_t nwu = prep[bi]->nwu;
    Slot &sl = slots[slot % kSlots];
    if (sl.busy) {
      SJ_HIP(hipEventSynchronize(sl.done_copy.e));
      sl.busy = false;
    }
    // a batch holds about est / nb pairs (min_batches may ask for more
    // batches than the budget needs)
    const uint64_t expect = std::min(per_batch, est / nb + est / nb / 4);
    uint64_t cap = expect + expect / 8 + (1u << 16);
    if (debug_undersize()) cap = std::max<uint64_t>(1, expect / 16);
    uint64_t got = 0;
    for (int attempt = 0; attempt < 3; ++attempt) {
      sl.keys.ensure(cap * 8);
      SJ_HIP(hipMemsetAsync(ix.counters.p, 0, 32, s));
      join_launch(ix, wu, nwu, ix.runs_full, p32.as<uint32_t>(), 0, 0, sl.keys.as<uint64_t>(),
                  cap, s, &ms_join, sym ? (uint32_t)i0 : 0u);
      uint64_t c4[4];
      SJ_HIP(hipMemcpyAsync(c4, ix.counters.p, 32, hipMemcpyDeviceToHost, s));
      SJ_HIP(hipStreamSynchronize(s));
      got = c4[0];
      if (got <= cap) {
        ix.info.rechecks += c4[1];
        skipped += c4[3];
        break;
      }
      if (attempt == 2) fail(SJ_ERR_DEVICE, "batch result count did not settle");
      cap = got;
    }
    auto e0 = std::make_unique<Event>(), e1 = std::make_unique<Event>();
    SJ_HIP(hipEventRecord(e0->e, s));
    DevBuf *res = &sl.keys;
    uint64_t cnt = got;
    if (sym) {
      // this batch's pairs: the kept and mirrored join output, and the
      // spilled mirrors of earlier batches that belong here
      const uint64_t cap_o = 2 * got + spill_n + 1;
      sl.other.ensure(cap_o * 8);
      auto *c2 = cnt2.as<unsigned long long>();
      launch_fill_u64(c2, 2, 0ull, s);
      launch_spill_take(spill[sc].as<uint64_t>(), spill_n, (uint32_t)i1, sl.other.as<uint64_t>(),
                        c2, cap_o, spill[sc ^ 1].as<uint64_t>(), c2 + 1, spill_cap, s);
      launch_mirror_split(sl.keys.as<uint64_t>(), got, (uint32_t)i1, sl.other.as<uint64_t>(), c2,
                          cap_o, spill[sc ^ 1].as<uint64_t>(), c2 + 1, spill_cap, s);
      uint64_t h2[2];
      SJ_HIP(hipMemcpyAsync(h2, c2, 16, hipMemcpyDeviceToHost, s));
      SJ_HIP(hipStreamSynchronize(s));
      if (h2[1] > spill_cap) throw OneWayRetry{};
      spill_n = h2[1];
      sc ^= 1;
      cnt = h2[0];  // <= cap_o by construction
      sl.keys.ensure(std::max<uint64_t>(cnt, 1) * 8);  // the sort's second buffer
      sort_pairs(ix, sl.other, sl.keys, cnt, s, &sl.sort_tmp);
      res = &sl.other;
    } else {
      if (mf)
        launch_pos_to_id(sl.keys.as<uint64_t>(), got, ix.orig_id.as<uint32_t>(),
                         entries_of(ix).orig_id.as<uint32_t>(), s);
      sl.other.ensure(std::max<uint64_t>(got, 1) * 8);
      sort_pairs(ix, sl.keys, sl.other, got, s, &sl.sort_tmp);
    }
    SJ_HIP(hipEventRecord(e1->e, s));
    sort_ev.push_back(std::move(e0));
    sort_ev.push_back(std::move(e1));
    PinnedBuf hb;
    hb.alloc(std::max<uint64_t>(cnt, 1) * 8);
    SJ_HIP(hipStreamWaitEvent(copy.cs, sort_ev.back()->e, 0));
    SJ_HIP(hipMemcpyAsync(hb.p, res->p, cnt * 8, hipMemcpyDeviceToHost, copy.cs));
    SJ_HIP(hipEventRecord(sl.done_copy.e, copy.cs));
    sl.busy = true;
    ix.host_res.push_back(std::move(hb));
    ix.host_cnt.push_back(cnt);
    ix.total += cnt;
    ++slot;
  }
  SJ_HIP(hipStreamSynchronize(copy.cs));
  if (sym && spill_n) fail(SJ_ERR_DEVICE, "internal: mirrored pairs left after the last batch");
  for (size_t e = 0; e + 1 < sort_ev.size(); e += 2)
    ix.info.ms_sort += elapsed_ms(*sort_ev[e], *sort_ev[e + 1]);
  ix.info.ms_join += ms_join;
  ix.info.batches = (uint32_t)ix.host_res.size();
  ix.info.evaluated = evaluated - std::min(evaluated, skipped);
  ix.on_host = true;
}

void run(sj_index &ix, hipStream_t s) {
  ix.info.ms_join = 0.0f;
  ix.info.ms_sort = 0.0f;
  ix.info.join_launches = 0;
  Event e0, e1;
  SJ_HIP(hipEventRecord(e0.e, s));
  ix.pairs.reset();
  ix.host_res.clear();
  ix.host_cnt.clear();
  if (ix.n == 0 || ix.n_near == 0 || ix.ncell == 0) {
    ix.total = 0;
    ix.info.batches = 0;
  } else {
    float ms_est = 0.0f;
    const uint64_t est = estimate_pairs(ix, s, &ms_est);
    const uint64_t budget = ix.opt.mem_budget ? ix.opt.mem_budget : default_budget();
    // a single batch holds the keys twice (sort ping-pong) plus sort scratch
    const uint64_t fit = budget / 20;
    uint64_t per_batch = ix.opt.batch_pairs ? ix.opt.batch_pairs : fit;
    per_batch = std::min(per_batch, fit);
    per_batch = std::min<uint64_t>(per_batch, 1ull << 36);  // 512 GiB of keys: beyond HBM
    const uint32_t min_b = ix.opt.min_batches;
    if (est + est / 8 <= per_batch && min_b <= 1) {
      run_single(ix, est, s);
    } else {
      // FP32 self-joins take each unordered pair once across batches when
      // the spill fits the budget next to the batches
      const bool sym = ix.prec == SJ_PREC_FP32 && !ix.entries &&
                       (est / 4 + est / 8) * 16 <= budget / 2;
      try {
        run_batched(ix, est, std::max<uint64_t>(per_batch, 1), sym, s);
      } catch (const OneWayRetry &) {
        SJ_HIP(hipStreamSynchronize(s));
        run_batched(ix, est, std::max<uint64_t>(per_batch, 1), false, s);
      }
    }
  }
  SJ_HIP(hipEventRecord(e1.e, s));
  SJ_HIP(hipEventSynchronize(e1.e));
  ix.info.ms_run = elapsed_ms(e0, e1);
  ix.info.pairs = ix.total;
  ix.info.result_on_host = ix.on_host ? 1u : 0u;
  ix.ran = true;
}

// Device pointer to the sorted keys [g, g + c): the device-resident result,
// or a copy of them from the host batches into stage.
const uint64_t *stage_keys(sj_index &ix, uint64_t g, uint64_t c, DevBuf &stage, hipStream_t s) {
  if (!ix.on_host) return ix.pairs.as<uint64_t>() + g;
  stage.ensure(c * 8);
  uint64_t off = 0, copied = 0, gg = g;
  for (size_t b = 0; b < ix.host_res.size() && copied < c; ++b) {
    const uint64_t bc = ix.host_cnt[b];
    if (gg >= off + bc) {
      off += bc;
      continue;
    }
    const uint64_t from = gg - off;
    const uint64_t take = std::min(bc - from, c - copied);
    SJ_HIP(hipMemcpyAsync(stage.as<uint64_t>() + copied,
                          static_cast<uint64_t *>(ix.host_res[b].p) + from, take * 8,
                          hipMemcpyHostToDevice, s));
    copied += take;
    gg += take;
    off += bc;
  }
  return stage.as<uint64_t>();
}

// CSR row starts of the sorted result (Algorithm 1's neighbour table):
// offsets[i] = index of the first pair (i, .), offsets[n] = |R|, from the
// pairs per row (counted on the device, chunk by chunk) by an exclusive
// scan.  In a self-join every point is its own neighbour, so no row is
// empty; a query join's rows may be.
void fetch_offsets(sj_index &ix, uint64_t *offsets, hipStream_t s) {
  if (!ix.ran) fail(SJ_ERR_STATE, "fetch before a successful run");
  const uint64_t n = ix.n;
  const bool dev = is_device_pointer(offsets);
  ScratchScope scope;  // the stream is synchronised before returning
  TmpBuf counts, scan, total_d;
  DevBuf tmp, stage;
  uint64_t *doff = offsets;
  if (!dev) {
    tmp.alloc((n + 1) * 8);
    doff = tmp.as<uint64_t>();
  }
  counts.alloc((n + 1) * 8);
  scan.alloc(scan_tmp_bytes(n + 1) + 64);
  total_d.alloc(64);
  SJ_HIP(hipMemsetAsync(counts.p, 0, (n + 1) * 8, s));
  const uint64_t total = ix.total;
  const uint64_t chunk = ix.on_host ? (1ull << 24) : std::max<uint64_t>(total, 1);
  for (uint64_t g = 0; g < total; g += chunk) {
    const uint64_t c = std::min(chunk, total - g);
    const uint64_t *src = stage_keys(ix, g, c, stage, s);
    launch_row_counts(src, c, counts.as<unsigned long long>(), s);
    SJ_HIP(hipStreamSynchronize(s));  // the stage is reused by the next chunk
  }
  exclusive_scan_u64(counts.as<uint64_t>(), doff, n + 1, total_d.as<uint64_t>(), scan.p, s);
  if (!dev) SJ_HIP(hipMemcpyAsync(offsets, doff, (n + 1) * 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
}

// Pairs [first, first + cnt) of a host-resident result (pinned batches of
// sorted keys i << 32 | j) written to host columns by up to 16 threads.
void fetch_host_split(const sj_index &ix, uint64_t first, uint64_t cnt, uint32_t *oi,
                      uint32_t *oj) {
  if (!cnt || (!oi && !oj)) return;
  auto part = [&](uint64_t a, uint64_t e) {  // output entries [a, e)
    uint64_t off = 0, g = first + a;
    for (size_t b = 0; b < ix.host_res.size() && a < e; ++b) {
      const uint64_t bc = ix.host_cnt[b];
      if (g >= off + bc) {
        off += bc;
        continue;
      }
      const uint64_t *k = static_cast<const uint64_t *>(ix.host_res[b].p) + (g - off);
      const uint64_t take = std::min(off + bc - g, e - a);
      for (uint64_t t = 0; t < take; ++t) {
        const uint64_t key = k[t];
        if (oi) oi[a + t] = (uint32_t)(key >> 32);
        if (oj) oj[a + t] = (uint32_t)key;
      }
      a += take;
      g += take;
      off += bc;
    }
  };
  const uint64_t per = (uint64_t)1 << 22;
  const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
  const uint32_t nt = (uint32_t)std::min<uint64_t>(std::min(hw, 16u), (cnt + per - 1) / per);
  if (nt <= 1) {
    part(0, cnt);
    return;
  }
  std::vector<std::thread> th;
  for (uint32_t t = 0; t < nt; ++t)
    th.emplace_back(part, cnt * t / nt, cnt * (t + 1) / nt);
  for (auto &x : th) x.join();
}

void fetch(sj_index &ix, uint64_t first, uint64_t max_pairs, uint32_t *oi, uint32_t *oj,
           float *od, uint64_t *n_written, hipStream_t s) {
  if (!ix.ran) fail(SJ_ERR_STATE, "fetch before a successful run");
  if (first > ix.total) fail(SJ_ERR_RANGE, "first is beyond the result");
  const uint64_t cnt = std::min(max_pairs, ix.total - first);
  const sj_index &E = entries_of(ix);  // the j column's points
  const bool dev_i = !oi || is_device_pointer(oi);
  const bool dev_j = !oj || is_device_pointer(oj);
  const bool dev_d = !od || is_device_pointer(od);
  const bool all_dev = dev_i && dev_j && dev_d;
  if (ix.on_host && !od && (!oi || !dev_i) && (!oj || !dev_j)) {
    // host result into host columns: split the keys on host threads
    fetch_host_split(ix, first, cnt, oi, oj);
    *n_written = cnt;
    return;
  }
  const uint64_t chunk = 1ull << 24;
  DevBuf keys_stage, si, sj2, sd;
  uint64_t done = 0;
  while (done < cnt) {
    const uint64_t c = std::min(chunk, cnt - done);
    const uint64_t g = first + done;  // global index of the chunk's first pair
    const uint64_t *src = stage_keys(ix, g, c, keys_stage, s);
    if (all_dev) {
      launch_unpack(src, c, oi ? oi + done : nullptr, oj ? oj + done : nullptr,
                    od ? od + done : nullptr, ix.X.as<float>(), ix.pos_of.as<uint32_t>(),
                    E.X.as<float>(), E.pos_of.as<uint32_t>(), ix.inv_perm_d.as<uint16_t>(), ix.d,
                    ix.dp, s);
    } else {
      si.ensure(c * 4);
      sj2.ensure(c * 4);
      sd.ensure(c * 4);
      launch_unpack(src, c, oi ? si.as<uint32_t>() : nullptr, oj ? sj2.as<uint32_t>() : nullptr,
                    od ? sd.as<float>() : nullptr, ix.X.as<float>(), ix.pos_of.as<uint32_t>(),
                    E.X.as<float>(), E.pos_of.as<uint32_t>(), ix.inv_perm_d.as<uint16_t>(), ix.d,
                    ix.dp, s);
      if (oi) SJ_HIP(hipMemcpyAsync(oi + done, si.p, c * 4, hipMemcpyDefault, s));
      if (oj) SJ_HIP(hipMemcpyAsync(oj + done, sj2.p, c * 4, hipMemcpyDefault, s));
      if (od) SJ_HIP(hipMemcpyAsync(od + done, sd.p, c * 4, hipMemcpyDefault, s));
    }
    SJ_HIP(hipStreamSynchronize(s));
    done += c;
  }
  SJ_HIP(hipStreamSynchronize(s));
  *n_written = cnt;
}

int debug_box_mode() {
  const char *v = std::getenv("SJ_DEBUG_BOX");
  return v && (v[0] == '0' || v[0] == '1') ? v[0] - '0' : -1;
}

int debug_hits_mode() {
  const char *v = std::getenv("SJ_DEBUG_HITS");
  return v && (v[0] == '0' || v[0] == '1') ? v[0] - '0' : -1;
}

bool debug_undersize() {
  const char *v = std::getenv("SJ_DEBUG_UNDERSIZE");
  return v && v[0] == '1';
}

sj_options checked_options(const float *points, uint64_t n, uint32_t d, double epsilon,
                           const sj_options *opts) {
  if (d == 0 || d > SJ_MAX_DIM)
    fail(SJ_ERR_INVALID_ARG, "d must be in [1, " + std::to_string(SJ_MAX_DIM) + "]");
  if (n > 0xffffffffull) fail(SJ_ERR_INVALID_ARG, "n must be below 2^32");
  if (n > 0 && !points) fail(SJ_ERR_INVALID_ARG, "points is NULL");
  if (!std::isfinite(epsilon) || !(epsilon > 0.0))
    fail(SJ_ERR_INVALID_ARG, "epsilon must be finite and > 0");
  if (!std::isfinite(epsilon * epsilon)) fail(SJ_ERR_INVALID_ARG, "epsilon^2 overflows");
  sj_options o;
  fill_defaults(&o);
  if (opts) {
    if (opts->struct_size < offsetof(sj_options, autotune) || opts->struct_size > sizeof(o))
      fail(SJ_ERR_INVALID_ARG, "sj_options.struct_size is not a known size");
    std::memcpy(&o, opts, opts->struct_size);
    o.struct_size = sizeof(o);
  }
  if (o.precision > SJ_PREC_BF16) fail(SJ_ERR_INVALID_ARG, "unknown precision");
  if (o.fp32_form > SJ_FP32_NORM) fail(SJ_ERR_INVALID_ARG, "unknown fp32_form");
  if (o.sortidu > 1) fail(SJ_ERR_INVALID_ARG, "sj_options.sortidu must be 0 or 1");
  if (o.k < 0) fail(SJ_ERR_INVALID_ARG, "k must be >= 0");
  return o;
}

}  // namespace sj

extern "C" {

void selfjoin_default_options(sj_options *opts) {
  if (opts) sj::fill_defaults(opts);
}

int selfjoin_build_index(const float *points, uint64_t n, uint32_t d, double epsilon,
                         const sj_options *opts, void *stream, sj_index **out) {
  return sj::guarded([&] {
    if (!out) fail(SJ_ERR_INVALID_ARG, "out is NULL");
    const sj_options o = sj::checked_options(points, n, d, epsilon, opts);
    const double eps2 = epsilon * epsilon;
    std::unique_ptr<sj_index> ix(new sj_index());
    SJ_HIP(hipGetDevice(&ix->device));
    ix->n = n;
    ix->d = d;
    ix->eps = epsilon;
    ix->eps2 = eps2;
    ix->opt = o;
    ix->info.struct_size = sizeof(sj_info);
    sj::build(*ix, points, static_cast<hipStream_t>(stream));
    *out = ix.release();
  });
}

int selfjoin_build_query(const sj_index *entries, const float *queries, uint64_t m,
                         void *stream, sj_index **out) {
  return sj::guarded([&] {
    if (!out || !entries) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (entries->entries) fail(SJ_ERR_INVALID_ARG, "entries is itself a query handle");
    if (m > 0xffffffffull) fail(SJ_ERR_INVALID_ARG, "m must be below 2^32");
    if (m > 0 && !queries) fail(SJ_ERR_INVALID_ARG, "queries is NULL");
    int dev = 0;
    SJ_HIP(hipGetDevice(&dev));
    if (dev != entries->device)
      fail(SJ_ERR_INVALID_ARG, "the current device is not the device of entries");
    std::unique_ptr<sj_index> q(new sj_index());
    q->device = dev;
    q->n = m;
    q->info.struct_size = sizeof(sj_info);
    sj::build_query(*q, *entries, queries, static_cast<hipStream_t>(stream));
    const_cast<sj_index *>(entries)->refs.fetch_add(1);  // kept until the query handle goes
    *out = q.release();
  });
}

int selfjoin_run(sj_index *idx, void *stream, uint64_t *total_pairs) {
  return sj::guarded([&] {
    if (!idx || !total_pairs) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (!idx->ran) sj::run(*idx, static_cast<hipStream_t>(stream));
    *total_pairs = idx->total;
  });
}

int selfjoin_fetch_pairs(sj_index *idx, uint64_t first, uint64_t max_pairs, uint32_t *out_i,
                         uint32_t *out_j, float *out_dist, uint64_t *n_written, void *stream) {
  return sj::guarded([&] {
    if (!idx || !n_written) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    sj::fetch(*idx, first, max_pairs, out_i, out_j, out_dist, n_written,
              static_cast<hipStream_t>(stream));
  });
}

int selfjoin_fetch_offsets(sj_index *idx, uint64_t *offsets, void *stream) {
  return sj::guarded([&] {
    if (!idx || !offsets) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    sj::fetch_offsets(*idx, offsets, static_cast<hipStream_t>(stream));
  });
}

int selfjoin_get_info(const sj_index *idx, sj_info *info) {
  return sj::guarded([&] {
    if (!idx || !info) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (info->struct_size < sizeof(uint32_t) || info->struct_size > sizeof(sj_info))
      fail(SJ_ERR_INVALID_ARG, "sj_info.struct_size is not a known size");
    sj_info x = idx->info;
    x.struct_size = info->struct_size;
    x.d = idx->d;
    x.n = idx->n;
    x.epsilon = idx->eps;
    x.k = idx->k;
    x.precision = idx->prec;
    x.n_cells = idx->ncell;
    x.candidates = idx->candidates;
    if (!idx->ran) x.evaluated = idx->evaluated_sym;
    std::memcpy(info, &x, info->struct_size);
  });
}

int selfjoin_get_perm(const sj_index *idx, uint32_t *perm, uint32_t cap) {
  return sj::guarded([&] {
    if (!idx || (!perm && cap)) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    for (uint32_t r = 0; r < std::min<uint32_t>(cap, idx->d); ++r) perm[r] = idx->perm[r];
  });
}

void selfjoin_free(sj_index *idx) {
  // a handle goes when the caller has freed it and no query handle still
  // reads it; freeing a query handle releases its entries' reference
  while (idx && idx->refs.fetch_sub(1) == 1) {
    sj_index *e = const_cast<sj_index *>(idx->entries);
    delete idx;
    idx = e;
  }
}

int selfjoin_release_cache(uint64_t *released) {
  return sj::guarded([&] {
    int dev = 0;
    SJ_HIP(hipGetDevice(&dev));
    thread_scratch().trim();
    const size_t b = dev_cached_bytes(dev) + host_cached_bytes();
    dev_cache_release(dev);
    host_cache_release();
    if (released) *released = b;
  });
}

const char *selfjoin_last_error(void) { return sj::g_last_error.c_str(); }

}  // extern "C"
