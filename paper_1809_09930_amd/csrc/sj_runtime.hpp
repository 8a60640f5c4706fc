// Host runtime shared by the translation units of libselfjoin: device and
// pinned buffers, events, the index handle and the build/run helpers.
#pragma once

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <utility>
#include <vector>

#include "sj_index.hpp"
#include "sj_internal.hpp"
#include "sj_mfma.hpp"

namespace sj {

extern thread_local std::string g_last_error;

// Device blocks of the library go through a per-device cache: a freed block
// is kept (after the device has finished all queued work, as hipFree would
// wait) and handed to the next request of a size it fits without wasting
// more than half of it.  Repeated joins then allocate nothing, and do not
// pay the driver's occasional long hipMalloc / hipFree of multi-GB blocks.
// The cache holds at most a quarter of the device's memory (SJ_CACHE_BYTES
// overrides; 0 turns caching off); a failed allocation empties the device's
// cache and tries once more.  dev_alloc returns the block's capacity in
// *got and its device in *dev.
// `idle`: the caller knows no queued work uses the block (no wait needed).
void *dev_alloc(size_t bytes, size_t *got, int *dev);
void dev_free(void *p, size_t got, int dev, bool idle = false);
// bytes held in the cache of device `dev` (idle, reusable by the library)
size_t dev_cached_bytes(int dev);
// frees every cached block of device `dev`
void dev_cache_release(int dev);

// Device allocation owned by a handle.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t got = 0;
  int dev = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) dev_free(p, got, dev);
    p = nullptr;
    bytes = 0;
    got = 0;
  }
  void alloc(size_t b) {
    reset();
    if (b == 0) b = 256;
    p = dev_alloc(b, &got, &dev);
    bytes = b;
  }
  // at least b bytes; a block that must grow gets a quarter more, so that
  // buffers reused across batches of varying size are seldom replaced (a
  // replacement waits for the device)
  void ensure(size_t b) {
    if (!p || b > got) alloc(b + b / 4);
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

// Per-thread scratch for the temporaries of one index build or sampled
// count.  Temporaries are bump-allocated from a few large chunks and all die
// together when the outermost ScratchScope of the thread ends; the code
// inside a scope synchronises every stream that used them before the scope
// ends.  This replaces dozens of allocate/free pairs per build (each free
// waits for the whole device) with a handful of chunk allocations, and with
// none at all on a thread that keeps its chunks between scopes.
class Scratch {
 public:
  void *take(size_t bytes);
  // end of the outermost scope: every temporary is dead; keep at most
  // `keep_bytes` of chunks for the next scope (free the rest)
  void release(bool error);
  // free every chunk (no scope open on this thread)
  void trim();
  size_t keep_bytes = 0;
  int depth = 0;
  ~Scratch();

 private:
  struct Chunk {
    void *p;
    size_t size;
    int dev;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, used_ = 0;
};

Scratch &thread_scratch();

struct ScratchScope {
  ScratchScope() { ++thread_scratch().depth; }
  ~ScratchScope();
  ScratchScope(const ScratchScope &) = delete;
  ScratchScope &operator=(const ScratchScope &) = delete;
  int uncaught = std::uncaught_exceptions();
};

// A temporary device buffer taken from the thread's scratch (no free).
struct TmpBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void alloc(size_t b) {
    p = thread_scratch().take(b);
    bytes = b;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

// Pinned host blocks go through a process-wide cache as device blocks do:
// a freed block (no device work may use it any more) is kept for the next
// request it fits, up to SJ_HOST_CACHE_BYTES bytes (default: an eighth of
// the host's memory, at most 64 GiB; 0 turns caching off).
void *host_alloc(size_t bytes, size_t *got);
void host_free(void *p, size_t got);
size_t host_cached_bytes();
void host_cache_release();

struct PinnedBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t got = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf &) = delete;
  PinnedBuf &operator=(const PinnedBuf &) = delete;
  PinnedBuf(PinnedBuf &&o) noexcept : p(o.p), bytes(o.bytes), got(o.got) {
    o.p = nullptr;
    o.bytes = 0;
    o.got = 0;
  }
  ~PinnedBuf() {
    if (p) host_free(p, got);
  }
  void alloc(size_t b) {
    if (p) host_free(p, got);
    p = nullptr;
    if (b == 0) b = 64;
    p = host_alloc(b, &got);
    bytes = b;
  }
};

struct Event {
  hipEvent_t e = nullptr;
  Event() { SJ_HIP(hipEventCreate(&e)); }
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
  Event(const Event &) = delete;
  Event &operator=(const Event &) = delete;
};

inline float elapsed_ms(const Event &a, const Event &b) {
  float ms = 0.0f;
  SJ_HIP(hipEventElapsedTime(&ms, a.e, b.e));
  return ms;
}

inline uint32_t bits_for(uint64_t v) {  // bits needed to represent v
  uint32_t b = 0;
  while (v) { ++b; v >>= 1; }
  return b;
}

// Radix digits over bits [0, lo_bits) and [32, 32 + hi_bits): each field in
// as few passes as 8-bit digits need, its bits spread evenly over them
// (21 bits: 7 + 7 + 7), so runs of equal digits are as long as possible.
inline void digit_plan(uint32_t lo_bits, uint32_t hi_bits, std::vector<int> &shifts,
                       std::vector<int> &widths) {
  shifts.clear();
  widths.clear();
  const uint32_t field[2] = {lo_bits, hi_bits}, base[2] = {0, 32};
  for (int f = 0; f < 2; ++f) {
    const uint32_t b = field[f];
    if (!b) continue;
    const uint32_t p = (b + 7) / 8;
    uint32_t at = base[f];
    for (uint32_t i = 0; i < p; ++i) {
      const uint32_t w = b / p + (i < b % p ? 1u : 0u);
      shifts.push_back((int)at);
      widths.push_back((int)w);
      at += w;
    }
  }
}

inline bool is_device_pointer(const void *ptr) {
  if (!ptr) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
#if HIP_VERSION_MAJOR >= 6
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
#else
  return attr.memoryType == hipMemoryTypeDevice;
#endif
}

// Grid geometry for one choice of k.
struct Geometry {
  uint32_t k = 0;
  KeyParams kp{};
  NbrParams np{};
  uint32_t key_bits = 0;   // bits of the sort key
  uint32_t fine_bits = 0;  // low bits of the sort key below the cell key
  uint32_t u_rank = 0;     // SORTIDU: reordered position of the dimension u
};

inline double gamma_n(double m, double u) { return m * u / (1.0 - m * u); }


}  // namespace sj

namespace sj {
// Groups of consecutive small cells that share one work unit (see
// build_cell_groups): n groups, group g holds the positions
// [start[g], start[g + 1]) and the candidate runs
// runs[run_off[g] .. run_off[g + 1]), the union of its cells' runs.
struct CellGroups {
  uint64_t n = 0;
  DevBuf start, run_off, runs;
};
}  // namespace sj

// The opaque handle of the C ABI.
struct sj_index {
  typedef sj::DevBuf DevBuf;
  typedef sj::PinnedBuf PinnedBuf;
  int device = 0;
  uint64_t n = 0;
  uint32_t d = 0, dp = 0, k = 0;
  double eps = 0.0, eps2 = 0.0;
  sj_options opt{};
  std::vector<uint32_t> perm;
  std::vector<uint16_t> inv_perm;
  std::vector<double> dmin, dmax, dmean;  // per caller dimension; dmean from the variance sample
  float lo32 = 0.0f, hi32 = 0.0f;

  // General join Q join_eps E (Section 3.1): a query handle holds the query
  // points Q (n = |Q|) in the grid of the indexed set `entries` (E, which
  // must outlive it); its X / orig_id / pos_of / cells / norm tables / 16-bit
  // query operands describe Q, and the candidates are E's.  Null in a
  // self-join (the handle is its own entries).
  const sj_index *entries = nullptr;
  std::atomic<uint32_t> refs{1};  // the caller's handle plus the query handles built on it
  bool batch_job = false;  // built for the batched path: no single-join work units
  bool small_cells = false;  // FP32 units of 64 queries (most lane work in small cells)
  uint64_t n_near = 0;    // points in cells (a query handle drops far queries)
  sj::Geometry geom{};    // grid of the build (k, key and neighbour parameters)
  std::vector<float> mfma_centre;  // matrix-core centring of the indexed set
  sj::MfmaBand mfma_band{};        // and its error-band constants
  DevBuf mfma_max;                 // its maxima (k_mfma_maxima) on the device

  // index
  DevBuf X, orig_id, pos_of, perm_d, inv_perm_d;
  DevBuf skey;  // SORTIDU: sorted keys (cell key << fine bits | quantised u), position order
  DevBuf cell_key, cell_start;
  uint64_t ncell = 0;
  DevBuf nbr_off, nbr_cell;
  uint64_t n_nbr = 0;
  DevBuf run_off_sym, runs_sym, run_off_full, runs_full;
  uint64_t n_runs_sym = 0, n_runs_full = 0;
  DevBuf wu;
  uint64_t n_wu = 0;
  DevBuf uruns, uruns_m;  // SORTIDU: per-query-block candidate ranges of wu / wu_m
  uint32_t tq = 256, tc = 16384;
  uint64_t candidates = 0, evaluated_sym = 0;
  DevBuf counters;  // [0] cursor, [1] rechecks

  // matrix-core path
  uint32_t prec = SJ_PREC_FP32;  // precision actually used
  int fmt = 0;
  uint32_t kp = 0;
  uint64_t n_pad = 0;
  DevBuf XA, XB, cn, thi, tlo;  // 16-bit operands, FP32 candidate norms, thresholds
  bool mfma_per_wave = false;   // matrix-core single join with per-wave units
  uint32_t tq_single = 0, tc_single = 0;  // its unit shape (queries, candidates)
  DevBuf band;                  // deferred recheck list of the matrix-core join
  uint64_t band_cap = 0;
  uint64_t band_hint = 0;       // its expected size from the sampled count
  double hit_density = 0.0;     // result + band pairs per evaluated pair of the sampled count
  bool norm_form = false;       // FP32 filter in norm form
  DevBuf norm_qa, norm_cr;      // its per-point tables
  DevBuf wu_m;
  uint64_t n_wu_m = 0, evaluated_sym_m = 0;
  sj::CellGroups groups;       // groups of small cells (n = 0: none built)
  bool wu_grouped = false;     // the FP32 units wu are cut from the groups
  uint32_t tq_m = 128, tc_m = 4096;

  // results
  bool ran = false;
  uint64_t total = 0;
  DevBuf pairs;                     // sorted keys when device-resident
  std::vector<PinnedBuf> host_res;  // sorted keys per batch when host-resident
  std::vector<uint64_t> host_cnt;
  bool on_host = false;
  DevBuf fetch_stage;

  sj_info info{};
};


namespace sj {

void fill_defaults(sj_options *o);
// Validates arguments and options of an index build (throws Error).
sj_options checked_options(const float *points, uint64_t n, uint32_t d, double epsilon,
                           const sj_options *opts);
void build(sj_index &ix, const float *points, hipStream_t s);
// Work units of the distance kernels over the runs (run_off, runs) of ix's
// cells, queries contiguous or from qlist; *eval receives the pairs they
// cover.  by_stretch orders them by stretch index; u_ranges (SORTIDU,
// contiguous queries) cuts them from per-block ranges stored there.
uint64_t build_workunits(sj_index &ix, int sym, const uint32_t *qlist, uint64_t nq,
                         const DevBuf &run_off, const DevBuf &runs, uint32_t tq, uint32_t tc,
                         DevBuf &out, uint64_t *eval, hipStream_t s, bool by_stretch = false,
                         DevBuf *u_ranges = nullptr, const CellGroups *groups = nullptr);
// Groups of consecutive non-empty cells of ix (symmetric runs) for units of
// up to max_q queries: a group takes the next cell while that cell lies in
// the same row of the last indexed dimension, at most two cells past the
// group's first, and the group stays within max_q points.  Its runs are the
// union of its cells' symmetric runs.
void build_cell_groups(sj_index &ix, uint32_t max_q, CellGroups &g, hipStream_t s);
// Builds the query handle q (opt, n set) of the points `queries` against
// the indexed set E (see sj_index::entries).
void build_query(sj_index &q, const sj_index &E, const float *queries, hipStream_t s);
// The indexed (candidate) side of a handle: its entries, or itself.
inline const sj_index &entries_of(const sj_index &ix) { return ix.entries ? *ix.entries : ix; }
uint64_t estimate_pairs(sj_index &ix, hipStream_t s, float *ms);
uint64_t default_budget();
MfmaView mfma_view(const sj_index &ix, const uint2 *runs, const uint32_t *qlist, int sym);
// Fault injection from the host: SJ_DEBUG_UNDERSIZE=1 makes the first
// result buffer of every run (and the first band list of the matrix-core
// join) far too small, so the device-side overflow detection and the
// resize-and-rerun paths are exercised.
bool debug_undersize();
// Test hook: SJ_DEBUG_HITS=0 or 1 forces the hit mode of the matrix-core
// single-join kernels (rare: per-tile minimum first; frequent: element scan)
// instead of the choice from the sampled count; -1 when unset.
int debug_hits_mode();
// Test hook: SJ_DEBUG_BOX=0 or 1 switches the query-box prefilter of the
// matrix-core workgroup kernel off or on (default: on up to 32 dimensions).
int debug_box_mode();

template <typename F>
int guarded(F &&f) {
  try {
    g_last_error.clear();
    f();
    return SJ_OK;
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SJ_ERR_OUT_OF_MEMORY;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return SJ_ERR_DEVICE;
  }
}

}  // namespace sj
