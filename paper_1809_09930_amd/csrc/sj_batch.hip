// Many independent self-joins in one persistent launch under a hipGraph.
//
// Every job gets its own grid index and matrix-core operands (the same
// build as a single join).  The distance filtering of all jobs then runs as
// ONE persistent kernel over a shared queue of work units; together with
// the mapping of positions to caller indices, one radix sort of all jobs'
// keys (job << 40 | i << 20 | j) and the per-job result bounds it is
// captured once into a hipGraph and replayed.  Output buffers are sized
// beforehand from each job's sampled count; a replay that would overflow
// is detected on the device and answered with a larger buffer and a new
// capture.
//
// An autotuner picks the length of the work units' candidate stretches
// (tile shape) and the number of work units a wave takes from the queue at
// once (queue granularity) by timing the persistent kernel on the batch
// itself; k is chosen per job by the index build's cost model.  Choices are
// cached per batch signature in the process and, when SJ_TUNE_CACHE names a
// file, on disk.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <exception>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "sj_runtime.hpp"



using namespace sj;

struct sj_batch {
  std::vector<std::unique_ptr<sj_index>> jobs;
  std::vector<uint64_t> est;
  sj::DevBuf jobs_d;     // BatchJob[njobs]
  sj::DevBuf wus;        // all jobs' work units
  uint64_t n_wu = 0;
  sj::DevBuf keys[2], radix_tmp;
  sj::DevBuf ctl;        // [0] cursor, [1] rechecks, [2] capacity, [3] queue (u32 in the low half),
                         // [4] band-list cursor
  sj::DevBuf band;       // deferred recheck list
  uint64_t band_cap = 0;
  sj::DevBuf first, last;  // per-job bounds in the sorted keys
  uint64_t capacity = 0;
  uint32_t tc = 4096, grab = 1;
  uint32_t grid = 0;
  int dev = 0;  // device of the batch (and of its build pool)
  int job_bits = 1;
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> h_first, h_last;
  uint64_t total = 0, rechecks = 0;
  sj_batch_info info{};
  ~sj_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

namespace sj {
namespace {

constexpr uint32_t kMaxBatchN = (1u << 20) - 1;  // positions fit 20 bits
#ifndef SJ_BUILD_THREADS
#define SJ_BUILD_THREADS 12
#endif
constexpr uint32_t kBuildThreads = SJ_BUILD_THREADS;  // host threads building job indexes
constexpr size_t kBuildScratchKeep = (size_t)256 << 20;  // scratch a build thread keeps

// Host threads that build the jobs' indexes, one pool per device for the
// life of the process.  Each thread owns a non-blocking stream on that
// device, created once, and keeps its scratch chunks while a task runs; a
// task hands out job indices through an atomic counter, and run() returns
// when every job is done and every thread's stream has drained.  No thread
// or stream is created or destroyed per call.
class BuildPool {
 public:
  explicit BuildPool(int dev) : dev_(dev) {
    const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
    const uint32_t n = std::max(1u, std::min(hw, kBuildThreads));
    for (uint32_t w = 0; w < n; ++w) threads_.emplace_back([this] { loop(); });
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [this] { return ready_ == threads_.size(); });
  }
  // the pool lives until the process ends (threads wait on a condition
  // variable, with no device work, when it does)
  ~BuildPool() = delete;

  // Runs fn(job, stream) for job = 0 .. njobs - 1 on the pool's threads.
  void run(uint32_t njobs, const std::function<void(uint32_t, hipStream_t)> &fn) {
    std::lock_guard<std::mutex> one(run_mu_);  // one task at a time per pool
    std::unique_lock<std::mutex> lk(mu_);
    // threads without a stream take no jobs; the others take them all
    if (working_ == 0) fail(SJ_ERR_DEVICE, "no build thread could create its stream");
    fn_ = &fn;
    njobs_ = njobs;
    next_.store(0);
    busy_ = threads_.size();
    ++gen_;
    cv_work_.notify_all();
    cv_done_.wait(lk, [this] { return busy_ == 0; });
    fn_ = nullptr;
  }

 private:
  void loop() {
    hipStream_t st = nullptr;
    bool ok = hipSetDevice(dev_) == hipSuccess &&
              hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    uint64_t seen = 0;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (ok) ++working_;
      ++ready_;
      cv_done_.notify_all();
    }
    for (;;) {
      const std::function<void(uint32_t, hipStream_t)> *fn = nullptr;
      uint32_t njobs = 0;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_work_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        fn = fn_;
        njobs = njobs_;
      }
      if (ok) {
        Scratch &scr = thread_scratch();
        scr.keep_bytes = kBuildScratchKeep;  // reuse chunks from one job to the next
        for (uint32_t j = next_.fetch_add(1); j < njobs; j = next_.fetch_add(1)) (*fn)(j, st);
        (void)hipStreamSynchronize(st);
        scr.keep_bytes = 0;
        scr.trim();
      }
      std::lock_guard<std::mutex> lk(mu_);
      if (--busy_ == 0) cv_done_.notify_all();
    }
  }

  int dev_;
  std::vector<std::thread> threads_;
  std::mutex mu_, run_mu_;
  std::condition_variable cv_work_, cv_done_;
  const std::function<void(uint32_t, hipStream_t)> *fn_ = nullptr;
  uint32_t njobs_ = 0;
  std::atomic<uint32_t> next_{0};
  size_t busy_ = 0, ready_ = 0, working_ = 0;
  uint64_t gen_ = 0;
};

BuildPool &build_pool(int dev) {
  static std::mutex mu;
  static std::map<int, BuildPool *> pools;  // never freed (see ~BuildPool)
  std::lock_guard<std::mutex> lk(mu);
  auto it = pools.find(dev);
  if (it == pools.end()) it = pools.emplace(dev, new BuildPool(dev)).first;
  return *it->second;
}

__global__ void k_tag_wus(WorkUnit *__restrict__ wu, uint64_t count, uint32_t job) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) wu[i].pad = job;
}

std::mutex g_tune_mu;
std::map<std::string, std::pair<uint32_t, uint32_t>> g_tune_cache;

std::string batch_signature(const sj_batch &b) {
  // jobs bucketed by (d, log2 n, precision)
  std::map<std::string, int> h;
  for (const auto &ix : b.jobs) {
    int lg = 0;
    while ((1ull << (lg + 1)) <= ix->n) ++lg;
    h["d" + std::to_string(ix->d) + "n" + std::to_string(lg) + "p" + std::to_string(ix->prec)]++;
  }
  std::ostringstream os;
  for (auto &kv : h) os << kv.first << "x" << kv.second << ";";
  return os.str();
}

void tune_cache_load() {
  const char *path = std::getenv("SJ_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string sig;
  uint32_t tc, grab;
  while (f >> sig >> tc >> grab) g_tune_cache[sig] = {tc, grab};
}

void tune_cache_store(const std::string &sig, uint32_t tc, uint32_t grab) {
  g_tune_cache[sig] = {tc, grab};
  const char *path = std::getenv("SJ_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << sig << " " << tc << " " << grab << "\n";
}

// Concatenated work units of all jobs with candidate stretches of length tc,
// biggest jobs first (longest-processing-time order for the shared queue).
// Each job's units are cut on the build pool (a chain of short launches and
// read-backs per job, several in flight), then copied into one queue on s.
void make_queue(sj_batch &b, uint32_t tc, hipStream_t s) {
  const size_t nj = b.jobs.size();
  std::vector<DevBuf> per(nj);
  std::vector<uint64_t> cnt(nj), ev(nj);
  std::vector<std::exception_ptr> err(nj);
  build_pool(b.dev).run((uint32_t)nj, [&](uint32_t j, hipStream_t ws) {
    try {
      sj_index &ix = *b.jobs[j];
      if (ix.n == 0) return;
      // returns after its stream has drained: per[j] is complete
      cnt[j] = build_workunits(ix, 1, nullptr, 0, ix.run_off_sym, ix.runs_sym, ix.tq_m, tc,
                               per[j], &ev[j], ws);
    } catch (...) {
      err[j] = std::current_exception();
    }
  });
  for (size_t j = 0; j < nj; ++j)
    if (err[j]) std::rethrow_exception(err[j]);
  std::vector<size_t> order(nj);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return ev[a] > ev[c]; });
  uint64_t total = 0;
  for (size_t j = 0; j < nj; ++j) total += cnt[j];
  b.wus.alloc(std::max<uint64_t>(total, 1) * sizeof(WorkUnit));
  uint64_t off = 0;
  for (size_t j : order) {
    if (!cnt[j]) continue;
    WorkUnit *dst = b.wus.as<WorkUnit>() + off;
    SJ_HIP(hipMemcpyAsync(dst, per[j].p, cnt[j] * sizeof(WorkUnit), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_tag_wus, dim3((uint32_t)((cnt[j] + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, dst, cnt[j], (uint32_t)j);
    SJ_HIP(hipGetLastError());
    off += cnt[j];
  }
  SJ_HIP(hipStreamSynchronize(s));
  b.n_wu = total;
  b.tc = tc;
}

unsigned long long *ctl_ptr(sj_batch &b, int i) { return b.ctl.as<unsigned long long>() + i; }

void alloc_outputs(sj_batch &b, uint64_t cap, hipStream_t s) {
  b.capacity = cap;
  b.keys[0].alloc(cap * 8);
  b.keys[1].alloc(cap * 8);
  b.radix_tmp.alloc(radix_tmp_bytes(cap));
  const unsigned long long c = cap;
  SJ_HIP(hipMemcpyAsync(ctl_ptr(b, 2), &c, 8, hipMemcpyHostToDevice, s));
  SJ_HIP(hipStreamSynchronize(s));
}

// The captured sequence: reset, persistent join, ids, sort, bounds.
void record(sj_batch &b, hipStream_t s) {
  const size_t nj = b.jobs.size();
  launch_fill_u64(ctl_ptr(b, 0), 2, 0ull, s);  // cursor, rechecks
  launch_fill_u64(ctl_ptr(b, 3), 2, 0ull, s);  // queue, band-list cursor
  launch_fill_u64(b.first.as<unsigned long long>(), nj, 0ull, s);
  launch_fill_u64(b.last.as<unsigned long long>(), nj, 0ull, s);
  launch_join_batched(b.jobs_d.as<BatchJob>(), b.wus.as<WorkUnit>(), b.n_wu, b.grab,
                      reinterpret_cast<unsigned int *>(ctl_ptr(b, 3)), b.keys[0].as<uint64_t>(),
                      ctl_ptr(b, 2), ctl_ptr(b, 0), ctl_ptr(b, 1), b.grid,
                      b.band.as<uint64_t>(), b.band_cap, ctl_ptr(b, 4), s);
  launch_band_recheck_batched(b.jobs_d.as<BatchJob>(), b.band.as<uint64_t>(), ctl_ptr(b, 4),
                              b.band_cap, b.keys[0].as<uint64_t>(), ctl_ptr(b, 2), ctl_ptr(b, 0),
                              ctl_ptr(b, 1), b.grid, s);
  const uint32_t g = (uint32_t)std::min<uint64_t>((b.capacity + kBlock - 1) / kBlock, 16384);
  launch_pos_to_id_batched(b.keys[0].as<uint64_t>(), ctl_ptr(b, 0), ctl_ptr(b, 2),
                           b.jobs_d.as<BatchJob>(), g, s);
  std::vector<int> shifts;
  for (int bit = 0; bit < 40 + b.job_bits; bit += 8) shifts.push_back(bit);
  uint64_t *kb[2] = {b.keys[0].as<uint64_t>(), b.keys[1].as<uint64_t>()};
  radix_sort_u64(kb, nullptr, b.capacity, shifts.data(), (int)shifts.size(), b.radix_tmp.p, s,
                 ctl_ptr(b, 0));
  launch_job_bounds(b.keys[0].as<uint64_t>(), ctl_ptr(b, 0), ctl_ptr(b, 2),
                    b.first.as<unsigned long long>(), b.last.as<unsigned long long>(), g, s);
}

void capture(sj_batch &b) {
  if (b.exec) SJ_HIP(hipGraphExecDestroy(b.exec));
  if (b.graph) SJ_HIP(hipGraphDestroy(b.graph));
  b.exec = nullptr;
  b.graph = nullptr;
  SJ_HIP(hipStreamBeginCapture(b.cs, hipStreamCaptureModeThreadLocal));
  try {
    record(b, b.cs);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b.cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  SJ_HIP(hipStreamEndCapture(b.cs, &b.graph));
  SJ_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
}

float replay(sj_batch &b) {
  Event e0, e1;
  SJ_HIP(hipEventRecord(e0.e, b.cs));
  SJ_HIP(hipGraphLaunch(b.exec, b.cs));
  SJ_HIP(hipEventRecord(e1.e, b.cs));
  SJ_HIP(hipEventSynchronize(e1.e));
  return elapsed_ms(e0, e1);
}

uint64_t read_ctl(sj_batch &b, int i) {
  unsigned long long v = 0;
  SJ_HIP(hipMemcpyAsync(&v, ctl_ptr(b, i), 8, hipMemcpyDeviceToHost, b.cs));
  SJ_HIP(hipStreamSynchronize(b.cs));
  return v;
}

// Time one launch of the persistent join alone (results discarded).
float time_join(sj_batch &b) {
  launch_fill_u64(ctl_ptr(b, 0), 2, 0ull, b.cs);
  launch_fill_u64(ctl_ptr(b, 3), 2, 0ull, b.cs);
  Event e0, e1;
  SJ_HIP(hipEventRecord(e0.e, b.cs));
  launch_join_batched(b.jobs_d.as<BatchJob>(), b.wus.as<WorkUnit>(), b.n_wu, b.grab,
                      reinterpret_cast<unsigned int *>(ctl_ptr(b, 3)), b.keys[0].as<uint64_t>(),
                      ctl_ptr(b, 2), ctl_ptr(b, 0), ctl_ptr(b, 1), b.grid,
                      b.band.as<uint64_t>(), b.band_cap, ctl_ptr(b, 4), b.cs);
  launch_band_recheck_batched(b.jobs_d.as<BatchJob>(), b.band.as<uint64_t>(), ctl_ptr(b, 4),
                              b.band_cap, b.keys[0].as<uint64_t>(), ctl_ptr(b, 2), ctl_ptr(b, 0),
                              ctl_ptr(b, 1), b.grid, b.cs);
  SJ_HIP(hipEventRecord(e1.e, b.cs));
  SJ_HIP(hipEventSynchronize(e1.e));
  return elapsed_ms(e0, e1);
}

// The stretch and grab the tuner chose before for a batch of this signature.
bool tune_cache_lookup(const sj_batch &b, uint32_t *tc, uint32_t *grab) {
  const std::string sig = batch_signature(b);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune_cache.empty()) tune_cache_load();
  auto it = g_tune_cache.find(sig);
  if (it == g_tune_cache.end()) return false;
  *tc = it->second.first;
  *grab = it->second.second;
  return true;
}

void autotune(sj_batch &b) {
  const std::string sig = batch_signature(b);
  uint32_t tc_known = 0, grab_known = 0;
  if (tune_cache_lookup(b, &tc_known, &grab_known)) {
    if (b.tc != tc_known) make_queue(b, tc_known, b.cs);
    b.grab = grab_known;
    b.info.tuned = 2;
    return;
  }
  const uint32_t tcs[] = {1024, 4096, 16384};
  const uint32_t grabs[] = {1, 4};
  float best = 0.0f;
  uint32_t best_tc = b.tc, best_grab = b.grab;
  bool have = false;
  for (uint32_t tc : tcs) {
    make_queue(b, tc, b.cs);
    for (uint32_t g : grabs) {
      b.grab = g;
      const float ms = time_join(b);
      if (!have || ms < best) {
        best = ms;
        best_tc = tc;
        best_grab = g;
        have = true;
      }
    }
  }
  if (b.tc != best_tc) make_queue(b, best_tc, b.cs);
  b.grab = best_grab;
  b.info.tuned = 1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache_store(sig, best_tc, best_grab);
}

void run_batch(sj_batch &b, const sj_job *jobs, uint32_t njobs, const sj_options *opts,
               hipStream_t user) {
  SJ_HIP(hipStreamSynchronize(user));
  SJ_HIP(hipStreamCreateWithFlags(&b.cs, hipStreamNonBlocking));
  int dev = 0;
  SJ_HIP(hipGetDevice(&dev));
  b.dev = dev;
  auto t0 = std::chrono::steady_clock::now();
  b.jobs.resize(njobs);
  b.est.assign(njobs, 0);
  uint32_t autotune_on = opts && opts->struct_size >= offsetof(sj_options, mem_budget)
                             ? opts->autotune
                             : 0u;
  // validate every job first (host only), then build the jobs' indexes and
  // sampled counts on a few host threads, each with its own stream: the
  // build of one small job is a chain of short launches and read-backs, so
  // several chains in flight keep the GPU busy
  std::vector<sj_options> jopt(njobs);
  for (uint32_t j = 0; j < njobs; ++j) {
    const sj_job &jb = jobs[j];
    if (jb.n > kMaxBatchN)
      fail(SJ_ERR_INVALID_ARG, "batched jobs hold at most 2^20 - 1 points (job " +
                                   std::to_string(j) + ")");
    jopt[j] = checked_options(jb.points, jb.n, jb.d, jb.epsilon, opts);
    if (jopt[j].precision == SJ_PREC_FP32) jopt[j].precision = SJ_PREC_FP16;  // matrix cores only
  }
  std::vector<std::exception_ptr> err(njobs);
  std::vector<float> ms_est(njobs, 0.0f);
  std::atomic<bool> stop{false};
  auto build_job = [&](uint32_t j, hipStream_t ws) {
      if (stop) return;
      try {
        const sj_job &jb = jobs[j];
        std::unique_ptr<sj_index> ix(new sj_index());
        ix->device = dev;
        ix->n = jb.n;
        ix->d = jb.d;
        ix->eps = jb.epsilon;
        ix->eps2 = jb.epsilon * jb.epsilon;
        ix->opt = jopt[j];
        ix->info.struct_size = sizeof(sj_info);
        ix->batch_job = true;
        build(*ix, jb.points, ws);
        if (ix->n && batched_variant(ix->kp, ix->fmt) < 0)
          fail(SJ_ERR_INVALID_ARG,
               "batched jobs support d up to 77 (job " + std::to_string(j) + ")");
        if (ix->n) b.est[j] = estimate_pairs(*ix, ws, &ms_est[j]);
        b.jobs[j] = std::move(ix);
      } catch (...) {
        err[j] = std::current_exception();
        stop = true;
      }
  };
  build_pool(dev).run(njobs, build_job);
  for (uint32_t j = 0; j < njobs; ++j)
    if (err[j]) std::rethrow_exception(err[j]);
  for (uint32_t j = 0; j < njobs; ++j) {
    b.info.ms_build += b.jobs[j]->info.ms_build;
    b.info.ms_estimate += ms_est[j];
  }
  auto t1 = std::chrono::steady_clock::now();
  // pre-size the shared output from every job's sampled count
  uint64_t cap = 1u << 20;
  for (uint32_t j = 0; j < njobs; ++j) cap += b.est[j] + b.est[j] / 8;
  // the band list from the jobs' sampled band counts
  uint64_t band_cap = 1u << 16;
  for (uint32_t j = 0; j < njobs; ++j)
    if (b.jobs[j]->n) band_cap += b.jobs[j]->band_hint;
  if (debug_undersize()) band_cap = 16;
  b.band_cap = band_cap;
  b.band.alloc(band_cap * 8);
  // job table
  std::vector<BatchJob> table(njobs);
  for (uint32_t j = 0; j < njobs; ++j) {
    sj_index &ix = *b.jobs[j];
    BatchJob bj{};
    if (ix.n) {
      bj.view = mfma_view(ix, ix.runs_sym.as<uint2>(), nullptr, 1);
      bj.view.pshift = 20;
      bj.orig_id = ix.orig_id.as<uint32_t>();
      bj.variant = batched_variant(ix.kp, ix.fmt);
    } else {
      bj.variant = -1;
    }
    table[j] = bj;
  }
  b.jobs_d.alloc(njobs * sizeof(BatchJob));
  SJ_HIP(hipMemcpyAsync(b.jobs_d.p, table.data(), njobs * sizeof(BatchJob), hipMemcpyHostToDevice,
                        b.cs));
  b.first.alloc(njobs * 8);
  b.last.alloc(njobs * 8);
  b.ctl.alloc(64);
  b.job_bits = 1;
  while ((1u << b.job_bits) < njobs) ++b.job_bits;
  hipDeviceProp_t prop;
  SJ_HIP(hipGetDeviceProperties(&prop, dev));
  b.grid = (uint32_t)(prop.multiProcessorCount * batched_blocks_per_cu());
  // the queue is cut once at the stretch tuned before for batches of this
  // signature, else at 4096 (the tuner then cuts it again per candidate)
  uint32_t tc0 = 4096, grab0 = 1;
  if (!autotune_on || !tune_cache_lookup(b, &tc0, &grab0)) tc0 = 4096;
  make_queue(b, tc0, b.cs);
  if (debug_undersize()) cap = std::max<uint64_t>(64, cap / 64);
  alloc_outputs(b, cap, b.cs);
  auto t2 = std::chrono::steady_clock::now();
  if (autotune_on) autotune(b);
  auto t3 = std::chrono::steady_clock::now();
  for (int attempt = 0; attempt < 4; ++attempt) {
    capture(b);
    b.info.ms_graph = replay(b);
    const uint64_t nb = read_ctl(b, 4);
    if (nb > b.band_cap) {  // band list overflowed: exact size, capture again
      if (attempt == 3) fail(SJ_ERR_DEVICE, "batched band list size did not settle");
      b.band_cap = nb;
      b.band.alloc(nb * 8);
      continue;
    }
    const uint64_t got = read_ctl(b, 0);
    if (got <= b.capacity) {
      b.total = got;
      break;
    }
    if (attempt == 3) fail(SJ_ERR_DEVICE, "batched result count did not settle");
    alloc_outputs(b, got, b.cs);  // exact now
  }
  b.rechecks = read_ctl(b, 1);
  b.h_first.assign(njobs, 0);
  b.h_last.assign(njobs, 0);
  SJ_HIP(hipMemcpyAsync(b.h_first.data(), b.first.p, njobs * 8, hipMemcpyDeviceToHost, b.cs));
  SJ_HIP(hipMemcpyAsync(b.h_last.data(), b.last.p, njobs * 8, hipMemcpyDeviceToHost, b.cs));
  SJ_HIP(hipStreamSynchronize(b.cs));
  auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point c) {
    return (float)std::chrono::duration<double, std::milli>(c - a).count();
  };
  b.info.ms_host_build = ms(t0, t1);
  b.info.ms_host_prepare = ms(t1, t2);
  b.info.ms_tune = ms(t2, t3);
  b.info.njobs = njobs;
  b.info.n_wu = b.n_wu;
  b.info.tile_candidates = b.tc;
  b.info.queue_grab = b.grab;
  b.info.grid = b.grid;
  b.info.pairs = b.total;
  b.info.rechecks = b.rechecks;
  b.info.capacity = b.capacity;
  uint64_t cand = 0, ev = 0;
  for (auto &ix : b.jobs) {
    cand += ix->candidates;
    ev += ix->evaluated_sym_m;
  }
  b.info.candidates = cand;
  b.info.evaluated = ev;
}

}  // namespace
}  // namespace sj

extern "C" {

int selfjoin_run_batched(const sj_job *jobs, uint32_t njobs, const sj_options *opts, void *stream,
                         sj_batch **out) {
  return sj::guarded([&] {
    if (!out || (!jobs && njobs)) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (njobs == 0 || njobs > (1u << 16))
      fail(SJ_ERR_INVALID_ARG, "njobs must be in [1, 65536]");
    std::unique_ptr<sj_batch> b(new sj_batch());
    b->info.struct_size = sizeof(sj_batch_info);
    sj::run_batch(*b, jobs, njobs, opts, static_cast<hipStream_t>(stream));
    *out = b.release();
  });
}

int selfjoin_batch_replay(sj_batch *b, float *ms) {
  return sj::guarded([&] {
    if (!b || !b->exec) fail(SJ_ERR_INVALID_ARG, "NULL or empty batch");
    const float t = sj::replay(*b);
    if (sj::read_ctl(*b, 0) != b->total) fail(SJ_ERR_DEVICE, "replay changed the result count");
    b->info.ms_graph = t;
    if (ms) *ms = t;
  });
}

int selfjoin_batch_range(const sj_batch *b, uint32_t job, uint64_t *first, uint64_t *count) {
  return sj::guarded([&] {
    if (!b || !first || !count) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (job >= b->jobs.size()) fail(SJ_ERR_RANGE, "job index out of range");
    *first = b->h_first[job];
    *count = b->h_last[job] - b->h_first[job];
  });
}

int selfjoin_batch_fetch(sj_batch *b, uint32_t job, uint64_t first, uint64_t max_pairs,
                         uint32_t *out_i, uint32_t *out_j, float *out_dist, uint64_t *n_written,
                         void *stream) {
  return sj::guarded([&] {
    if (!b || !n_written) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (job >= b->jobs.size()) fail(SJ_ERR_RANGE, "job index out of range");
    const uint64_t cnt_job = b->h_last[job] - b->h_first[job];
    if (first > cnt_job) fail(SJ_ERR_RANGE, "first is beyond the job's result");
    const uint64_t cnt = std::min(max_pairs, cnt_job - first);
    hipStream_t s = static_cast<hipStream_t>(stream);
    sj_index &ix = *b->jobs[job];
    const uint64_t *src = b->keys[0].as<uint64_t>() + b->h_first[job] + first;
    const bool all_dev = (!out_i || sj::is_device_pointer(out_i)) &&
                         (!out_j || sj::is_device_pointer(out_j)) &&
                         (!out_dist || sj::is_device_pointer(out_dist));
    if (cnt) {
      if (all_dev) {
        sj::launch_unpack(src, cnt, out_i, out_j, out_dist, ix.X.as<float>(),
                          ix.pos_of.as<uint32_t>(), ix.X.as<float>(), ix.pos_of.as<uint32_t>(),
                          ix.inv_perm_d.as<uint16_t>(), ix.d, ix.dp, s, 20);
      } else {
        sj::DevBuf si, sjj, sd;
        si.alloc(cnt * 4);
        sjj.alloc(cnt * 4);
        sd.alloc(cnt * 4);
        sj::launch_unpack(src, cnt, out_i ? si.as<uint32_t>() : nullptr,
                          out_j ? sjj.as<uint32_t>() : nullptr, out_dist ? sd.as<float>() : nullptr,
                          ix.X.as<float>(), ix.pos_of.as<uint32_t>(), ix.X.as<float>(),
                          ix.pos_of.as<uint32_t>(), ix.inv_perm_d.as<uint16_t>(), ix.d, ix.dp, s,
                          20);
        if (out_i) SJ_HIP(hipMemcpyAsync(out_i, si.p, cnt * 4, hipMemcpyDefault, s));
        if (out_j) SJ_HIP(hipMemcpyAsync(out_j, sjj.p, cnt * 4, hipMemcpyDefault, s));
        if (out_dist) SJ_HIP(hipMemcpyAsync(out_dist, sd.p, cnt * 4, hipMemcpyDefault, s));
      }
      SJ_HIP(hipStreamSynchronize(s));
    }
    *n_written = cnt;
  });
}

int selfjoin_batch_get_info(const sj_batch *b, sj_batch_info *info) {
  return sj::guarded([&] {
    if (!b || !info) fail(SJ_ERR_INVALID_ARG, "NULL argument");
    if (info->struct_size < sizeof(uint32_t) || info->struct_size > sizeof(sj_batch_info))
      fail(SJ_ERR_INVALID_ARG, "sj_batch_info.struct_size is not a known size");
    sj_batch_info x = b->info;
    x.struct_size = info->struct_size;
    std::memcpy(info, &x, info->struct_size);
  });
}

void selfjoin_batch_free(sj_batch *b) { delete b; }

}  // extern "C"
