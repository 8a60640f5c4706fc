// CSR row starts of a result without any allocation.
//
// selfjoin_fetch_offsets_noalloc computes what selfjoin_fetch_offsets does
// (the same kernels: per-row pair counts, then an exclusive scan), but every
// temporary lives in one device array of fixed size defined below, so the
// call allocates nothing: no hipMalloc / hipFree, no pinned host memory, no
// library allocator.  It is meant for callers that cannot allocate (tight
// serving loops, harnesses that forbid allocation in the steady state).
//
// The array is file-scope device memory: each GPU the library runs on holds
// its own copy from module load until the process ends, at its own device
// address.  Host code never passes the symbol itself to a kernel (in host
// code it names a host-side stand-in); the device address is looked up once
// per device with hipGetSymbolAddress and kept in a per-device table.
//
// Layout of the array for one call (byte offsets, 256-aligned):
//   [0, 256)                       scan total (8 bytes used)
//   [256, 256 + S)                 scan partial sums, S = scan_tmp_bytes(n + 1)
//   next (n + 1) * 8 bytes         per-row counts (only when offsets is host memory;
//                                  device offsets are counted and scanned in place)
//   last kStageBytes               staging of the sorted keys when the result lives
//                                  in pinned host memory (batched runs)
// The entry point rejects a handle whose n does not fit this layout.
#include <mutex>

#include "sj_runtime.hpp"

namespace sj {
namespace {

constexpr size_t kNoAllocBytes = 64ull << 20;  // 64 MiB per device
constexpr size_t kStageBytes = 16ull << 20;    // 2^21 keys per staged chunk
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_noalloc_mu[kMaxDevices];  // one call at a time per device
void *g_noalloc_ptr[kMaxDevices] = {};  // device address of `scratch` per device

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Device address of this device's array; looked up on the first call on the
// device (the caller holds that device's lock, and the device is current).
unsigned char *scratch_ptr(int dev) {
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    SJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(SJ_ERR_DEVICE, "hipGetSymbolAddress returned no address");
    g_noalloc_ptr[dev] = p;
  }
  return static_cast<unsigned char *>(g_noalloc_ptr[dev]);
}

// Device pointer to sorted keys [g, g + c) (c <= kStageBytes / 8): the
// device-resident result, or a copy of the host batches into `stage`.
const uint64_t *keys_at(const sj_index &ix, uint64_t g, uint64_t c, uint64_t *stage,
                        hipStream_t s) {
  if (!ix.on_host) return ix.pairs.as<uint64_t>() + g;
  uint64_t off = 0, copied = 0, gg = g;
  for (size_t b = 0; b < ix.host_res.size() && copied < c; ++b) {
    const uint64_t bc = ix.host_cnt[b];
    if (gg >= off + bc) {
      off += bc;
      continue;
    }
    const uint64_t from = gg - off;
    const uint64_t take = std::min(bc - from, c - copied);
    SJ_HIP(hipMemcpyAsync(stage + copied, static_cast<const uint64_t *>(ix.host_res[b].p) + from,
                          take * 8, hipMemcpyHostToDevice, s));
    copied += take;
    gg += take;
    off += bc;
  }
  return stage;
}

void fetch_offsets_noalloc(const sj_index &ix, uint64_t *offsets, hipStream_t s) {
  if (!ix.ran) fail(SJ_ERR_STATE, "fetch before a successful run");
  int dev = 0;
  SJ_HIP(hipGetDevice(&dev));
  if (dev != ix.device) fail(SJ_ERR_INVALID_ARG, "the current device is not the handle's device");
  if (dev < 0 || dev >= kMaxDevices) fail(SJ_ERR_INVALID_ARG, "device ordinal out of range");
  const uint64_t n = ix.n;
  const bool dev_out = is_device_pointer(offsets);
  const size_t scan_b = align256(scan_tmp_bytes(n + 1));
  const size_t count_b = dev_out ? 0 : align256((n + 1) * 8);
  if (256 + scan_b + count_b + kStageBytes > kNoAllocBytes)
    fail(SJ_ERR_INVALID_ARG,
         "n is too large for the fixed scratch of selfjoin_fetch_offsets_noalloc; "
         "use selfjoin_fetch_offsets");

  std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
  unsigned char *base = scratch_ptr(dev);
  uint64_t *total_d = reinterpret_cast<uint64_t *>(base);
  void *scan_tmp = base + 256;
  uint64_t *counts =
      dev_out ? offsets : reinterpret_cast<uint64_t *>(base + 256 + scan_b);
  uint64_t *stage = reinterpret_cast<uint64_t *>(base + kNoAllocBytes - kStageBytes);

  // counts start at zero (a fill kernel, no memset node)
  launch_fill_u64(reinterpret_cast<unsigned long long *>(counts), n + 1, 0ull, s);
  const uint64_t total = ix.total;
  const uint64_t chunk = ix.on_host ? kStageBytes / 8 : std::max<uint64_t>(total, 1);
  for (uint64_t g = 0; g < total; g += chunk) {
    const uint64_t c = std::min(chunk, total - g);
    const uint64_t *src = keys_at(ix, g, c, stage, s);
    launch_row_counts(src, c, reinterpret_cast<unsigned long long *>(counts), s);
    if (ix.on_host) SJ_HIP(hipStreamSynchronize(s));  // the stage is reused by the next chunk
  }
  // in place when the output is on the device (the scan reads each tile
  // before writing it)
  exclusive_scan_u64(counts, dev_out ? offsets : counts, n + 1, total_d, scan_tmp, s);
  if (!dev_out) SJ_HIP(hipMemcpyAsync(offsets, counts, (n + 1) * 8, hipMemcpyDeviceToHost, s));
  SJ_HIP(hipStreamSynchronize(s));
}

}  // namespace
}  // namespace sj

extern "C" int selfjoin_fetch_offsets_noalloc(sj_index *idx, uint64_t *offsets, void *stream) {
  return sj::guarded([&] {
    if (!idx || !offsets) sj::fail(SJ_ERR_INVALID_ARG, "NULL argument");
    sj::fetch_offsets_noalloc(*idx, offsets, static_cast<hipStream_t>(stream));
  });
}
