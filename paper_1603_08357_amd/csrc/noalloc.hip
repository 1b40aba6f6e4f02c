// Sequential cluster ids without a caller workspace and without any device
// allocation: ccl_cluster_ids_noalloc.  For callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The workspace of ccl_cluster_ids -- one int32 per 4096 sites,
// the per-span minimum counts and then their exclusive scan -- lives in the
// file-scope device array `scratch` instead, sized for the largest valid
// input (INT32_MAX sites: 524288 words, 2 MiB per device, held until the
// process ends).  Every word of it that a call reads is written earlier in
// the same call (the span-count kernel writes one word per span before the
// scan reads it), so nothing needs clearing between calls; calls that
// overlap on one device share the array and race.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace ccl {

constexpr int64_t kNoAllocMaxSites = INT32_MAX;
constexpr int64_t kNoAllocScratchWords = (kNoAllocMaxSites + 4095) / 4096;

static __device__ __align__(256) int32_t scratch[kNoAllocScratchWords];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: the device address of `scratch`
}  // namespace

// The device address of this device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's own name is
// only a stand-in for the symbol, never a device address.
static ccl_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e);
    if (p == nullptr) return CCL_ERR_HIP;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return CCL_OK;
}

}  // namespace ccl

using namespace ccl;

extern "C" {

size_t ccl_cluster_ids_noalloc_max_sites(void) { return (size_t)kNoAllocMaxSites; }

ccl_status ccl_cluster_ids_noalloc(int64_t n_sites, const int32_t* labels, int32_t* ids_out,
                                   int32_t* n_clusters_out, void* stream) {
  if (n_sites < 0) return CCL_ERR_INVALID_VALUE;
  if (n_sites > kNoAllocMaxSites) return CCL_ERR_TOO_LARGE;
  if (n_sites == 0) return CCL_OK;
  const size_t lb = (size_t)n_sites * 4;
  if (!labels || !ids_out || !n_clusters_out) return CCL_ERR_INVALID_VALUE;
  if (overlaps(labels, lb, ids_out, lb) || overlaps(n_clusters_out, 4, labels, lb) ||
      overlaps(n_clusters_out, 4, ids_out, lb))
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  void* ws = nullptr;
  const ccl_status st = scratch_address(d->device, &ws);
  if (st != CCL_OK) return st;
  if (cluster_ids_workspace_bytes(n_sites) > sizeof(scratch)) return CCL_ERR_TOO_LARGE;
  const NoTraceScope quiet;  // kernel timing would create HIP events
  return launch_cluster_ids(n_sites, labels, ids_out, n_clusters_out, ws, (hipStream_t)stream, *d);
}

}  // extern "C"
