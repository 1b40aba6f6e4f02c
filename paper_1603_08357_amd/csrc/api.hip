// C ABI of libccl.so: argument checks, dispatch, status strings, kernel
// timing.  Every check here runs on the host before any HIP call.
#include <string.h>

#include <mutex>
#include <vector>

#include <math.h>

#include "common.hpp"
#include "philox.hpp"

namespace ccl {

static thread_local int g_last_hip_error = 0;

ccl_status fail_hip(hipError_t e) {
  g_last_hip_error = (int)e;
  return e == hipErrorOutOfMemory ? CCL_ERR_OUT_OF_MEMORY : CCL_ERR_HIP;
}

// ---------------------------------------------------------------- devices

static std::mutex g_dev_mu;
static std::vector<DeviceInfo> g_devs;

const DeviceInfo* current_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    fail_hip(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_dev_mu);
  if ((int)g_devs.size() <= dev) g_devs.resize(dev + 1);
  DeviceInfo& d = g_devs[dev];
  if (d.device < 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
      fail_hip(e);
      return nullptr;
    }
    d.cu_count = prop.multiProcessorCount;
    d.max_lds_per_block = (int)prop.sharedMemPerBlock;
    d.is_gfx950 = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    d.device = dev;
  }
  return &d;
}

// ---------------------------------------------------------------- tracing

namespace {
constexpr int kMaxTrace = 65536;
struct TraceRec {
  const char* name;
  hipEvent_t start;
  hipEvent_t stop;
};
std::mutex g_tr_mu;
bool g_tr_on = false;
std::vector<TraceRec> g_tr;
std::vector<hipEvent_t> g_ev_pool;

hipEvent_t pool_event() {
  if (!g_ev_pool.empty()) {
    hipEvent_t e = g_ev_pool.back();
    g_ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void clear_records_locked() {
  for (auto& r : g_tr) {
    g_ev_pool.push_back(r.start);
    g_ev_pool.push_back(r.stop);
  }
  g_tr.clear();
}
}  // namespace

static thread_local int g_no_trace = 0;
NoTraceScope::NoTraceScope() { ++g_no_trace; }
NoTraceScope::~NoTraceScope() { --g_no_trace; }

TraceScope::TraceScope(const char* name, hipStream_t stream) {
  if (g_no_trace > 0) return;
  std::lock_guard<std::mutex> lock(g_tr_mu);
  if (!g_tr_on || (int)g_tr.size() >= kMaxTrace) return;
  TraceRec r{name, pool_event(), pool_event()};
  if (!r.start || !r.stop || hipEventRecord(r.start, stream) != hipSuccess) {
    if (r.start) g_ev_pool.push_back(r.start);
    if (r.stop) g_ev_pool.push_back(r.stop);
    return;
  }
  slot_ = (int)g_tr.size();
  stream_ = stream;
  g_tr.push_back(r);
}

TraceScope::~TraceScope() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lock(g_tr_mu);
  if (slot_ < (int)g_tr.size()) (void)hipEventRecord(g_tr[slot_].stop, stream_);
}

// ---------------------------------------------------------------- checks

}  // namespace ccl

using namespace ccl;

extern "C" {

static ccl_status label_edges_checked(int64_t n_sites, int64_t n_bonds, const int32_t* src,
                                      const int32_t* dst, const uint8_t* occupied,
                                      const PhiloxOcc* draw, int32_t* labels_out, void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX || n_bonds < 0) return CCL_ERR_INVALID_VALUE;
  if (n_bonds > 0 && n_sites == 0) return CCL_ERR_INVALID_VALUE;  // no valid ids exist
  if (n_sites > 0 && labels_out == nullptr) return CCL_ERR_INVALID_VALUE;
  if (n_bonds > 0 && (src == nullptr || dst == nullptr)) return CCL_ERR_INVALID_VALUE;
  const size_t lb = (size_t)n_sites * 4, bb = (size_t)n_bonds * 4;
  if (overlaps(labels_out, lb, src, bb) || overlaps(labels_out, lb, dst, bb) ||
      overlaps(labels_out, lb, occupied, (size_t)n_bonds))
    return CCL_ERR_INVALID_VALUE;
  if (n_sites == 0) return CCL_OK;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_label_edges(n_sites, n_bonds, src, dst, occupied, draw, labels_out,
                            (hipStream_t)stream, *d);
}

ccl_status ccl_label(int64_t n_sites, int64_t n_bonds, const int32_t* src, const int32_t* dst,
                     const uint8_t* occupied, int32_t* labels_out, void* stream) {
  return label_edges_checked(n_sites, n_bonds, src, dst, occupied, nullptr, labels_out, stream);
}

size_t ccl_label_csr_workspace_size(int64_t n_sites, int64_t n_bonds) {
  if (n_sites <= 0 || n_bonds < 0) return 0;
  return csr_workspace_bytes(n_sites, n_bonds);
}

static ccl_status label_csr_checked(int64_t n_sites, int64_t n_bonds, int64_t grid_width,
                                    const int32_t* row_ptr, const int32_t* col,
                                    const uint8_t* occupied, const PhiloxOcc* draw,
                                    int32_t* labels_out, void* workspace, size_t workspace_bytes,
                                    void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX || n_bonds < 0 || n_bonds > INT32_MAX || grid_width < 0)
    return CCL_ERR_INVALID_VALUE;
  if (n_sites == 0) return CCL_OK;
  if (row_ptr == nullptr || labels_out == nullptr || (n_bonds > 0 && col == nullptr))
    return CCL_ERR_INVALID_VALUE;
  const size_t need = ccl_label_csr_workspace_size(n_sites, n_bonds);
  if (need > 0 && (workspace == nullptr || workspace_bytes < need || ((uintptr_t)workspace & 7) != 0))
    return CCL_ERR_INVALID_VALUE;
  const size_t lb = (size_t)n_sites * 4;
  if (overlaps(labels_out, lb, row_ptr, lb + 4) || overlaps(labels_out, lb, col, (size_t)n_bonds * 4) ||
      overlaps(labels_out, lb, occupied, (size_t)n_bonds) ||
      overlaps(labels_out, lb, workspace, need))
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_label_csr(n_sites, grid_width, row_ptr, col, occupied, draw, labels_out,
                          need ? workspace : nullptr, (hipStream_t)stream, *d);
}

// occupied iff word < floor(p 2^32); 2^32 (p >= 1) occupies every bond
static uint64_t occupancy_threshold(double p) {
  return !(p > 0.0) ? 0 : (p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(p * 4294967296.0));
}

ccl_status ccl_label_csr(int64_t n_sites, int64_t n_bonds, const int32_t* row_ptr,
                         const int32_t* col, const uint8_t* occupied, int32_t* labels_out,
                         void* workspace, size_t workspace_bytes, void* stream) {
  return label_csr_checked(n_sites, n_bonds, 0, row_ptr, col, occupied, nullptr, labels_out,
                           workspace, workspace_bytes, stream);
}

ccl_status ccl_label_csr_grid(int64_t n_sites, int64_t n_bonds, int64_t grid_width,
                              const int32_t* row_ptr, const int32_t* col, const uint8_t* occupied,
                              int32_t* labels_out, void* workspace, size_t workspace_bytes,
                              void* stream) {
  return label_csr_checked(n_sites, n_bonds, grid_width, row_ptr, col, occupied, nullptr,
                           labels_out, workspace, workspace_bytes, stream);
}

static ccl_status label_csr_philox_checked(int64_t n_sites, int64_t n_bonds, int64_t grid_width,
                                           const int32_t* row_ptr, const int32_t* col, uint64_t seed,
                                           uint32_t stream_id, double p, int32_t* labels_out,
                                           void* workspace, size_t workspace_bytes, void* stream) {
  if (p != p) return CCL_ERR_INVALID_VALUE;  // NaN
  const PhiloxOcc draw{seed, stream_id, occupancy_threshold(p)};
  return label_csr_checked(n_sites, n_bonds, grid_width, row_ptr, col, nullptr, &draw, labels_out,
                           workspace, workspace_bytes, stream);
}

ccl_status ccl_label_csr_philox(int64_t n_sites, int64_t n_bonds, const int32_t* row_ptr,
                                const int32_t* col, uint64_t seed, uint32_t stream_id, double p,
                                int32_t* labels_out, void* workspace, size_t workspace_bytes,
                                void* stream) {
  return label_csr_philox_checked(n_sites, n_bonds, 0, row_ptr, col, seed, stream_id, p, labels_out,
                                  workspace, workspace_bytes, stream);
}

ccl_status ccl_label_csr_grid_philox(int64_t n_sites, int64_t n_bonds, int64_t grid_width,
                                     const int32_t* row_ptr, const int32_t* col, uint64_t seed,
                                     uint32_t stream_id, double p, int32_t* labels_out,
                                     void* workspace, size_t workspace_bytes, void* stream) {
  return label_csr_philox_checked(n_sites, n_bonds, grid_width, row_ptr, col, seed, stream_id, p,
                                  labels_out, workspace, workspace_bytes, stream);
}

ccl_status ccl_label_philox(int64_t n_sites, int64_t n_bonds, const int32_t* src, const int32_t* dst,
                            uint64_t seed, uint32_t stream_id, double p, int32_t* labels_out,
                            void* stream) {
  if (p != p) return CCL_ERR_INVALID_VALUE;  // NaN
  const PhiloxOcc draw{seed, stream_id, occupancy_threshold(p)};
  return label_edges_checked(n_sites, n_bonds, src, dst, nullptr, &draw, labels_out, stream);
}

ccl_status ccl_label_ell(int64_t n_sites, int32_t z_max, const int32_t* nn_list,
                         const uint8_t* occupied, int32_t* labels_out, void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX || z_max < 0) return CCL_ERR_INVALID_VALUE;
  // at most 2^40 list entries (4 TiB): more than any device holds, and the
  // byte sizes below cannot overflow
  if (z_max > 0 && n_sites > ((int64_t)1 << 40) / z_max) return CCL_ERR_INVALID_VALUE;
  if (n_sites == 0) return CCL_OK;
  if (labels_out == nullptr || (z_max > 0 && nn_list == nullptr)) return CCL_ERR_INVALID_VALUE;
  const size_t lb = (size_t)n_sites * 4, eb = (size_t)n_sites * (size_t)z_max;
  if (overlaps(labels_out, lb, nn_list, eb * 4) || overlaps(labels_out, lb, occupied, eb))
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_label_ell(n_sites, z_max, nn_list, z_max > 0 ? occupied : nullptr, labels_out,
                          (hipStream_t)stream, *d);
}

static ccl_status philox_common(uint64_t first, int64_t n, const void* out) {
  if (n < 0 || (n > 0 && out == nullptr)) return CCL_ERR_INVALID_VALUE;
  if (n > 0 && first > UINT64_MAX - (uint64_t)n) return CCL_ERR_INVALID_VALUE;
  return CCL_OK;
}

ccl_status ccl_philox_u32(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n,
                          uint32_t* out, void* stream) {
  ccl_status st = philox_common(first, n, out);
  if (st != CCL_OK || n == 0) return st;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_philox(seed, stream_id, first, n, 0, false, out, (hipStream_t)stream, *d);
}

ccl_status ccl_bernoulli(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n, double p,
                         uint8_t* out, void* stream) {
  ccl_status st = philox_common(first, n, out);
  if (st != CCL_OK || n == 0) return st;
  if (p != p) return CCL_ERR_INVALID_VALUE;  // NaN
  const uint64_t threshold = occupancy_threshold(p);
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_philox(seed, stream_id, first, n, threshold, true, out, (hipStream_t)stream, *d);
}

size_t ccl_cluster_ids_workspace_size(int64_t n_sites) {
  return n_sites > 0 ? cluster_ids_workspace_bytes(n_sites) : 0;
}

ccl_status ccl_cluster_ids(int64_t n_sites, const int32_t* labels, int32_t* ids_out,
                           int32_t* n_clusters_out, void* workspace, size_t workspace_bytes,
                           void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX) return CCL_ERR_INVALID_VALUE;
  if (n_sites == 0) return CCL_OK;
  const size_t need = cluster_ids_workspace_bytes(n_sites), lb = (size_t)n_sites * 4;
  if (!labels || !ids_out || !n_clusters_out || !workspace || workspace_bytes < need ||
      ((uintptr_t)workspace & 3) != 0)
    return CCL_ERR_INVALID_VALUE;
  if (overlaps(labels, lb, ids_out, lb) || overlaps(labels, lb, workspace, need) ||
      overlaps(ids_out, lb, workspace, need) || overlaps(n_clusters_out, 4, labels, lb) ||
      overlaps(n_clusters_out, 4, ids_out, lb) || overlaps(n_clusters_out, 4, workspace, need))
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_cluster_ids(n_sites, labels, ids_out, n_clusters_out, workspace, (hipStream_t)stream,
                            *d);
}

ccl_status ccl_cluster_sizes(int64_t n_sites, const int32_t* labels, int32_t* sizes_out,
                             void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX) return CCL_ERR_INVALID_VALUE;
  if (n_sites == 0) return CCL_OK;
  const size_t lb = (size_t)n_sites * 4;
  if (!labels || !sizes_out || overlaps(labels, lb, sizes_out, lb)) return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_cluster_sizes(n_sites, labels, sizes_out, (hipStream_t)stream, *d);
}

ccl_status ccl_cluster_size_histogram(int64_t n_sites, const int32_t* sizes, int64_t n_bins,
                                      int64_t* hist_out, void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX || n_bins < 2 || hist_out == nullptr)
    return CCL_ERR_INVALID_VALUE;
  if (n_sites > 0 && sizes == nullptr) return CCL_ERR_INVALID_VALUE;
  if (((uintptr_t)hist_out & 7) != 0) return CCL_ERR_INVALID_VALUE;
  if (overlaps(hist_out, (size_t)n_bins * 8, sizes, (size_t)n_sites * 4)) return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_size_histogram(n_sites, sizes, n_bins, hist_out, (hipStream_t)stream, *d);
}

ccl_status ccl_spans(int64_t n_sites, const int32_t* labels, int64_t n_a, const int32_t* sites_a,
                     int64_t n_b, const int32_t* sites_b, uint8_t* flags, int32_t* result_out,
                     void* stream) {
  if (n_sites < 0 || n_sites > INT32_MAX || n_a < 0 || n_b < 0) return CCL_ERR_INVALID_VALUE;
  if (!result_out) return CCL_ERR_INVALID_VALUE;
  if ((n_a > 0 || n_b > 0) && n_sites == 0) return CCL_ERR_INVALID_VALUE;  // no valid ids
  if (n_sites > 0 && (!labels || !flags)) return CCL_ERR_INVALID_VALUE;
  if ((n_a > 0 && !sites_a) || (n_b > 0 && !sites_b)) return CCL_ERR_INVALID_VALUE;
  const size_t lb = (size_t)n_sites * 4, fb = (size_t)n_sites;
  if (overlaps(flags, fb, labels, lb) || overlaps(flags, fb, sites_a, (size_t)n_a * 4) ||
      overlaps(flags, fb, sites_b, (size_t)n_b * 4) || overlaps(result_out, 4, flags, fb) ||
      overlaps(result_out, 4, labels, lb))
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_spans(n_sites, labels, n_a, sites_a, n_b, sites_b, flags, result_out,
                      (hipStream_t)stream, *d);
}

static ccl_status run_count(unsigned long long* n_bad, hipStream_t s,
                            ccl_status (*launch)(const void*, unsigned long long*, hipStream_t,
                                                 const DeviceInfo&),
                            const void* args) {
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  unsigned long long* dc = nullptr;
  hipError_t e = hipMalloc(&dc, sizeof(unsigned long long));
  if (e != hipSuccess) return fail_hip(e);
  ccl_status st = CCL_OK;
  e = hipMemsetAsync(dc, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) st = fail_hip(e);
  if (st == CCL_OK) st = launch(args, dc, s, *d);
  if (st == CCL_OK) {
    e = hipMemcpyAsync(n_bad, dc, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail_hip(e);
  }
  (void)hipFree(dc);
  return st;
}

struct EdgeCheckArgs {
  int64_t n, m;
  const int32_t *src, *dst;
};
struct CsrCheckArgs {
  int64_t n, n_col;
  const int32_t *row_ptr, *col;
};

ccl_status ccl_validate_edges(int64_t n_sites, int64_t n_bonds, const int32_t* src,
                              const int32_t* dst, int64_t* n_bad_host, void* stream) {
  if (n_sites < 0 || n_bonds < 0 || n_bad_host == nullptr) return CCL_ERR_INVALID_VALUE;
  if (n_bonds > 0 && (src == nullptr || dst == nullptr)) return CCL_ERR_INVALID_VALUE;
  *n_bad_host = 0;
  if (n_bonds == 0) return CCL_OK;
  EdgeCheckArgs a{n_sites, n_bonds, src, dst};
  unsigned long long bad = 0;
  ccl_status st = run_count(
      &bad, (hipStream_t)stream,
      [](const void* p, unsigned long long* dc, hipStream_t s, const DeviceInfo& d) {
        auto* x = static_cast<const EdgeCheckArgs*>(p);
        return launch_validate_edges(x->n, x->m, x->src, x->dst, dc, s, d);
      },
      &a);
  if (st != CCL_OK) return st;
  *n_bad_host = (int64_t)bad;
  return bad ? CCL_ERR_INDEX_OUT_OF_RANGE : CCL_OK;
}

ccl_status ccl_validate_csr(int64_t n_sites, const int32_t* row_ptr, const int32_t* col,
                            int64_t n_col, int64_t* n_bad_host, void* stream) {
  if (n_sites < 0 || n_col < 0 || n_bad_host == nullptr) return CCL_ERR_INVALID_VALUE;
  if ((n_sites > 0 && row_ptr == nullptr) || (n_col > 0 && col == nullptr))
    return CCL_ERR_INVALID_VALUE;
  *n_bad_host = 0;
  if (n_sites == 0 && n_col == 0) return CCL_OK;
  CsrCheckArgs a{n_sites, n_col, row_ptr, col};
  unsigned long long bad = 0;
  ccl_status st = run_count(
      &bad, (hipStream_t)stream,
      [](const void* p, unsigned long long* dc, hipStream_t s, const DeviceInfo& d) {
        auto* x = static_cast<const CsrCheckArgs*>(p);
        return launch_validate_csr(x->n, x->row_ptr, x->col, x->n_col, dc, s, d);
      },
      &a);
  if (st != CCL_OK) return st;
  *n_bad_host = (int64_t)bad;
  return bad ? CCL_ERR_INDEX_OUT_OF_RANGE : CCL_OK;
}

const char* ccl_status_string(ccl_status s) {
  switch (s) {
    case CCL_OK:
      return "CCL_OK";
    case CCL_ERR_INVALID_VALUE:
      return "CCL_ERR_INVALID_VALUE: bad argument";
    case CCL_ERR_INDEX_OUT_OF_RANGE:
      return "CCL_ERR_INDEX_OUT_OF_RANGE: site id outside [0, n_sites)";
    case CCL_ERR_OUT_OF_MEMORY:
      return "CCL_ERR_OUT_OF_MEMORY: device allocation failed";
    case CCL_ERR_HIP:
      return "CCL_ERR_HIP: a HIP call failed";
    case CCL_ERR_NOT_SUPPORTED:
      return "CCL_ERR_NOT_SUPPORTED: device is not gfx950";
    case CCL_ERR_TOO_LARGE:
      return "CCL_ERR_TOO_LARGE: input exceeds the fixed capacity of a no-allocation entry point";
  }
  return "unknown ccl_status";
}

int ccl_last_hip_error(void) { return g_last_hip_error; }

int ccl_version(void) { return 100; }

ccl_status ccl_trace_enable(int on) {
  std::lock_guard<std::mutex> lock(g_tr_mu);
  if (on) clear_records_locked();
  g_tr_on = on != 0;
  return CCL_OK;
}

int ccl_trace_count(void) {
  std::lock_guard<std::mutex> lock(g_tr_mu);
  for (auto& r : g_tr)
    if (hipEventSynchronize(r.stop) != hipSuccess) return -1;
  return (int)g_tr.size();
}

ccl_status ccl_trace_get(int i, const char** kernel_name, float* ms) {
  std::lock_guard<std::mutex> lock(g_tr_mu);
  if (i < 0 || i >= (int)g_tr.size() || !kernel_name || !ms) return CCL_ERR_INVALID_VALUE;
  hipError_t e = hipEventSynchronize(g_tr[i].stop);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, g_tr[i].start, g_tr[i].stop);
  if (e != hipSuccess) return fail_hip(e);
  *kernel_name = g_tr[i].name;
  return CCL_OK;
}

ccl_status ccl_probe_copy(const void* in, void* out, size_t bytes, void* stream) {
  if (bytes == 0) return CCL_OK;
  if (!in || !out || ((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  return launch_probe_copy(in, out, bytes, (hipStream_t)stream, *d);
}

}  // extern "C"
