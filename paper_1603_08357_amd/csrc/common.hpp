// Host-side internals shared by the translation units of libccl.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccl.h"

namespace ccl {

struct DeviceInfo {
  int device = -1;
  int cu_count = 0;
  int max_lds_per_block = 0;
  bool is_gfx950 = false;
};

// Properties of the current device (queried once per device, then cached).
// Returns nullptr and records the HIP error when the query fails.
const DeviceInfo* current_device();

// Record a failed HIP call for ccl_last_hip_error() and map it to a status.
ccl_status fail_hip(hipError_t e);

// Kernel timing (ccl_trace_*): while enabled, the scope records a HIP event
// on `stream` when it opens and another when it closes.
class TraceScope {
 public:
  TraceScope(const char* name, hipStream_t stream);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  int slot_ = -1;
  hipStream_t stream_ = nullptr;
};

// While one of these is alive on a host thread, TraceScope records nothing on
// that thread (used where creating HIP events is not allowed).
class NoTraceScope {
 public:
  NoTraceScope();
  ~NoTraceScope();
  NoTraceScope(const NoTraceScope&) = delete;
  NoTraceScope& operator=(const NoTraceScope&) = delete;
};

// Grid for a grid-stride kernel: enough workgroups to cover `work` items at
// `per_block` items each, capped at `per_cu` resident workgroups per CU.
inline unsigned grid_for(int64_t work, int64_t per_block, int per_cu, const DeviceInfo& d) {
  int64_t need = (work + per_block - 1) / per_block;
  int64_t cap = (int64_t)d.cu_count * per_cu;
  if (need < 1) need = 1;
  return (unsigned)(need < cap ? need : cap);
}

// True when the byte ranges [a, a+na) and [b, b+nb) intersect.
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + nb && b0 < a0 + na;
}

// Launch + error check; returns from the calling function on failure.
#define CCL_LAUNCH(name, kernel, grid, block, lds, stream, ...)                          \
  do {                                                                                  \
    {                                                                                   \
      ::ccl::TraceScope ccl_trace_scope_(name, stream);                                 \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, __VA_ARGS__);    \
    }                                                                                   \
    hipError_t ccl_launch_err_ = hipGetLastError();                                     \
    if (ccl_launch_err_ != hipSuccess) return ::ccl::fail_hip(ccl_launch_err_);         \
  } while (0)

// Workgroups of a launch are dispatched to the 8 XCDs (each with its own L2)
// in round-robin order.  This renumbering gives each XCD one contiguous range
// of logical workgroup ids, so neighbouring data lands in one L2.
struct XcdSlot {
  uint32_t xcd;    // XCD this workgroup runs on
  uint32_t index;  // its rank among that XCD's workgroups
  uint32_t count;  // workgroups on that XCD
};
constexpr uint32_t kNumXcd = 8;
__device__ __forceinline__ XcdSlot xcd_slot() {
  const uint32_t n = gridDim.x, b = blockIdx.x;
  XcdSlot s;
  s.xcd = b % kNumXcd;
  s.index = b / kNumXcd;
  s.count = n / kNumXcd + (s.xcd < n % kNumXcd ? 1u : 0u);
  return s;
}
__device__ __forceinline__ uint32_t xcd_block_id() {
  const XcdSlot s = xcd_slot();
  const uint32_t per = gridDim.x / kNumXcd, rem = gridDim.x % kNumXcd;
  return s.xcd * per + (s.xcd < rem ? s.xcd : rem) + s.index;
}

// Launchers (one translation unit each); arguments already validated.
ccl_status launch_init(int64_t n, int32_t* label, hipStream_t s, const DeviceInfo& d);
ccl_status launch_flatten(int64_t n, int32_t* label, hipStream_t s, const DeviceInfo& d);
struct PhiloxOcc;
// occ: a mask aligned with the bonds (src/dst, or col), or NULL; draw (only
// with occ NULL): draw the occupancy of bond e as word e of that Philox
// stream; both NULL: all occupied
ccl_status launch_label_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              const uint8_t* occ, const PhiloxOcc* draw, int32_t* label,
                              hipStream_t s, const DeviceInfo& d);
// grid_w: row length of the id grid (tiles of 32 rows x 2048 columns), or 0
ccl_status launch_label_csr(int64_t n, int64_t grid_w, const int32_t* row_ptr, const int32_t* col,
                            const uint8_t* occ, const PhiloxOcc* draw, int32_t* label,
                            void* workspace, hipStream_t s, const DeviceInfo& d);
size_t csr_workspace_bytes(int64_t n_sites, int64_t n_bonds);
ccl_status launch_label_ell(int64_t n, int32_t z, const int32_t* nn, const uint8_t* occ,
                            int32_t* label, hipStream_t s, const DeviceInfo& d);
ccl_status launch_philox(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n,
                         uint64_t threshold, bool bytes, void* out, hipStream_t s,
                         const DeviceInfo& d);
size_t cluster_ids_workspace_bytes(int64_t n);
ccl_status launch_cluster_ids(int64_t n, const int32_t* label, int32_t* ids, int32_t* n_clusters,
                              void* workspace, hipStream_t s, const DeviceInfo& d);
ccl_status launch_cluster_sizes(int64_t n, const int32_t* label, int32_t* sizes, hipStream_t s,
                                const DeviceInfo& d);
ccl_status launch_size_histogram(int64_t n, const int32_t* sizes, int64_t n_bins, int64_t* hist,
                                 hipStream_t s, const DeviceInfo& d);
ccl_status launch_spans(int64_t n, const int32_t* label, int64_t n_a, const int32_t* a, int64_t n_b,
                        const int32_t* b, uint8_t* flags, int32_t* result, hipStream_t s,
                        const DeviceInfo& d);
ccl_status launch_validate_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                 unsigned long long* d_count, hipStream_t s, const DeviceInfo& d);
ccl_status launch_validate_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                               int64_t n_col, unsigned long long* d_count, hipStream_t s,
                               const DeviceInfo& d);
ccl_status launch_probe_random(int32_t* table, int64_t len, int64_t n_ops, int32_t mode, int32_t* sink,
                               hipStream_t s, const DeviceInfo& d);
ccl_status launch_probe_copy(const void* in, void* out, size_t bytes, hipStream_t s,
                             const DeviceInfo& d);

// Sites per tile of the CSR path (one workgroup, a 16-bit LDS slot per site).
constexpr int kCsrTile = 65536;

}  // namespace ccl
