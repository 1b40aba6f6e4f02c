// Measurement probes for the ceilings of random-access work (the random
// graphs' merge and flatten are bound by scattered 4-byte accesses, not by
// streaming bandwidth): random gathers, random-address atomicMin (with the
// result discarded, and with it used as Algorithm 1 uses it), and chains of
// dependent loads.  Addresses come from a multiplicative hash of the
// operation index mapped onto the table; nothing here is part of labeling.
#include "common.hpp"

namespace ccl {

constexpr int kProbeBlock = 256;
constexpr int kProbeIlp = 16;  // independent operations a lane keeps in flight

__device__ __forceinline__ uint32_t probe_index(uint64_t i, uint64_t len) {
  const uint64_t h = (i + 0x632BE59BD9B4E019ull) * 0x9E3779B97F4A7C15ull;
  return (uint32_t)(((h >> 32) * len) >> 32);  // multiply-shift onto [0, len)
}

// mode: 0 gather, 1 atomicMin result unused, 2 atomicMin result used,
// 3 dependent chase (table[i] holds the next index), 4 fill the chase table
__global__ void __launch_bounds__(kProbeBlock)
    k_probe_random(int32_t* table, int64_t len, int64_t n_ops, int32_t mode, int32_t* sink) {
  const int64_t lanes = (int64_t)gridDim.x * kProbeBlock;
  const int64_t tid = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  if (mode == 4) {
    for (int64_t i = tid; i < len; i += lanes) table[i] = (int32_t)probe_index((uint64_t)i * 7919u + 1u, (uint64_t)len);
    return;
  }
  int32_t acc = 0;
  if (mode == 3) {
    // kProbeIlp independent chains per lane, n_ops / lanes / kProbeIlp steps each
    const int64_t steps = n_ops / (lanes * kProbeIlp);
    int32_t x[kProbeIlp];
#pragma unroll
    for (int k = 0; k < kProbeIlp; ++k) x[k] = (int32_t)probe_index((uint64_t)(tid * kProbeIlp + k), (uint64_t)len);
    for (int64_t s = 0; s < steps; ++s)
#pragma unroll
      for (int k = 0; k < kProbeIlp; ++k) x[k] = __hip_atomic_load(table + x[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
#pragma unroll
    for (int k = 0; k < kProbeIlp; ++k) acc ^= x[k];
  } else {
    for (int64_t i0 = tid * kProbeIlp; i0 < n_ops; i0 += lanes * kProbeIlp) {
      int32_t r[kProbeIlp];
#pragma unroll
      for (int k = 0; k < kProbeIlp; ++k) {
        const uint32_t a = probe_index((uint64_t)(i0 + k), (uint64_t)len);
        if (mode == 0)
          r[k] = __hip_atomic_load(table + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        else if (mode == 1)
          __hip_atomic_fetch_min(table + a, (int32_t)(i0 + k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), r[k] = 0;
        else
          r[k] = __hip_atomic_fetch_min(table + a, (int32_t)(i0 + k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int k = 0; k < kProbeIlp; ++k) acc ^= r[k];
    }
  }
  if (acc == 0x7F3A9C11) sink[0] = acc;  // keeps the loads alive; practically never taken
}

ccl_status launch_probe_random(int32_t* table, int64_t len, int64_t n_ops, int32_t mode, int32_t* sink,
                               hipStream_t s, const DeviceInfo& d) {
  const unsigned g = (unsigned)(d.cu_count * 8);
  static const char* names[5] = {"ccl_probe_gather", "ccl_probe_atomic_min", "ccl_probe_atomic_min_ret",
                                  "ccl_probe_chase", "ccl_probe_fill"};
  CCL_LAUNCH(names[mode], k_probe_random, g, kProbeBlock, 0, s, table, len, n_ops, mode, sink);
  return CCL_OK;
}

}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_probe_random(int32_t* table, int64_t table_len, int64_t n_ops, int32_t mode,
                                       int32_t* sink, void* stream) {
  if (table == nullptr || sink == nullptr || table_len <= 0 || table_len > INT32_MAX || n_ops < 0 ||
      mode < 0 || mode > 4)
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  return launch_probe_random(table, table_len, n_ops, mode, sink, (hipStream_t)stream, *d);
}
