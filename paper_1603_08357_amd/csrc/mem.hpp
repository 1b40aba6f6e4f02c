// Global-memory access helpers shared by the kernels of libccl.so.
//
// Stores.  A store whose word a later kernel of the same call overwrites,
// or updates with atomics, is a device-scope (agent) store: on gfx950 it
// carries the sc1 cache-policy bit and is written through to the
// device-coherent level when it completes, instead of waiting as a dirty
// line in the writing XCD's L2.  A serving run on MI355X (eight streams of
// random-graph jobs) once found a label holding a merge-step compression
// store's value where the following flatten kernel had stored the final
// root: that plain store became visible after a later kernel's store of the
// same word.  The compression stores are atomicMin since (uf.hpp); every
// other store of that kind -- init, tile labels, the neighbour-list step
// (i), the batched items, counters and flags that later kernels update --
// goes through these helpers.  Measured cost on MI355X: none for the
// edge-list init and flatten, 0.011 ms for the tile kernel of the 2^26-site
// lattice.  The plain stores left are a call's final values that no later
// kernel of the call touches (the windowed CSR flatten, the batched FLATTEN
// items).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

// ---------------------------------------------------------------- buffers

// Raw buffer loads and stores (gfx9 buffer resource, 32-bit offsets): an
// offset past the resource's byte size reads 0 (a store there is dropped)
// instead of faulting, so a whole batch of loads can be issued without
// branches and stays in flight together.  The base must be wavefront-uniform.
constexpr uint32_t kBufWord3 = 0x00020000;
constexpr uint32_t kOffNone = 0xFFFFFFF0u;  // beyond any resource used here
constexpr int kCpolSc1 = 16;                // cache policy: device-scope (sc1)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, (int)kBufWord3);
}
__device__ __forceinline__ int32_t buf_i32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ uint32_t buf_u32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ uint32_t buf_u8(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ int4 buf_i32x4(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0);
  return make_int4((int32_t)v[0], (int32_t)v[1], (int32_t)v[2], (int32_t)v[3]);
}

// ---------------------------------------------------------------- stores

// Device-scope stores of one, two and four int32 words.
__device__ __forceinline__ void st_dev(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint8_t* p, uint8_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev2(int2* p, int2 v) {
  const uint64_t w = (uint64_t)(uint32_t)v.x | ((uint64_t)(uint32_t)v.y << 32);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// 16 bytes at byte offset off of a buffer resource (wavefront-uniform base)
__device__ __forceinline__ void st_dev4(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, int4 v) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 w = {(unsigned)v.x, (unsigned)v.y, (unsigned)v.z, (unsigned)v.w};
  __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)byte_off, 0, kCpolSc1);
}
// 4 bytes (e.g. four occupancy bytes) at byte offset off of a buffer resource
__device__ __forceinline__ void st_dev_u32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)byte_off, 0, kCpolSc1);
}

}  // namespace ccl
