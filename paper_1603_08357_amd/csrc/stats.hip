// Cluster statistics of a finished labeling (label[i] = minimum site id of
// i's cluster), for the percolation application of section 4:
//   * sequential cluster ids (the renumbering the paper points to at the end
//     of section 3): the k-th smallest cluster minimum gets id k;
//   * cluster sizes, indexed by the cluster's minimum site;
//   * the spanning test: does one cluster hold a site of set A and one of B.
// A site i is its cluster's minimum exactly when label[i] == i.
#include "common.hpp"
#include "mem.hpp"

namespace ccl {

// ---------------------------------------------------------------- ids

constexpr int kIdBlock = 1024;
constexpr int kIdPer = 4;                        // sites per lane
constexpr int kIdSpan = kIdBlock * kIdPer;       // sites per workgroup
static_assert(kIdPer == 4, "a lane moves its four sites as one int4");

// Inclusive prefix sum of v over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive prefix of v over the workgroup (kIdBlock lanes); *total gets the
// sum.  `scratch` holds one word per wavefront.
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t* scratch, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int kWaves = kIdBlock / 64;
  const uint32_t inc = wave_inclusive_sum(v);
  if (lane == 63) scratch[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const uint32_t w = lane < kWaves ? scratch[lane] : 0u;
    const uint32_t wi = wave_inclusive_sum(w);
    if (lane < kWaves) scratch[lane] = wi - w;  // exclusive per wavefront
    if (lane == kWaves - 1) scratch[kWaves] = wi;
  }
  __syncthreads();
  const uint32_t r = scratch[wave] + inc - v;
  *total = scratch[kWaves];
  __syncthreads();  // scratch is reused by the caller's next call
  return r;
}

// ids[i] = number of cluster minima before i within the workgroup's span;
// the span's count goes to part[block].
// vec: label and ids are 16-byte aligned.
__global__ void __launch_bounds__(kIdBlock)
    k_ids_local(int64_t n, const int32_t* __restrict__ label, int32_t* __restrict__ ids,
                int32_t* __restrict__ part, bool vec) {
  __shared__ uint32_t scratch[kIdBlock / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kIdSpan + (int64_t)threadIdx.x * kIdPer;
  const bool whole = vec && base + kIdPer <= n;  // four sites in one 16-byte access
  int32_t lab[kIdPer];
  if (whole) {
    const int4 v = reinterpret_cast<const int4*>(label + base)[0];
    lab[0] = v.x; lab[1] = v.y; lab[2] = v.z; lab[3] = v.w;
  } else {
#pragma unroll
    for (int k = 0; k < kIdPer; ++k) lab[k] = base + k < n ? label[base + k] : -1;
  }
  uint32_t f[kIdPer], s = 0;
#pragma unroll
  for (int k = 0; k < kIdPer; ++k) {
    f[k] = lab[k] == (int32_t)(base + k) ? 1u : 0u;
    s += f[k];
  }
  uint32_t total;
  const uint32_t run = block_exclusive_sum(s, scratch, &total);
  const int32_t r0 = (int32_t)run, r1 = r0 + (int32_t)f[0], r2 = r1 + (int32_t)f[1], r3 = r2 + (int32_t)f[2];
  if (whole) {
    // 16 bytes through a resource based at the workgroup's span (uniform)
    const int64_t b0 = (int64_t)blockIdx.x * kIdSpan;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(ids + b0, 4u * (uint32_t)min((int64_t)kIdSpan, n - b0));
    st_dev4(rs, 16u * threadIdx.x, make_int4(r0, r1, r2, r3));
  } else {
    const int32_t r[kIdPer] = {r0, r1, r2, r3};
#pragma unroll
    for (int k = 0; k < kIdPer; ++k)
      if (base + k < n) st_dev(ids + base + k, r[k]);
  }
  if (threadIdx.x == 0) st_dev(part + blockIdx.x, (int32_t)total);
}

// Exclusive scan of the per-workgroup counts, in one workgroup, chunk by
// chunk; the total is the number of clusters.
__global__ void __launch_bounds__(kIdBlock)
    k_ids_parts(int64_t n_parts, int32_t* __restrict__ part, int32_t* __restrict__ n_clusters) {
  __shared__ uint32_t scratch[kIdBlock / 64 + 1];
  uint32_t carry = 0;
  for (int64_t c = 0; c < n_parts; c += kIdBlock) {
    const int64_t j = c + threadIdx.x;
    const uint32_t v = j < n_parts ? (uint32_t)part[j] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_sum(v, scratch, &total);
    if (j < n_parts) st_dev(part + j, (int32_t)(carry + ex));
    carry += total;
  }
  if (threadIdx.x == 0) st_dev(n_clusters, (int32_t)carry);
}

// Adds each span's offset: ids[i] becomes the number of minima before i.
__global__ void __launch_bounds__(kIdBlock)
    k_ids_offset(int64_t n, const int32_t* __restrict__ part, int32_t* __restrict__ ids, bool vec) {
  const int64_t base = (int64_t)blockIdx.x * kIdSpan + (int64_t)threadIdx.x * kIdPer;
  const int32_t off = part[blockIdx.x];
  if (vec && base + kIdPer <= n) {
    int4 v = reinterpret_cast<int4*>(ids + base)[0];
    v.x += off; v.y += off; v.z += off; v.w += off;
    const int64_t b0 = (int64_t)blockIdx.x * kIdSpan;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(ids + b0, 4u * (uint32_t)min((int64_t)kIdSpan, n - b0));
    st_dev4(rs, 16u * threadIdx.x, v);
    return;
  }
#pragma unroll
  for (int k = 0; k < kIdPer; ++k)
    if (base + k < n) st_dev(ids + base + k, ids[base + k] + off);
}

// ids[i] = ids[label[i]]: a minimum's entry is its own id and is rewritten
// with the same value, and only minima are read, so this is done in place.
// A label outside [0, n) (not a finished labeling) gives -1, never an access
// outside the arrays.
// vec: label and ids are 16-byte aligned; a lane then moves four sites with
// one 16-byte load of labels and one 16-byte store of ids.
__global__ void __launch_bounds__(kIdBlock)
    k_ids_gather(int64_t n, const int32_t* __restrict__ label, int32_t* ids, bool vec) {
  const int64_t stride = (int64_t)gridDim.x * kIdBlock;
  const int64_t tid = (int64_t)blockIdx.x * kIdBlock + threadIdx.x;
  auto id_of = [&](int32_t r) { return (r >= 0 && r < n) ? ids[r] : -1; };
  int64_t done = 0;
  if (vec) {
    const int64_t n4 = n >> 2;
    for (int64_t q0 = (int64_t)blockIdx.x * kIdBlock; q0 < n4; q0 += stride) {
      const int64_t q = q0 + threadIdx.x;
      // 16-byte stores through a resource based at the step's first group
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(ids + 4 * q0, 16u * (uint32_t)min((int64_t)kIdBlock, n4 - q0));
      const int4 l = reinterpret_cast<const int4*>(label)[min(q, n4 - 1)];
      if (q < n4) st_dev4(rs, 16u * threadIdx.x, make_int4(id_of(l.x), id_of(l.y), id_of(l.z), id_of(l.w)));
    }
    done = 4 * n4;
  }
  for (int64_t i = done + tid; i < n; i += stride) st_dev(ids + i, id_of(label[i]));
}

size_t cluster_ids_workspace_bytes(int64_t n) {
  const int64_t parts = (n + kIdSpan - 1) / kIdSpan;
  return (size_t)(parts > 0 ? parts : 1) * sizeof(int32_t);
}

ccl_status launch_cluster_ids(int64_t n, const int32_t* label, int32_t* ids, int32_t* n_clusters,
                              void* workspace, hipStream_t s, const DeviceInfo& d) {
  const int64_t parts = (n + kIdSpan - 1) / kIdSpan;
  int32_t* part = static_cast<int32_t*>(workspace);
  const bool vec = ((reinterpret_cast<uintptr_t>(label) | reinterpret_cast<uintptr_t>(ids)) & 15) == 0;
  CCL_LAUNCH("ccl_ids_local", k_ids_local, (unsigned)parts, kIdBlock, 0, s, n, label, ids, part, vec);
  CCL_LAUNCH("ccl_ids_parts", k_ids_parts, 1u, kIdBlock, 0, s, parts, part, n_clusters);
  CCL_LAUNCH("ccl_ids_offset", k_ids_offset, (unsigned)parts, kIdBlock, 0, s, n, part, ids, vec);
  CCL_LAUNCH("ccl_ids_gather", k_ids_gather, grid_for(vec ? (n + 3) / 4 : n, kIdBlock, 8, d), kIdBlock,
             0, s, n, label, ids, vec);
  return CCL_OK;
}

// ---------------------------------------------------------------- sizes

// Sizes in two passes over spans of kSzSpan sites, one workgroup per span.
// Labels are cluster minima, so a label r that appears in span [b, b+S) with
// r >= b has its own site r in that span: the span owns entry r.
//   1. own: each span counts the sites labelled by its own entries in a
//      direct-indexed LDS array and writes its whole range of `sizes` with
//      non-atomic stores (zero where the site is no minimum), so no fill is needed;
//   2. foreign: each span counts the labels r < b (clusters whose minimum is
//      in an earlier span) in an LDS hash table and adds them with one global
//      atomic per distinct label, after pass 1 has written every entry.
// Runs of equal labels inside a lane are counted first.  At the percolation
// threshold most clusters are small and local: on the 2^26-site triangle
// lattice 7.5 M of the 12.4 M (label, span) pairs are owned, so the global
// atomics drop to the 4.9 M foreign ones.  Labels outside [0, n) are skipped.
constexpr int kSzBlock = 512;
constexpr int kSzPer = 8;
constexpr int kSzSpan = kSzBlock * kSzPer;
constexpr int kSzSlots = 2 * kSzSpan;  // a span has at most kSzSpan distinct labels
static_assert((kSzSlots & (kSzSlots - 1)) == 0, "power of two");

// Calls add(label, count) once per run of equal labels among the lane's
// kSzPer consecutive sites (two 16-byte loads when `vec`: label is 16-byte
// aligned and the lane's sites are all below n).
static_assert(kSzPer == 8, "a lane reads its sites as two int4");
template <class Add>
__device__ __forceinline__ void lane_runs(int64_t n, const int32_t* __restrict__ label, bool vec,
                                          Add add) {
  const int64_t base = (int64_t)blockIdx.x * kSzSpan + (int64_t)threadIdx.x * kSzPer;
  int32_t lab[kSzPer];
  int cnt = 0;
  if (vec && base + kSzPer <= n) {
    const int4 u = reinterpret_cast<const int4*>(label + base)[0];
    const int4 v = reinterpret_cast<const int4*>(label + base)[1];
    lab[0] = u.x; lab[1] = u.y; lab[2] = u.z; lab[3] = u.w;
    lab[4] = v.x; lab[5] = v.y; lab[6] = v.z; lab[7] = v.w;
    cnt = kSzPer;
  } else {
#pragma unroll
    for (int k = 0; k < kSzPer; ++k) lab[k] = base + k < n ? label[base + k] : 0;
    cnt = base >= n ? 0 : (int)min((int64_t)kSzPer, n - base);
  }
  int32_t cur = -1;
  uint32_t run = 0;
#pragma unroll
  for (int k = 0; k < kSzPer; ++k) {
    if (k >= cnt) break;
    const int32_t r = lab[k];
    if (r == cur) {
      ++run;
    } else {
      if (run) add(cur, run);
      cur = r;
      run = 1;
    }
  }
  if (run) add(cur, run);
}

__global__ void __launch_bounds__(kSzBlock)
    k_sizes_own(int64_t n, const int32_t* __restrict__ label, int32_t* __restrict__ sizes, bool vec) {
  __shared__ uint32_t cnt[kSzSpan];
  for (int t = threadIdx.x; t < kSzSpan; t += kSzBlock) cnt[t] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * kSzSpan;
  lane_runs(n, label, vec, [&](int32_t r, uint32_t c) {
    const int64_t t = (int64_t)r - b;
    if (t >= 0 && t < kSzSpan)
      __hip_atomic_fetch_add(&cnt[t], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  });
  __syncthreads();
  const int32_t span = (int32_t)min((int64_t)kSzSpan, n - b);
  for (int t = threadIdx.x; t < span; t += kSzBlock) st_dev(sizes + b + t, (int32_t)cnt[t]);
}

__global__ void __launch_bounds__(kSzBlock)
    k_sizes_foreign(int64_t n, const int32_t* __restrict__ label, int32_t* sizes, bool vec) {
  __shared__ int32_t key[kSzSlots];
  __shared__ uint32_t cnt[kSzSlots];
  for (int t = threadIdx.x; t < kSzSlots; t += kSzBlock) {
    key[t] = -1;
    cnt[t] = 0;
  }
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * kSzSpan;
  lane_runs(n, label, vec, [&](int32_t r, uint32_t c) {
    if (r < 0 || r >= b) return;  // owned by this span, or not a site id
    uint32_t h = ((uint32_t)r * 2654435761u) & (kSzSlots - 1);
    for (;;) {
      int32_t seen = -1;
      if (__hip_atomic_compare_exchange_strong(&key[h], &seen, r, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP) ||
          seen == r) {
        __hip_atomic_fetch_add(&cnt[h], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
      }
      h = (h + 1) & (kSzSlots - 1);
    }
  });
  __syncthreads();
  for (int t = threadIdx.x; t < kSzSlots; t += kSzBlock)
    if (key[t] >= 0) atomicAdd(sizes + key[t], (int32_t)cnt[t]);
}

ccl_status launch_cluster_sizes(int64_t n, const int32_t* label, int32_t* sizes, hipStream_t s,
                                const DeviceInfo& d) {
  (void)d;
  const unsigned spans = (unsigned)((n + kSzSpan - 1) / kSzSpan);
  const bool vec = (reinterpret_cast<uintptr_t>(label) & 15) == 0;
  CCL_LAUNCH("ccl_sizes_own", k_sizes_own, spans, kSzBlock, 0, s, n, label, sizes, vec);
  if (spans > 1)
    CCL_LAUNCH("ccl_sizes_foreign", k_sizes_foreign, spans, kSzBlock, 0, s, n, label, sizes, vec);
  return CCL_OK;
}

// ---------------------------------------------------------------- size histogram

// n_s, the number of clusters of s sites, from the sizes at the cluster
// minima (zero elsewhere): hist[min(s, n_bins - 1)] += 1 for every s > 0.
// Each workgroup counts the bins below kHistLds in LDS and adds them to the
// global histogram with one 64-bit atomic per nonzero bin; larger sizes (rare
// at any p: few clusters are that large) go straight to global atomics.  The
// histogram is cleared by a kernel, so the sequence can be captured in a graph.
constexpr int kHistBlock = 1024;
constexpr int kHistLds = 8192;

__global__ void __launch_bounds__(256) k_hist_clear(int64_t n_bins, unsigned long long* hist) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_bins; i += stride)
    __hip_atomic_store(hist + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kHistBlock)
    k_hist_count(int64_t n, const int32_t* __restrict__ sizes, int64_t n_bins,
                 unsigned long long* hist, bool vec) {
  __shared__ uint32_t cnt[kHistLds];
  const int64_t lds_bins = min((int64_t)kHistLds, n_bins);
  for (int t = threadIdx.x; t < lds_bins; t += kHistBlock) cnt[t] = 0;
  __syncthreads();
  auto add = [&](int32_t sz) {
    if (sz <= 0) return;
    const int64_t b = min((int64_t)sz, n_bins - 1);
    if (b < lds_bins)
      __hip_atomic_fetch_add(&cnt[b], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      atomicAdd(hist + b, 1ull);
  };
  const int64_t stride = (int64_t)gridDim.x * kHistBlock;
  const int64_t tid = (int64_t)blockIdx.x * kHistBlock + threadIdx.x;
  int64_t done = 0;
  if (vec) {
    const int64_t n4 = n >> 2;
    for (int64_t q = tid; q < n4; q += stride) {
      const int4 v = reinterpret_cast<const int4*>(sizes)[q];
      add(v.x);
      add(v.y);
      add(v.z);
      add(v.w);
    }
    done = n4 << 2;
  }
  for (int64_t i = done + tid; i < n; i += stride) add(sizes[i]);
  __syncthreads();
  for (int t = threadIdx.x; t < lds_bins; t += kHistBlock)
    if (cnt[t]) atomicAdd(hist + t, (unsigned long long)cnt[t]);
}

ccl_status launch_size_histogram(int64_t n, const int32_t* sizes, int64_t n_bins, int64_t* hist,
                                 hipStream_t s, const DeviceInfo& d) {
  unsigned long long* h = reinterpret_cast<unsigned long long*>(hist);
  CCL_LAUNCH("ccl_hist_clear", k_hist_clear, grid_for(n_bins, 256, 4, d), 256, 0, s, n_bins, h);
  if (n == 0) return CCL_OK;
  const bool vec = (reinterpret_cast<uintptr_t>(sizes) & 15) == 0;
  CCL_LAUNCH("ccl_hist_count", k_hist_count, grid_for(vec ? (n + 3) / 4 : n, kHistBlock, 1, d), kHistBlock,
             0, s, n, sizes, n_bins, h, vec);
  return CCL_OK;
}

// ---------------------------------------------------------------- spanning

// flags[label[a]] = 1 for every site a of A; then any site b of B whose
// cluster is flagged sets *result.  Site ids and labels outside [0, n) are
// skipped.  Flag stores are byte stores of the
// same value (races are benign); the flag array is cleared by a kernel, so
// the sequence can be captured in a graph.
constexpr int kSpBlock = 256;

__global__ void __launch_bounds__(kSpBlock)
    k_span_clear(int64_t n, uint8_t* __restrict__ flags, int32_t* __restrict__ result) {
  const int64_t stride = (int64_t)gridDim.x * kSpBlock;
  for (int64_t i = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; i < n; i += stride) st_dev(flags + i, (uint8_t)0);
  if (blockIdx.x == 0 && threadIdx.x == 0) st_dev(result, 0);
}

__global__ void __launch_bounds__(kSpBlock)
    k_span_mark(int64_t n, int64_t n_a, const int32_t* __restrict__ a, const int32_t* __restrict__ label,
                uint8_t* __restrict__ flags) {
  const int64_t stride = (int64_t)gridDim.x * kSpBlock;
  for (int64_t j = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; j < n_a; j += stride) {
    const int32_t i = a[j];
    const int32_t r = (i >= 0 && i < n) ? label[i] : -1;
    if (r >= 0 && r < n) st_dev(flags + r, (uint8_t)1);
  }
}

__global__ void __launch_bounds__(kSpBlock)
    k_span_test(int64_t n, int64_t n_b, const int32_t* __restrict__ b, const int32_t* __restrict__ label,
                const uint8_t* __restrict__ flags, int32_t* __restrict__ result) {
  const int64_t stride = (int64_t)gridDim.x * kSpBlock;
  bool hit = false;
  for (int64_t j = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; j < n_b; j += stride) {
    const int32_t i = b[j];
    const int32_t r = (i >= 0 && i < n) ? label[i] : -1;
    hit = hit || (r >= 0 && r < n && flags[r] != 0);
  }
  if (__any(hit) && (threadIdx.x & 63) == 0) st_dev(result, 1);
}

ccl_status launch_spans(int64_t n, const int32_t* label, int64_t n_a, const int32_t* a, int64_t n_b,
                        const int32_t* b, uint8_t* flags, int32_t* result, hipStream_t s,
                        const DeviceInfo& d) {
  CCL_LAUNCH("ccl_span_clear", k_span_clear, grid_for(n, kSpBlock, 8, d), kSpBlock, 0, s, n, flags,
             result);
  if (n_a > 0 && n_b > 0) {
    CCL_LAUNCH("ccl_span_mark", k_span_mark, grid_for(n_a, kSpBlock, 8, d), kSpBlock, 0, s, n, n_a,
               a, label, flags);
    CCL_LAUNCH("ccl_span_test", k_span_test, grid_for(n_b, kSpBlock, 8, d), kSpBlock, 0, s, n, n_b,
               b, label, flags, result);
  }
  return CCL_OK;
}

}  // namespace ccl
