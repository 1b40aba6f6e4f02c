// Batched labeling: many independent instances in one persistent launch.
//
// Each instance runs the three steps of section 3 -- init (i), the Algorithm 1
// merge over its occupied bonds (iii), flatten (iv) -- split into work items:
//   SMALL    an instance of at most `small_sites` sites, labelled entirely in
//            LDS by one workgroup (init, merge and flatten on the LDS copy,
//            then one coalesced store);
//   INIT c   sites [c*S, (c+1)*S) of a large instance;
//   MERGE c  bonds [c*Bc, (c+1)*Bc), after every INIT item of the instance;
//   FLATTEN c sites [c*S, ...), after every MERGE item of the instance.
// Workgroups take items in table order from one atomic counter.  An item only
// waits for items earlier in the table, which were already taken by running
// workgroups and never wait for later ones, so the schedule cannot deadlock
// whatever the number of resident workgroups.  Waits are bounded anyway: a
// wait that exceeds its spin limit sets an error word and gives up, so every
// wave always exits.
//
// Table order: instances by decreasing size, software-pipelined so that the
// INIT items of instance s, the MERGE items of instance s-1 and the FLATTEN
// items of instance s-2 form stage s; SMALL items come last and fill the tail.
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "uf.hpp"

namespace ccl {

enum : uint32_t { kItemSmall = 0, kItemInit = 1, kItemMerge = 2, kItemFlatten = 3 };

__host__ __device__ inline uint64_t pack_item(uint32_t inst, uint32_t kind, uint32_t chunk) {
  return ((uint64_t)inst << 32) | ((uint64_t)kind << 30) | chunk;
}

struct BatchArgs {
  const int64_t* site_off;
  const int64_t* bond_off;
  const uint64_t* items;
  int64_t n_items;
  uint32_t* head;        // next item to take
  uint32_t* error;       // nonzero: a wait hit its spin limit
  int32_t* init_done;    // per instance: finished INIT items
  int32_t* merge_done;   // per instance: finished MERGE items
  const int32_t* src;
  const int32_t* dst;
  const uint8_t* occ;
  int32_t* label;
  int32_t sites_per_chunk;
  int32_t bonds_per_chunk;
  int32_t small_sites;
  uint32_t spin_limit;
};

__device__ __forceinline__ int32_t n_chunks(int64_t count, int32_t per) {
  return (int32_t)((count + per - 1) / per);
}

// Thread 0 waits until *ctr >= need (acquire), then the workgroup proceeds.
__device__ __forceinline__ void wait_count(const BatchArgs& a, int32_t* ctr, int32_t need) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (++spins > a.spin_limit) {
        __hip_atomic_fetch_or(a.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

// Every thread's stores are ordered before thread 0's release increment by
// the barrier; the release makes them visible device-wide.
__device__ __forceinline__ void signal_done(int32_t* ctr) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_batched_reset(uint32_t* head, uint32_t* error, int32_t* done, int64_t n_done) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) {
    *head = 0;
    *error = 0;
  }
  for (int64_t i = tid; i < n_done; i += stride) done[i] = 0;
}

__global__ void k_batched(BatchArgs a) {
  extern __shared__ int32_t lds[];
  __shared__ uint32_t item_slot;
  for (;;) {
    if (threadIdx.x == 0)
      item_slot = __hip_atomic_fetch_add(a.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t it = item_slot;
    __syncthreads();  // item_slot is rewritten on the next round
    if ((int64_t)it >= a.n_items) break;
    const uint64_t w = a.items[it];
    const uint32_t k = (uint32_t)(w >> 32);
    const uint32_t kind = (uint32_t)(w >> 30) & 3u;
    const int32_t c = (int32_t)(w & 0x3FFFFFFFu);
    const int64_t s0 = a.site_off[k];
    const int32_t n = (int32_t)(a.site_off[k + 1] - s0);
    const int64_t b0 = a.bond_off[k];
    const int64_t m = a.bond_off[k + 1] - b0;
    int32_t* lab = a.label + s0;
    const int32_t* src = a.src + b0;
    const int32_t* dst = a.dst + b0;
    const uint8_t* occ = a.occ ? a.occ + b0 : nullptr;

    if (kind == kItemSmall) {
      for (int32_t i = threadIdx.x; i < n; i += blockDim.x) lds[i] = i;
      __syncthreads();
      for (int64_t b = threadIdx.x; b < m; b += blockDim.x)
        if (occ == nullptr || occ[b] != 0) lds_unite(lds, src[b], dst[b]);
      __syncthreads();
      for (int32_t i = threadIdx.x; i < n; i += blockDim.x) lab[i] = lds_find(lds, i);
      __syncthreads();  // lds is reused by the next item
    } else if (kind == kItemInit) {
      const int32_t lo = c * a.sites_per_chunk;
      const int32_t hi = (int32_t)min((int64_t)lo + a.sites_per_chunk, (int64_t)n);
      for (int32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) lab[i] = i;
      signal_done(a.init_done + k);
    } else if (kind == kItemMerge) {
      wait_count(a, a.init_done + k, n_chunks(n, a.sites_per_chunk));
      const int64_t lo = (int64_t)c * a.bonds_per_chunk;
      const int64_t hi = min(lo + a.bonds_per_chunk, m);
      for (int64_t b = lo + threadIdx.x; b < hi; b += blockDim.x)
        if (occ == nullptr || occ[b] != 0) unite(lab, src[b], dst[b]);
      signal_done(a.merge_done + k);
    } else {
      wait_count(a, a.merge_done + k, n_chunks(m, a.bonds_per_chunk));
      const int32_t lo = c * a.sites_per_chunk;
      const int32_t hi = (int32_t)min((int64_t)lo + a.sites_per_chunk, (int64_t)n);
      for (int32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const int32_t p = lab_ld(lab + i);
        if (p == i) continue;
        const int32_t g = lab_ld(lab + p);
        if (g != p) lab_st(lab + i, find_root(lab, g));
      }
    }
  }
}

}  // namespace ccl

// ---------------------------------------------------------------- plan

struct ccl_plan_s {
  int device = -1;
  int32_t n_inst = 0;
  ccl_tuning tuning{};
  int64_t total_sites = 0, total_bonds = 0;
  int64_t n_items = 0;
  unsigned grid = 0;
  void* dev_block = nullptr;  // one allocation holding every table below
  int64_t* d_site_off = nullptr;
  int64_t* d_bond_off = nullptr;
  uint64_t* d_items = nullptr;
  uint32_t* d_head = nullptr;  // head, error, then the done counters
  int32_t* d_done = nullptr;   // init_done[K], merge_done[K]
};

using namespace ccl;

static ccl_tuning resolve_tuning(const ccl_tuning* t, const DeviceInfo& d) {
  ccl_tuning r{};
  if (t) r = *t;
  if (r.block_threads <= 0) r.block_threads = 512;
  if (r.blocks_per_cu <= 0) r.blocks_per_cu = 4;
  if (r.bonds_per_chunk <= 0) r.bonds_per_chunk = 65536;
  if (r.sites_per_chunk <= 0) r.sites_per_chunk = 32768;
  if (r.small_sites < 0) {
    r.small_sites = 0;  // LDS path off
  } else if (r.small_sites == 0) {
    // one small instance per resident workgroup must fit the CU's LDS
    const int cap = (160 * 1024) / r.blocks_per_cu / 4;
    r.small_sites = std::min(cap, std::min(8192, d.max_lds_per_block / 4));
  }
  return r;
}

static bool tuning_ok(const ccl_tuning& t, const DeviceInfo& d) {
  if (t.block_threads % 64 != 0 || t.block_threads > 1024) return false;
  if (t.blocks_per_cu > 32 || t.bonds_per_chunk <= 0 || t.sites_per_chunk <= 0) return false;
  if ((int64_t)t.small_sites * 4 > d.max_lds_per_block) return false;
  if ((int64_t)t.small_sites * 4 * t.blocks_per_cu > 160 * 1024) return false;
  return true;
}

extern "C" {

ccl_status ccl_plan_create(int32_t n_inst, const int64_t* site_off_host,
                           const int64_t* bond_off_host, const ccl_tuning* tuning,
                           ccl_plan* out) {
  if (out == nullptr || n_inst < 0) return CCL_ERR_INVALID_VALUE;
  *out = nullptr;
  if (site_off_host == nullptr || bond_off_host == nullptr) return CCL_ERR_INVALID_VALUE;
  if (site_off_host[0] != 0 || bond_off_host[0] != 0) return CCL_ERR_INVALID_VALUE;
  for (int32_t k = 0; k < n_inst; ++k) {
    const int64_t n = site_off_host[k + 1] - site_off_host[k];
    const int64_t m = bond_off_host[k + 1] - bond_off_host[k];
    if (n < 0 || n > INT32_MAX || m < 0 || (m > 0 && n == 0)) return CCL_ERR_INVALID_VALUE;
  }
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  const ccl_tuning t = resolve_tuning(tuning, *d);
  if (!tuning_ok(t, *d)) return CCL_ERR_INVALID_VALUE;
  for (int32_t k = 0; k < n_inst; ++k) {  // chunk ids must fit the 30-bit field
    const int64_t n = site_off_host[k + 1] - site_off_host[k];
    const int64_t m = bond_off_host[k + 1] - bond_off_host[k];
    if ((n + t.sites_per_chunk - 1) / t.sites_per_chunk >= (1 << 30) ||
        (m + t.bonds_per_chunk - 1) / t.bonds_per_chunk >= (1 << 30))
      return CCL_ERR_INVALID_VALUE;
  }

  // work-item table
  std::vector<int32_t> order(n_inst);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return site_off_host[x + 1] - site_off_host[x] > site_off_host[y + 1] - site_off_host[y];
  });
  std::vector<int32_t> large, small;
  for (int32_t k : order) {
    const int64_t n = site_off_host[k + 1] - site_off_host[k];
    if (n == 0) continue;
    if (n <= t.small_sites)
      small.push_back(k);
    else
      large.push_back(k);
  }
  std::vector<uint64_t> items;
  const int64_t L = (int64_t)large.size();
  for (int64_t stage = 0; stage < L + 2; ++stage) {
    if (stage < L) {
      const int32_t k = large[stage];
      const int64_t n = site_off_host[k + 1] - site_off_host[k];
      for (int64_t c = 0; c < (n + t.sites_per_chunk - 1) / t.sites_per_chunk; ++c)
        items.push_back(pack_item(k, kItemInit, (uint32_t)c));
    }
    if (stage >= 1 && stage - 1 < L) {
      const int32_t k = large[stage - 1];
      const int64_t m = bond_off_host[k + 1] - bond_off_host[k];
      for (int64_t c = 0; c < (m + t.bonds_per_chunk - 1) / t.bonds_per_chunk; ++c)
        items.push_back(pack_item(k, kItemMerge, (uint32_t)c));
    }
    if (stage >= 2 && stage - 2 < L) {
      const int32_t k = large[stage - 2];
      const int64_t n = site_off_host[k + 1] - site_off_host[k];
      const int64_t m = bond_off_host[k + 1] - bond_off_host[k];
      if (m > 0)
        for (int64_t c = 0; c < (n + t.sites_per_chunk - 1) / t.sites_per_chunk; ++c)
          items.push_back(pack_item(k, kItemFlatten, (uint32_t)c));
    }
  }
  for (int32_t k : small) items.push_back(pack_item(k, kItemSmall, 0));
  if ((int64_t)items.size() >= (int64_t)UINT32_MAX) return CCL_ERR_INVALID_VALUE;

  ccl_plan p = new (std::nothrow) ccl_plan_s();
  if (!p) return CCL_ERR_OUT_OF_MEMORY;
  p->device = d->device;
  p->n_inst = n_inst;
  p->tuning = t;
  p->total_sites = site_off_host[n_inst];
  p->total_bonds = bond_off_host[n_inst];
  p->n_items = (int64_t)items.size();
  p->grid = (unsigned)(d->cu_count * t.blocks_per_cu);

  const size_t off_bytes = sizeof(int64_t) * (size_t)(n_inst + 1);
  const size_t item_bytes = sizeof(uint64_t) * items.size();
  const size_t ctr_bytes = 256 + sizeof(int32_t) * 2 * (size_t)n_inst;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t total = up(off_bytes) * 2 + up(item_bytes) + up(ctr_bytes);
  hipError_t e = hipMalloc(&p->dev_block, total);
  if (e != hipSuccess) {
    delete p;
    return fail_hip(e);
  }
  char* base = static_cast<char*>(p->dev_block);
  p->d_site_off = reinterpret_cast<int64_t*>(base);
  p->d_bond_off = reinterpret_cast<int64_t*>(base + up(off_bytes));
  p->d_items = reinterpret_cast<uint64_t*>(base + 2 * up(off_bytes));
  p->d_head = reinterpret_cast<uint32_t*>(base + 2 * up(off_bytes) + up(item_bytes));
  p->d_done = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(p->d_head) + 256);
  e = hipMemcpy(p->d_site_off, site_off_host, off_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_bond_off, bond_off_host, off_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess && item_bytes)
    e = hipMemcpy(p->d_items, items.data(), item_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p->dev_block);
    delete p;
    return fail_hip(e);
  }
  *out = p;
  return CCL_OK;
}

ccl_status ccl_plan_destroy(ccl_plan plan) {
  if (plan == nullptr) return CCL_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipFree(plan->dev_block);
  delete plan;
  return e == hipSuccess ? CCL_OK : fail_hip(e);
}

ccl_status ccl_plan_get_tuning(ccl_plan plan, ccl_tuning* out) {
  if (plan == nullptr || out == nullptr) return CCL_ERR_INVALID_VALUE;
  *out = plan->tuning;
  return CCL_OK;
}

ccl_status ccl_plan_check(ccl_plan plan, int32_t* error_host) {
  if (plan == nullptr || error_host == nullptr) return CCL_ERR_INVALID_VALUE;
  uint32_t v = 0;
  hipError_t e = hipMemcpy(&v, plan->d_head + 1, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e);
  *error_host = (int32_t)v;
  return CCL_OK;
}

ccl_status ccl_label_batched(ccl_plan plan, const int32_t* src, const int32_t* dst,
                             const uint8_t* occupied, int32_t* labels_out, void* stream) {
  if (plan == nullptr) return CCL_ERR_INVALID_VALUE;
  if (plan->total_bonds > 0 && (src == nullptr || dst == nullptr)) return CCL_ERR_INVALID_VALUE;
  if (plan->total_sites > 0 && labels_out == nullptr) return CCL_ERR_INVALID_VALUE;
  const size_t lb = (size_t)plan->total_sites * 4, bb = (size_t)plan->total_bonds * 4;
  if (overlaps(labels_out, lb, src, bb) || overlaps(labels_out, lb, dst, bb) ||
      overlaps(labels_out, lb, occupied, (size_t)plan->total_bonds))
    return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (d->device != plan->device) return CCL_ERR_INVALID_VALUE;
  if (plan->n_items == 0) return CCL_OK;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n_done = 2 * (int64_t)plan->n_inst;
  CCL_LAUNCH("ccl_batched_reset", k_batched_reset, grid_for(n_done + 1, 256, 4, *d), 256, 0, s,
             plan->d_head, plan->d_head + 1, plan->d_done, n_done);
  BatchArgs a;
  a.site_off = plan->d_site_off;
  a.bond_off = plan->d_bond_off;
  a.items = plan->d_items;
  a.n_items = plan->n_items;
  a.head = plan->d_head;
  a.error = plan->d_head + 1;
  a.init_done = plan->d_done;
  a.merge_done = plan->d_done + plan->n_inst;
  a.src = src;
  a.dst = dst;
  a.occ = occupied;
  a.label = labels_out;
  a.sites_per_chunk = plan->tuning.sites_per_chunk;
  a.bonds_per_chunk = plan->tuning.bonds_per_chunk;
  a.small_sites = plan->tuning.small_sites;
  a.spin_limit = 1u << 22;
  const unsigned lds = (unsigned)plan->tuning.small_sites * 4;
  CCL_LAUNCH("ccl_batched", k_batched, plan->grid, plan->tuning.block_threads, lds, s, a);
  return CCL_OK;
}

ccl_status ccl_label_batched_per_instance(int32_t n_inst, const int64_t* site_off_host,
                                          const int64_t* bond_off_host, const int32_t* src,
                                          const int32_t* dst, const uint8_t* occupied,
                                          int32_t* labels_out, void* stream) {
  if (n_inst < 0 || site_off_host == nullptr || bond_off_host == nullptr)
    return CCL_ERR_INVALID_VALUE;
  for (int32_t k = 0; k < n_inst; ++k) {
    const int64_t s0 = site_off_host[k], b0 = bond_off_host[k];
    ccl_status st = ccl_label(site_off_host[k + 1] - s0, bond_off_host[k + 1] - b0,
                              src ? src + b0 : nullptr, dst ? dst + b0 : nullptr,
                              occupied ? occupied + b0 : nullptr, labels_out + s0, stream);
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

}  // extern "C"
