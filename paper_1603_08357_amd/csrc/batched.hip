// Batched labeling: many independent instances per launch.
//
// Each instance runs the three steps of section 3 -- init (i), the Algorithm 1
// merge over its occupied bonds (iii), flatten (iv) -- split into work items:
//   SMALL     an instance of at most `small_sites` sites, labelled entirely in
//             LDS by one workgroup (init, merge and flatten on a 16-bit LDS
//             parent array, then one coalesced store);
//   INIT c    sites [c*S, (c+1)*S) of a large instance;
//   MERGE c   bonds [c*Bc, (c+1)*Bc), after every INIT item of the instance;
//   FLATTEN c sites [c*S, ...), after every MERGE item of the instance.
// Workgroups of a persistent grid take items from an atomic counter.
//
// Two schedules over the same items:
//   phased : three launches (INIT + SMALL, then MERGE, then FLATTEN); the
//            kernel boundaries order the steps, no workgroup ever waits.
//   fused  : one launch; an item waits for the items of its instance it
//            depends on.  The table puts every such item earlier (instances by
//            decreasing size, software-pipelined: stage s holds the INIT items
//            of instance s, the MERGE items of s-1, the FLATTEN items of s-2;
//            SMALL items last), and items are taken in table order by running
//            workgroups that never wait for later items, so the wait graph
//            cannot deadlock whatever the number of resident workgroups.
//            Publication: every thread fences its own label stores device-wide
//            before the barrier that precedes the counter increment; the
//            waiter takes an acquire fence after seeing the count.
// Fail-safe: waits are bounded; a wait that gives up sets the error word and
// from then on every item skips its work, and root chases in this file reject
// a label that points upward or out of range (impossible for valid labels), so
// the kernel always drains even if a publication went wrong.  The host reads
// the error word with ccl_plan_check().
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "mem.hpp"
#include "tile.hpp"
#include "uf.hpp"

namespace ccl {

enum : uint32_t { kItemSmall = 0, kItemInit = 1, kItemMerge = 2, kItemFlatten = 3 };
constexpr int kLockstep = 4;  // bonds a lane carries through one lockstep join
enum : int32_t { kScheduleDefault = 0, kScheduleFused = 1, kSchedulePhased = 2, kScheduleTiled = 3 };

__host__ __device__ inline uint64_t pack_item(uint32_t inst, uint32_t kind, uint32_t chunk) {
  return ((uint64_t)inst << 32) | ((uint64_t)kind << 30) | chunk;
}

struct BatchArgs {
  const int64_t* site_off;
  const int64_t* bond_off;
  const uint64_t* items;
  int64_t n_items;
  uint32_t* head;        // next item to take
  uint32_t* error;       // nonzero: a wait gave up or a chase met an invalid label
  int32_t* init_done;    // per instance: finished INIT items (fused schedule)
  int32_t* merge_done;   // per instance: finished MERGE items (fused schedule)
  const int32_t* src;
  const int32_t* dst;
  const uint8_t* occ;
  int32_t* label;
  int32_t sites_per_chunk;
  int32_t bonds_per_chunk;
  uint32_t spin_limit;
  int32_t fused;
};

__device__ __forceinline__ int32_t n_chunks(int64_t count, int32_t per) {
  return (int32_t)((count + per - 1) / per);
}

__device__ __forceinline__ void raise_error(uint32_t* error, uint32_t bit) {
  __hip_atomic_fetch_or(error, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fused schedule: thread 0 waits for *ctr >= need; returns false (for the
// whole workgroup) when it gave up or the launch already failed.
__device__ bool wait_count(const BatchArgs& a, int32_t* ctr, int32_t need, uint32_t* ok_slot) {
  if (threadIdx.x == 0) {
    uint32_t ok = 1, spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      if (++spins > a.spin_limit) {
        raise_error(a.error, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *ok_slot = ok;
  }
  __syncthreads();
  return *ok_slot != 0;
}

// Fused schedule: every thread makes its own stores visible device-wide, the
// barrier orders all of them before thread 0's increment.
__device__ __forceinline__ void signal_done(int32_t* ctr) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_batched_reset(uint32_t* head, int64_t n_head, int32_t* done, int64_t n_done) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = tid; i < n_head; i += stride) st_dev(head + i, 0u);
  for (int64_t i = tid; i < n_done; i += stride) st_dev(done + i, 0);
}

__global__ void k_batched(BatchArgs a) {
  extern __shared__ int32_t lds[];
  __shared__ uint32_t item_slot;
  __shared__ uint32_t ok_slot;
  __shared__ uint32_t bad_any;
  for (;;) {
    if (threadIdx.x == 0) {
      item_slot = __hip_atomic_fetch_add(a.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bad_any = 0;
    }
    __syncthreads();
    const uint32_t it = item_slot;
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
    bool bad = false;

    if (kind == kItemSmall) {
      // 16-bit parents (the instance has at most 65536 sites), kLockstep
      // bonds per lane joined in lockstep; (0, 0) is the no-op bond
      uint16_t* par = reinterpret_cast<uint16_t*>(lds);
      for (int32_t w = threadIdx.x; 2 * w < n; w += blockDim.x)
        reinterpret_cast<uint32_t*>(par)[w] = (uint32_t)(2 * w) | ((uint32_t)(2 * w + 1) << 16);
      __syncthreads();
      const int64_t step = (int64_t)kLockstep * blockDim.x;
      for (int64_t b0 = 0; b0 < m; b0 += step) {
        int32_t u[kLockstep], v[kLockstep];
#pragma unroll
        for (int k = 0; k < kLockstep; ++k) {
          const int64_t b = b0 + (int64_t)k * blockDim.x + threadIdx.x;
          const int64_t bc = b < m ? b : 0;  // clamped: loads stay unconditional
          const bool on = b < m && (occ == nullptr || occ[bc] != 0);
          const int32_t x = src[bc], y = dst[bc];
          u[k] = on ? x : 0;
          v[k] = on ? y : 0;
        }
        lds16_unite_lockstep<kLockstep, 2>(par, u, v);
      }
      __syncthreads();
      for (int32_t i = threadIdx.x; i < n; i += blockDim.x) st_dev(lab + i, lds16_find(par, i));
    } else if (kind == kItemInit) {
      const int32_t lo = c * a.sites_per_chunk;
      const int32_t hi = (int32_t)min((int64_t)lo + a.sites_per_chunk, (int64_t)n);
      for (int32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) st_dev(lab + i, i);
      if (a.fused) signal_done(a.init_done + k);
    } else if (kind == kItemMerge) {
      const bool go =
          !a.fused || wait_count(a, a.init_done + k, n_chunks(n, a.sites_per_chunk), &ok_slot);
      if (go) {
        // kLockstep bonds per lane at a time (bond lo + (s*kLockstep + k) *
        // blockDim + tid: each load instruction coalesced), joined in lockstep
        const int64_t lo = (int64_t)c * a.bonds_per_chunk;
        const int64_t hi = min(lo + a.bonds_per_chunk, m);
        const int64_t step = (int64_t)kLockstep * blockDim.x;
        for (int64_t b0 = lo; b0 < hi && !bad; b0 += step) {
          int32_t u[kLockstep], v[kLockstep];
#pragma unroll
          for (int k = 0; k < kLockstep; ++k) {
            const int64_t b = b0 + (int64_t)k * blockDim.x + threadIdx.x;
            const int64_t bc = b < hi ? b : lo;  // clamped: loads stay unconditional
            const bool on = b < hi && (occ == nullptr || occ[bc] != 0);
            const int32_t x = src[bc], y = dst[bc];
            u[k] = on ? x : 0;  // (0, 0) is a no-op
            v[k] = on ? y : 0;
          }
          unite_lockstep<kLockstep, 2, true>(lab, u, v, bad);
        }
      }
      if (a.fused) signal_done(a.merge_done + k);
    } else {
      const bool go =
          !a.fused || wait_count(a, a.merge_done + k, n_chunks(m, a.bonds_per_chunk), &ok_slot);
      if (go) {
        const int32_t lo = c * a.sites_per_chunk;
        const int32_t hi = (int32_t)min((int64_t)lo + a.sites_per_chunk, (int64_t)n);
        // only roots are stored (see the flatten of the single-instance
        // path): the site's own root, and the root into the site's parent.
        // kLockstep sites per lane: their labels and their parents' labels
        // are read together, then the remaining chases advance one link per
        // round while any lane of the wavefront has one.
        constexpr int K = kLockstep;
        for (int32_t i0 = lo; i0 < hi; i0 += K * (int32_t)blockDim.x) {
          int32_t p[K], q[K], x[K], px[K];
          bool need[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int32_t i = i0 + k * (int32_t)blockDim.x + (int32_t)threadIdx.x;
            p[k] = lab_ld(lab + (i < hi ? i : lo));
          }
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int32_t i = i0 + k * (int32_t)blockDim.x + (int32_t)threadIdx.x;
            bool in = i < hi && p[k] != i;
            if (in && (p[k] > i || p[k] < 0)) {
              bad = true;
              in = false;
            }
            q[k] = lab_ld(lab + (in ? p[k] : 0));
            if (in && (q[k] > p[k] || q[k] < 0)) {
              bad = true;
              in = false;
            }
            need[k] = in && q[k] != p[k];
            x[k] = q[k];
            px[k] = lab_ld(lab + (need[k] ? x[k] : 0));
          }
          for (;;) {
            bool open = false;
#pragma unroll
            for (int k = 0; k < K; ++k) {
              if (need[k] && (px[k] > x[k] || px[k] < 0)) {
                bad = true;
                need[k] = false;
              }
              open = open || (need[k] && px[k] != x[k]);
            }
            if (!__any(open)) break;
#pragma unroll
            for (int k = 0; k < K; ++k) {
              // unconditional load (index 0 when idle); an idle chase keeps its value
              const bool go = need[k] && px[k] != x[k];
              x[k] = go ? px[k] : x[k];
              const int32_t nx = lab_ld(lab + (go ? x[k] : 0));
              px[k] = go ? nx : px[k];
            }
          }
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (!need[k]) continue;
            const int32_t i = i0 + k * (int32_t)blockDim.x + (int32_t)threadIdx.x;
            // final roots, which no later kernel of the call writes or updates:
            // plain stores (device-scope ones cost 0.37 ms on the 4096-instance batch)
            if (x[k] != q[k]) lab[p[k]] = x[k];
            lab[i] = x[k];
          }
          if (__any(bad)) break;
        }
      }
    }
    if (bad) bad_any = 1;  // benign race: every writer stores 1
    __syncthreads();       // item_slot, ok_slot, bad_any and lds are rewritten next round
    if (threadIdx.x == 0 && bad_any) raise_error(a.error, 2u);
  }
}

// ---------------------------------------------------------------- tiled schedule
//
// Schedule 3 ("tiled") gives every instance of more than small_sites sites
// the CSR path's treatment on its edge list: tiles of 65536 consecutive
// instance-local sites, one workgroup per tile joining the tile's bonds in LDS
// (16-bit parents), writing the tile's labels (tile-local roots) and listing
// the bonds that leave the tile; then one workgroup per tile joins its listed
// bonds in global memory (Algorithm 1), and the flatten items finish the
// instances of more than one tile.  A tile's bonds are the instance's bonds
// [r_t, r_t+1) with r_0 = 0, r_T = m and r_t = the first bond whose src is at
// least the tile's first site (a binary search, made non-decreasing over t),
// so the ranges partition the bonds: when each instance lists its bonds in
// order of src (as the lattice generators do) a tile's bonds are exactly those
// of its sites; otherwise any bond whose ends are not both in its range's tile
// is simply treated as leaving, and the labels are still exact.
constexpr int kTilePairs = 4096;  // listed leaving bonds per tile; a tile with more re-reads its range
constexpr int32_t kTilePiece = 1 << 28;  // bonds a tile reads through one buffer resource
constexpr int kBatchGroups = 2;           // groups of four bonds per lane per step of the tile stream
constexpr int32_t kBatchTile = kCsrTile;  // sites per tile (16-bit LDS parents)
constexpr int kBatchBlock = kTileBlock;   // threads of a tile workgroup
constexpr int kBatchTilesPerCu = 1;       // resident tile workgroups per compute unit

struct BatchTileArgs {
  const int64_t* site_off;
  const int64_t* bond_off;
  const int4* items;     // (instance, tile, index of the tile's range start, 0)
  const int4* tinst;     // per tiled instance: (instance, first item, tiles, first range index)
  int64_t* ranges;       // per tiled instance: tiles + 1 range bounds, instance-local bond indices
  int32_t* counts;       // per item: leaving bonds listed; -1: the list overflowed
  int2* pairs;           // per item: kTilePairs (src, dst), instance-local
  const int32_t* src;
  const int32_t* dst;
  const uint8_t* occ;
  int32_t* label;
};

// First index b of src[0..m) with src[b] >= x (src sorted in the fast case;
// any array gives some index in [0, m]).
__device__ __forceinline__ int64_t lower_bound_src(const int32_t* src, int64_t m, int32_t x) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (src[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One wavefront per tiled instance: the tiles' range starts in parallel,
// then made non-decreasing with a running maximum (carried across groups of
// 64 tiles).
__global__ void __launch_bounds__(64) k_batched_ranges(BatchTileArgs a) {
  const int4 ti = a.tinst[blockIdx.x];
  const int64_t b0 = a.bond_off[ti.x];
  const int64_t m = a.bond_off[ti.x + 1] - b0;
  const int32_t* src = a.src + b0;
  const int lane = threadIdx.x;
  int64_t* starts = a.ranges + ti.w;  // tiles + 1 bounds
  int64_t carry = 0;
  for (int32_t t0 = 0; t0 < ti.z; t0 += 64) {
    const int32_t t = t0 + lane;
    int64_t r = carry;
    if (t < ti.z && t > 0) r = max(carry, lower_bound_src(src, m, t * kBatchTile));
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(r, d, 64);
      if (lane >= d) r = max(r, o);
    }
    if (t < ti.z) st_dev2(reinterpret_cast<int2*>(starts + t), make_int2((int32_t)(uint32_t)r, (int32_t)(r >> 32)));
    carry = __shfl(r, 63, 64);
  }
  if (lane == 0) st_dev2(reinterpret_cast<int2*>(starts + ti.z), make_int2((int32_t)(uint32_t)m, (int32_t)(m >> 32)));
}

template <bool HAS_OCC>
__global__ void __launch_bounds__(kBatchBlock, kBatchTilesPerCu) k_batched_tile(BatchTileArgs a) {
  __shared__ uint16_t par[kBatchTile];
  __shared__ uint32_t stage[kBatchBlock / 64][kStageCap];
  __shared__ uint32_t n_out;
  const int tid = threadIdx.x, wave = tid >> 6;
  const int4 it = a.items[blockIdx.x];
  const int64_t s0 = a.site_off[it.x];
  const int32_t n = (int32_t)(a.site_off[it.x + 1] - s0);
  const int32_t lo = it.y * kBatchTile;
  const int32_t cnt = min(kBatchTile, n - lo);
  const int64_t b0 = a.bond_off[it.x];
  const int64_t r0 = a.ranges[it.z], r1 = a.ranges[it.z + 1];
  const int64_t nb = r1 - r0;
  const int32_t* src = a.src + b0 + r0;
  const int32_t* dst = a.dst + b0 + r0;
  const uint8_t* occ = HAS_OCC ? a.occ + b0 + r0 : nullptr;
  int2* my_pairs = a.pairs + (int64_t)blockIdx.x * kTilePairs;
  int32_t* lab = a.label + s0;
  for (int w = tid; w < kBatchTile / 8; w += kBatchBlock) {
    const uint32_t t = 8u * (uint32_t)w;
    reinterpret_cast<uint4*>(par)[w] =
        make_uint4(t | ((t + 1) << 16), (t + 2) | ((t + 3) << 16), (t + 4) | ((t + 5) << 16), (t + 6) | ((t + 7) << 16));
  }
  if (tid == 0) n_out = 0;
  __syncthreads();
  // bonds in groups of four per lane (buffer loads: an offset past the range
  // reads 0, which the per-bond bound below masks), staged joins as in the
  // CSR tile kernel, leaving occupied bonds listed; the range is read in
  // pieces of at most 2^28 bonds, so byte offsets fit the 32-bit resources
  const bool occ4 = ((reinterpret_cast<uintptr_t>(occ) & 3) == 0);
  uint32_t staged = 0;
  constexpr int G = kBatchGroups;
  for (int64_t c0 = 0; c0 < nb; c0 += kTilePiece) {
    const int64_t pn = min((int64_t)kTilePiece, nb - c0);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src + c0, (uint32_t)pn * 4u);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst + c0, (uint32_t)pn * 4u);
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(HAS_OCC ? occ + c0 : nullptr, HAS_OCC ? (uint32_t)pn : 0u);
    const int32_t groups = (int32_t)((pn + 3) >> 2);
    const int32_t iters = (groups + G * kBatchBlock - 1) / (G * kBatchBlock);
    // group g of step k, slot i: g = (G k + i) kBatchBlock + tid.  A load that
    // reaches past the range's end is range-checked as a whole, so the one
    // group that straddles the end loads word by word.
    auto load = [&](int32_t k, int i, int4& u4, int4& v4, uint32_t& o4) {
      const int32_t g = (G * k + i) * kBatchBlock + tid;
      const bool whole = 4 * (int64_t)g + 4 <= pn;
      const uint32_t off = whole ? 4u * (uint32_t)g : kOffNone;
      u4 = buf_i32x4(rs, off * 4u);
      v4 = buf_i32x4(rd, off * 4u);
      o4 = 0x01010101u;
      if (HAS_OCC) {
        if (occ4) {
          o4 = buf_u32(ro, off);
        } else {
          o4 = buf_u8(ro, off) | (buf_u8(ro, off + 1u) << 8) | (buf_u8(ro, off + 2u) << 16) | (buf_u8(ro, off + 3u) << 24);
        }
      }
      if (!whole && g < groups) {
        const uint32_t t0 = 4u * (uint32_t)g;
        u4 = make_int4(buf_i32(rs, 4u * t0), buf_i32(rs, 4u * t0 + 4u), buf_i32(rs, 4u * t0 + 8u), buf_i32(rs, 4u * t0 + 12u));
        v4 = make_int4(buf_i32(rd, 4u * t0), buf_i32(rd, 4u * t0 + 4u), buf_i32(rd, 4u * t0 + 8u), buf_i32(rd, 4u * t0 + 12u));
        if (HAS_OCC)
          o4 = buf_u8(ro, t0) | (buf_u8(ro, t0 + 1u) << 8) | (buf_u8(ro, t0 + 2u) << 16) | (buf_u8(ro, t0 + 3u) << 24);
      }
    };
    int4 cu[G], cv[G], nu[G], nv[G];
    uint32_t co[G], no[G];
#pragma unroll
    for (int i = 0; i < G; ++i) load(0, i, cu[i], cv[i], co[i]);
    for (int32_t k = 0; k < iters; ++k) {
      // the next step's loads go out before this step's joins
      if (k + 1 < iters) {
#pragma unroll
        for (int i = 0; i < G; ++i) load(k + 1, i, nu[i], nv[i], no[i]);
      }
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int32_t g = (G * k + i) * kBatchBlock + tid;
        const int32_t u[4] = {cu[i].x, cu[i].y, cu[i].z, cu[i].w};
        const int32_t v[4] = {cv[i].x, cv[i].y, cv[i].z, cv[i].w};
        uint32_t act = 0, leave = 0;
        uint32_t packed[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool on = 4 * (int64_t)g + j < pn && ((co[i] >> (8 * j)) & 0xFFu) != 0;
          const uint32_t ul = (uint32_t)(u[j] - lo), vl = (uint32_t)(v[j] - lo);
          const bool inside = ul < (uint32_t)cnt && vl < (uint32_t)cnt;
          act |= (uint32_t)(on && inside) << j;
          leave |= (uint32_t)(on && !inside && u[j] != v[j]) << j;
          packed[j] = (ul << 16) | (vl & 0xFFFFu);
        }
        tile_join_compact(par, stage[wave], staged, act, packed);
        uint32_t slot = reserve_slots<3>(__popc(leave), &n_out);
        if (leave) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if ((leave >> j) & 1u) {
              if (slot < (uint32_t)kTilePairs) st_dev2(my_pairs + slot, make_int2(u[j], v[j]));
              ++slot;
            }
        }
      }
#pragma unroll
      for (int i = 0; i < G; ++i) {
        cu[i] = nu[i];
        cv[i] = nv[i];
        co[i] = no[i];
      }
    }
  }
  drain_joins(par, stage[wave], staged);
  __syncthreads();
  // the tile's labels (instance-local): each site's tile-local root.  A
  // pass takes two runs of 4 kBatchBlock consecutive sites, four per lane,
  // all eight chases in lockstep rounds; 16-byte device-scope stores when
  // the tile's labels are 16-byte aligned.  In an instance of several tiles
  // a site deeper than six links keeps the ancestor the lockstep rounds
  // reached, which the leaving-bond joins and the flatten follow (a check
  // and a divergent chase to the root there cost 1.3 ms of the 4096-instance
  // batch's tile kernel and saved 1.0 ms of its flatten).
  {
    const bool single = n <= kBatchTile;
    constexpr int32_t kRun = 4 * kBatchBlock;
    const int32_t n_runs = (cnt + kRun - 1) / kRun;
    const bool vec = (reinterpret_cast<uintptr_t>(lab + lo) & 15) == 0;
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(lab + lo, vec ? (uint32_t)cnt * 4u : 0u);
    for (int32_t q0 = 0; q0 < n_runs; q0 += 2) {
      int32_t x[8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int32_t t0 = min(q0 + h, n_runs - 1) * kRun + 4 * tid;  // a missing run repeats the last
        const int32_t t = t0 < cnt ? t0 : 0;                          // past the tile: slot 0
        const uint2 wv = reinterpret_cast<const uint2*>(par)[t >> 2];
        x[4 * h + 0] = (int32_t)(wv.x & 0xFFFFu);
        x[4 * h + 1] = (int32_t)(wv.x >> 16);
        x[4 * h + 2] = (int32_t)(wv.y & 0xFFFFu);
        x[4 * h + 3] = (int32_t)(wv.y >> 16);
      }
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = lds16_ld(par + x[k]);  // a root reads itself
      if (single) {  // an instance of one tile has no later kernel: its labels must be roots
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int32_t p = lds16_ld(par + x[k]);
          if (p != x[k]) x[k] = lds16_find(par, x[k]);  // the rare longer chain
        }
      } else {  // two more lockstep rounds (fewer left to the flatten; measured best)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int k = 0; k < 8; ++k) x[k] = lds16_ld(par + x[k]);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int32_t t = (q0 + h) * kRun + 4 * tid;
        if (q0 + h >= n_runs || t >= cnt) continue;
        if (vec && t + 4 <= cnt) {
          st_dev4(rl, 4u * (uint32_t)t, make_int4(lo + x[4 * h], lo + x[4 * h + 1], lo + x[4 * h + 2], lo + x[4 * h + 3]));
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (t + k < cnt) st_dev(lab + lo + t + k, lo + x[4 * h + k]);
        }
      }
    }
  }
  if (tid == 0)
    st_dev(a.counts + blockIdx.x, n_out > (uint32_t)kTilePairs ? -1 : (int32_t)n_out);
}

// One workgroup per tile: the listed leaving bonds joined in global memory,
// one per lane in lockstep; a tile whose list overflowed reads its bond range
// again and joins every occupied bond that is not inside the tile.
__global__ void __launch_bounds__(512) k_batched_cross(BatchTileArgs a) {
  const int4 it = a.items[blockIdx.x];
  const int64_t s0 = a.site_off[it.x];
  const int32_t n = (int32_t)(a.site_off[it.x + 1] - s0);
  const int32_t lo = it.y * kBatchTile;
  const int32_t cnt = min(kBatchTile, n - lo);
  int32_t* lab = a.label + s0;
  const int32_t count = a.counts[blockIdx.x];
  bool unused = false;
  if (count >= 0) {
    const int2* p = a.pairs + (int64_t)blockIdx.x * kTilePairs;
    for (int32_t j0 = 0; j0 < count; j0 += 512) {
      const int32_t j = j0 + threadIdx.x;
      const int2 e = p[j < count ? j : 0];
      int32_t x[1] = {j < count ? e.x : 0}, y[1] = {j < count ? e.y : 0};
      unite_lockstep<1, 2, false>(lab, x, y, unused);
    }
    return;
  }
  // the list overflowed: the range is read again and every occupied bond
  // that is not inside the tile (those were joined in LDS) is joined here
  const int64_t b0 = a.bond_off[it.x];
  const int64_t r0 = a.ranges[it.z], r1 = a.ranges[it.z + 1];
  for (int64_t b = r0 + threadIdx.x; b < r1; b += 512) {
    if (a.occ && a.occ[b0 + b] == 0) continue;
    const int32_t u = a.src[b0 + b], v = a.dst[b0 + b];
    if ((uint32_t)(u - lo) < (uint32_t)cnt && (uint32_t)(v - lo) < (uint32_t)cnt) continue;
    unite(lab, u, v);
  }
}

}  // namespace ccl

// ---------------------------------------------------------------- plan

// Device tables of a plan, sized for capacities: a plan made for one layout
// has exactly that layout's sizes; a capacity plan has bounds that any
// layout within its limits fits, and takes a new layout per launch.
struct PlanCaps {
  int32_t inst = 0;
  int64_t items = 0, tiles = 0, tiled = 0, ranges = 0;
};

struct ccl_plan_s {
  int device = -1;
  ccl_tuning tuning{};
  PlanCaps cap;
  int64_t max_sites = 0, max_bonds = 0;  // capacity plans: the limits a layout must keep
  bool reusable = false;
  // the current layout
  int32_t n_inst = 0;
  int64_t total_sites = 0, total_bonds = 0;
  int64_t n_items = 0;
  int64_t phase_end[3] = {0, 0, 0};  // phased schedule: items [end[p-1], end[p]) form phase p
  int64_t n_tiles = 0;               // tiled schedule: tile items
  int32_t n_tiled = 0;               // instances split into tiles
  unsigned grid = 0;
  void* dev_block = nullptr;  // one allocation holding every table below
  int64_t* d_site_off = nullptr;
  int64_t* d_bond_off = nullptr;
  uint64_t* d_items = nullptr;
  int4* d_tiles = nullptr;    // (instance, tile, range index, 0)
  int4* d_tinst = nullptr;    // (instance, first tile item, tiles, first range index)
  uint32_t* d_ctl = nullptr;  // [0..2] queue heads, [3] error word
  int32_t* d_done = nullptr;  // init_done[K], merge_done[K]
  int64_t* d_ranges = nullptr;
  int32_t* d_counts = nullptr;
  int2* d_pairs = nullptr;
  // capacity plans: pinned staging of the uploaded tables, and the event of
  // the last upload (the staging is rewritten only after it has been read)
  char* stage = nullptr;
  hipEvent_t staged = nullptr;
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
    // one small instance per resident workgroup must fit the CU's LDS (two
    // bytes per site)
    const int cap = (160 * 1024) / r.blocks_per_cu / 2 - 128;
    r.small_sites = std::min(cap, std::min(16384, d.max_lds_per_block / 2 - 128));
  }
  if (r.schedule == kScheduleDefault) r.schedule = kScheduleTiled;
  return r;
}

// LDS a SMALL item takes: 16-bit parents, whole 32-bit words
static int64_t small_lds_bytes(const ccl_tuning& t) {
  return ((int64_t)std::max(t.small_sites, 0) + 1) / 2 * 4;
}

static bool tuning_ok(const ccl_tuning& t, const DeviceInfo& d) {
  if (t.block_threads % 64 != 0 || t.block_threads > 1024) return false;
  if (t.blocks_per_cu > 32 || t.bonds_per_chunk <= 0 || t.sites_per_chunk <= 0) return false;
  if (t.small_sites > 65536) return false;  // 16-bit LDS parents
  if (small_lds_bytes(t) + 64 > d.max_lds_per_block) return false;
  if ((small_lds_bytes(t) + 64) * t.blocks_per_cu > 160 * 1024) return false;
  if (t.schedule != kScheduleFused && t.schedule != kSchedulePhased && t.schedule != kScheduleTiled)
    return false;
  return true;
}

// The host tables of one layout.
struct PlanTables {
  std::vector<uint64_t> items;
  int64_t phase_end[3] = {0, 0, 0};
  std::vector<int4> tile_items, tiled;
  int64_t n_ranges = 0;
};

// Offsets start at 0, never decrease, instances fit int32 ids, and an
// instance with bonds has sites (checked before any device call).
static ccl_status check_offsets(int32_t n_inst, const int64_t* so, const int64_t* bo) {
  if (n_inst < 0 || so == nullptr || bo == nullptr) return CCL_ERR_INVALID_VALUE;
  if (so[0] != 0 || bo[0] != 0) return CCL_ERR_INVALID_VALUE;
  for (int32_t k = 0; k < n_inst; ++k) {
    const int64_t n = so[k + 1] - so[k];
    const int64_t m = bo[k + 1] - bo[k];
    if (n < 0 || n > INT32_MAX || m < 0 || (m > 0 && n == 0)) return CCL_ERR_INVALID_VALUE;
  }
  return CCL_OK;
}

// Chunk ids must fit the 30-bit field of a work item.
static ccl_status check_chunks(int32_t n_inst, const int64_t* so, const int64_t* bo, const ccl_tuning& t) {
  for (int32_t k = 0; k < n_inst; ++k) {
    const int64_t n = so[k + 1] - so[k];
    const int64_t m = bo[k + 1] - bo[k];
    if ((n + t.sites_per_chunk - 1) / t.sites_per_chunk >= (1 << 30) ||
        (m + t.bonds_per_chunk - 1) / t.bonds_per_chunk >= (1 << 30))
      return CCL_ERR_INVALID_VALUE;
  }
  return CCL_OK;
}

static ccl_status build_tables(const ccl_tuning& t, int32_t n_inst, const int64_t* so,
                               const int64_t* bo, PlanTables& pt) {
  // instances by decreasing size; small ones are labelled in LDS
  std::vector<int32_t> order(n_inst);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return so[x + 1] - so[x] > so[y + 1] - so[y];
  });
  std::vector<int32_t> large, small;
  for (int32_t k : order) {
    const int64_t n = so[k + 1] - so[k];
    if (n == 0) continue;
    (n <= t.small_sites ? small : large).push_back(k);
  }
  auto n_init = [&](int32_t k) { return (so[k + 1] - so[k] + t.sites_per_chunk - 1) / t.sites_per_chunk; };
  auto n_merge = [&](int32_t k) { return (bo[k + 1] - bo[k] + t.bonds_per_chunk - 1) / t.bonds_per_chunk; };
  auto emit = [](std::vector<uint64_t>& v, int32_t k, uint32_t kind, int64_t count) {
    for (int64_t c = 0; c < count; ++c) v.push_back(pack_item(k, kind, (uint32_t)c));
  };
  std::vector<uint64_t>& items = pt.items;
  int64_t* phase_end = pt.phase_end;
  if (t.schedule == kScheduleTiled) {
    // phase 1: SMALL items (the tile items run in their own launch); phase 3:
    // FLATTEN items of the instances of more than one tile
    for (int32_t k : small) emit(items, k, kItemSmall, 1);
    phase_end[0] = phase_end[1] = (int64_t)items.size();
    for (int32_t k : large) {
      const int64_t n = so[k + 1] - so[k];
      const int32_t nt = (int32_t)((n + kBatchTile - 1) / kBatchTile);
      pt.tiled.push_back(make_int4(k, (int32_t)pt.tile_items.size(), nt, (int32_t)pt.n_ranges));
      for (int32_t tt = 0; tt < nt; ++tt) pt.tile_items.push_back(make_int4(k, tt, (int32_t)(pt.n_ranges + tt), 0));
      pt.n_ranges += nt + 1;
      if (nt > 1) emit(items, k, kItemFlatten, n_init(k));
    }
    phase_end[2] = (int64_t)items.size();
    if ((int64_t)pt.tile_items.size() >= INT32_MAX || pt.n_ranges >= INT32_MAX) return CCL_ERR_INVALID_VALUE;
  } else if (t.schedule == kScheduleFused) {
    const int64_t L = (int64_t)large.size();
    for (int64_t s = 0; s < L + 2; ++s) {
      if (s < L) emit(items, large[s], kItemInit, n_init(large[s]));
      if (s >= 1 && s - 1 < L) emit(items, large[s - 1], kItemMerge, n_merge(large[s - 1]));
      if (s >= 2 && s - 2 < L && n_merge(large[s - 2]) > 0)
        emit(items, large[s - 2], kItemFlatten, n_init(large[s - 2]));
    }
    for (int32_t k : small) emit(items, k, kItemSmall, 1);
    phase_end[0] = phase_end[1] = phase_end[2] = (int64_t)items.size();
  } else {
    for (int32_t k : large) emit(items, k, kItemInit, n_init(k));
    for (int32_t k : small) emit(items, k, kItemSmall, 1);
    phase_end[0] = (int64_t)items.size();
    for (int32_t k : large) emit(items, k, kItemMerge, n_merge(k));
    phase_end[1] = (int64_t)items.size();
    for (int32_t k : large)
      if (n_merge(k) > 0) emit(items, k, kItemFlatten, n_init(k));
    phase_end[2] = (int64_t)items.size();
  }
  if ((int64_t)items.size() >= (int64_t)UINT32_MAX) return CCL_ERR_INVALID_VALUE;
  return CCL_OK;
}

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the tables in the device block (and, for the first five,
// in the pinned staging of a capacity plan).
struct PlanLayout {
  size_t site_off, bond_off, items, tiles, tinst, upload_end, ctl, ranges, counts, pairs, total;
};

static PlanLayout plan_layout(const PlanCaps& c) {
  PlanLayout L{};
  size_t o = 0;
  const size_t off_bytes = up256(sizeof(int64_t) * (size_t)(c.inst + 1));
  L.site_off = o;
  o += off_bytes;
  L.bond_off = o;
  o += off_bytes;
  L.items = o;
  o += up256(sizeof(uint64_t) * (size_t)c.items);
  L.tiles = o;
  o += up256(sizeof(int4) * (size_t)c.tiles);
  L.tinst = o;
  o += up256(sizeof(int4) * (size_t)c.tiled);
  L.upload_end = o;
  L.ctl = o;
  o += up256(256 + sizeof(int32_t) * 2 * (size_t)c.inst);
  L.ranges = o;
  o += up256(sizeof(int64_t) * (size_t)c.ranges);
  L.counts = o;
  o += up256(sizeof(int32_t) * (size_t)c.tiles);
  L.pairs = o;
  o += sizeof(int2) * (size_t)kTilePairs * (size_t)c.tiles;
  L.total = o;
  return L;
}

// Allocates the device block (and for capacity plans the staging and its
// event) and points the plan's tables into it.
static ccl_status plan_alloc(ccl_plan p) {
  const PlanLayout L = plan_layout(p->cap);
  hipError_t e = hipMalloc(&p->dev_block, L.total);
  if (e != hipSuccess) return fail_hip(e);
  char* b = static_cast<char*>(p->dev_block);
  p->d_site_off = reinterpret_cast<int64_t*>(b + L.site_off);
  p->d_bond_off = reinterpret_cast<int64_t*>(b + L.bond_off);
  p->d_items = reinterpret_cast<uint64_t*>(b + L.items);
  p->d_tiles = reinterpret_cast<int4*>(b + L.tiles);
  p->d_tinst = reinterpret_cast<int4*>(b + L.tinst);
  p->d_ctl = reinterpret_cast<uint32_t*>(b + L.ctl);
  p->d_done = reinterpret_cast<int32_t*>(b + L.ctl + 256);
  p->d_ranges = reinterpret_cast<int64_t*>(b + L.ranges);
  p->d_counts = reinterpret_cast<int32_t*>(b + L.counts);
  p->d_pairs = reinterpret_cast<int2*>(b + L.pairs);
  e = hipMemset(b + L.ctl, 0, L.ranges - L.ctl);
  if (e == hipSuccess && p->reusable) {
    e = hipHostMalloc(reinterpret_cast<void**>(&p->stage), L.upload_end, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e == hipSuccess ? CCL_OK : fail_hip(e);
}

static void plan_free(ccl_plan p) {
  if (p->staged) (void)hipEventDestroy(p->staged);
  if (p->stage) (void)hipHostFree(p->stage);
  if (p->dev_block) (void)hipFree(p->dev_block);
  delete p;
}

static void plan_take_layout(ccl_plan p, int32_t n_inst, const int64_t* so, const int64_t* bo,
                             const PlanTables& pt) {
  p->n_inst = n_inst;
  p->total_sites = so[n_inst];
  p->total_bonds = bo[n_inst];
  p->n_items = (int64_t)pt.items.size();
  for (int i = 0; i < 3; ++i) p->phase_end[i] = pt.phase_end[i];
  p->n_tiles = (int64_t)pt.tile_items.size();
  p->n_tiled = (int32_t)pt.tiled.size();
}

static bool fits(const PlanCaps& c, int32_t n_inst, const PlanTables& pt) {
  return n_inst <= c.inst && (int64_t)pt.items.size() <= c.items && (int64_t)pt.tile_items.size() <= c.tiles &&
         (int64_t)pt.tiled.size() <= c.tiled && pt.n_ranges <= c.ranges;
}

extern "C" {

ccl_status ccl_plan_create(int32_t n_inst, const int64_t* site_off_host,
                           const int64_t* bond_off_host, const ccl_tuning* tuning,
                           ccl_plan* out) {
  if (out == nullptr || n_inst < 0) return CCL_ERR_INVALID_VALUE;
  *out = nullptr;
  ccl_status st = check_offsets(n_inst, site_off_host, bond_off_host);
  if (st != CCL_OK) return st;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  const ccl_tuning t = resolve_tuning(tuning, *d);
  if (!tuning_ok(t, *d)) return CCL_ERR_INVALID_VALUE;
  st = check_chunks(n_inst, site_off_host, bond_off_host, t);
  if (st != CCL_OK) return st;
  PlanTables pt;
  st = build_tables(t, n_inst, site_off_host, bond_off_host, pt);
  if (st != CCL_OK) return st;

  ccl_plan p = new (std::nothrow) ccl_plan_s();
  if (!p) return CCL_ERR_OUT_OF_MEMORY;
  p->device = d->device;
  p->tuning = t;
  p->grid = (unsigned)(d->cu_count * t.blocks_per_cu);
  p->cap.inst = n_inst;
  p->cap.items = (int64_t)pt.items.size();
  p->cap.tiles = (int64_t)pt.tile_items.size();
  p->cap.tiled = (int64_t)pt.tiled.size();
  p->cap.ranges = pt.n_ranges;
  p->max_sites = site_off_host[n_inst];
  p->max_bonds = bond_off_host[n_inst];
  st = plan_alloc(p);
  if (st != CCL_OK) {
    plan_free(p);
    return st;
  }
  plan_take_layout(p, n_inst, site_off_host, bond_off_host, pt);
  const size_t ob = sizeof(int64_t) * (size_t)(n_inst + 1);
  hipError_t e = hipMemcpy(p->d_site_off, site_off_host, ob, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_bond_off, bond_off_host, ob, hipMemcpyHostToDevice);
  if (e == hipSuccess && !pt.items.empty())
    e = hipMemcpy(p->d_items, pt.items.data(), sizeof(uint64_t) * pt.items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pt.tile_items.empty())
    e = hipMemcpy(p->d_tiles, pt.tile_items.data(), sizeof(int4) * pt.tile_items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pt.tiled.empty())
    e = hipMemcpy(p->d_tinst, pt.tiled.data(), sizeof(int4) * pt.tiled.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    plan_free(p);
    return fail_hip(e);
  }
  *out = p;
  return CCL_OK;
}

ccl_status ccl_plan_create_capacity(int32_t max_inst, int64_t max_sites, int64_t max_bonds,
                                    const ccl_tuning* tuning, ccl_plan* out) {
  if (out == nullptr) return CCL_ERR_INVALID_VALUE;
  *out = nullptr;
  if (max_inst < 0 || max_sites < 0 || max_bonds < 0) return CCL_ERR_INVALID_VALUE;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (!d->is_gfx950) return CCL_ERR_NOT_SUPPORTED;
  const ccl_tuning t = resolve_tuning(tuning, *d);
  if (!tuning_ok(t, *d)) return CCL_ERR_INVALID_VALUE;
  // bounds over every layout of at most max_inst instances, max_sites sites
  // and max_bonds bonds: an instance adds at most one partial chunk or tile
  // to each count, and only instances above small_sites sites are tiled
  const int64_t spc = t.sites_per_chunk, bpc = t.bonds_per_chunk;
  PlanCaps c;
  c.inst = max_inst;
  c.items = 2 * ((max_sites + spc - 1) / spc) + (max_bonds + bpc - 1) / bpc + 4 * (int64_t)max_inst;
  if (t.schedule == kScheduleTiled) {
    c.tiled = std::min<int64_t>(max_inst, max_sites / ((int64_t)t.small_sites + 1));
    c.tiles = (max_sites + kBatchTile - 1) / kBatchTile + c.tiled;
    c.ranges = c.tiles + c.tiled;
  }
  if (c.items >= (int64_t)UINT32_MAX || c.tiles >= INT32_MAX || c.ranges >= INT32_MAX)
    return CCL_ERR_TOO_LARGE;
  ccl_plan p = new (std::nothrow) ccl_plan_s();
  if (!p) return CCL_ERR_OUT_OF_MEMORY;
  p->device = d->device;
  p->tuning = t;
  p->grid = (unsigned)(d->cu_count * t.blocks_per_cu);
  p->cap = c;
  p->max_sites = max_sites;
  p->max_bonds = max_bonds;
  p->reusable = true;
  const ccl_status st = plan_alloc(p);
  if (st != CCL_OK) {
    plan_free(p);
    return st;
  }
  *out = p;  // empty layout: ccl_label_batched does nothing until one is set
  return CCL_OK;
}

ccl_status ccl_plan_set_layout(ccl_plan plan, int32_t n_inst, const int64_t* site_off_host,
                               const int64_t* bond_off_host, void* stream) {
  if (plan == nullptr || !plan->reusable) return CCL_ERR_INVALID_VALUE;
  ccl_status st = check_offsets(n_inst, site_off_host, bond_off_host);
  if (st != CCL_OK) return st;
  const DeviceInfo* d = current_device();
  if (!d) return CCL_ERR_HIP;
  if (d->device != plan->device) return CCL_ERR_INVALID_VALUE;
  st = check_chunks(n_inst, site_off_host, bond_off_host, plan->tuning);
  if (st != CCL_OK) return st;
  if (site_off_host[n_inst] > plan->max_sites || bond_off_host[n_inst] > plan->max_bonds ||
      n_inst > plan->cap.inst)
    return CCL_ERR_TOO_LARGE;
  PlanTables pt;
  st = build_tables(plan->tuning, n_inst, site_off_host, bond_off_host, pt);
  if (st != CCL_OK) return st;
  if (!fits(plan->cap, n_inst, pt)) return CCL_ERR_TOO_LARGE;
  // the previous upload has read the staging before it is rewritten
  hipError_t e = hipEventSynchronize(plan->staged);
  if (e != hipSuccess) return fail_hip(e);
  const PlanLayout L = plan_layout(plan->cap);
  const size_t ob = sizeof(int64_t) * (size_t)(n_inst + 1);
  struct Part {
    size_t off, bytes;
    const void* src;
  } parts[5] = {{L.site_off, ob, site_off_host},
                {L.bond_off, ob, bond_off_host},
                {L.items, sizeof(uint64_t) * pt.items.size(), pt.items.data()},
                {L.tiles, sizeof(int4) * pt.tile_items.size(), pt.tile_items.data()},
                {L.tinst, sizeof(int4) * pt.tiled.size(), pt.tiled.data()}};
  hipStream_t s = (hipStream_t)stream;
  char* dev = static_cast<char*>(plan->dev_block);
  for (const Part& q : parts) {
    if (q.bytes == 0) continue;
    std::memcpy(plan->stage + q.off, q.src, q.bytes);
    e = hipMemcpyAsync(dev + q.off, plan->stage + q.off, q.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e);
  }
  e = hipEventRecord(plan->staged, s);
  if (e != hipSuccess) return fail_hip(e);
  plan_take_layout(plan, n_inst, site_off_host, bond_off_host, pt);
  return CCL_OK;
}

ccl_status ccl_plan_destroy(ccl_plan plan) {
  if (plan == nullptr) return CCL_OK;
  hipError_t e = hipDeviceSynchronize();
  plan_free(plan);
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
  hipError_t e = hipMemcpy(&v, plan->d_ctl + 3, sizeof(v), hipMemcpyDeviceToHost);
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
  if (plan->n_items == 0 && plan->n_tiles == 0) return CCL_OK;
  hipStream_t s = (hipStream_t)stream;
  const bool fused = plan->tuning.schedule == kScheduleFused;
  const int64_t n_done = fused ? 2 * (int64_t)plan->n_inst : 0;
  CCL_LAUNCH("ccl_batched_reset", k_batched_reset, grid_for(n_done + 4, 256, 4, *d), 256, 0, s,
             plan->d_ctl, (int64_t)4, plan->d_done, n_done);
  BatchArgs a;
  a.site_off = plan->d_site_off;
  a.bond_off = plan->d_bond_off;
  a.error = plan->d_ctl + 3;
  a.init_done = plan->d_done;
  a.merge_done = plan->d_done + plan->n_inst;
  a.src = src;
  a.dst = dst;
  a.occ = occupied;
  a.label = labels_out;
  a.sites_per_chunk = plan->tuning.sites_per_chunk;
  a.bonds_per_chunk = plan->tuning.bonds_per_chunk;
  a.spin_limit = 1u << 20;
  a.fused = fused ? 1 : 0;
  const unsigned lds = (unsigned)small_lds_bytes(plan->tuning);
  if (fused) {
    a.items = plan->d_items;
    a.n_items = plan->n_items;
    a.head = plan->d_ctl;
    CCL_LAUNCH("ccl_batched_fused", k_batched, plan->grid, plan->tuning.block_threads, lds, s, a);
    return CCL_OK;
  }
  static const char* names[3] = {"ccl_batched_init", "ccl_batched_merge", "ccl_batched_flatten"};
  BatchTileArgs ta;
  ta.site_off = plan->d_site_off;
  ta.bond_off = plan->d_bond_off;
  ta.items = plan->d_tiles;
  ta.tinst = plan->d_tinst;
  ta.ranges = plan->d_ranges;
  ta.counts = plan->d_counts;
  ta.pairs = plan->d_pairs;
  ta.src = src;
  ta.dst = dst;
  ta.occ = occupied;
  ta.label = labels_out;
  const bool tiled = plan->tuning.schedule == kScheduleTiled;
  if (tiled && plan->n_tiled > 0)
    CCL_LAUNCH("ccl_batched_ranges", k_batched_ranges, (unsigned)plan->n_tiled, 64, 0, s, ta);
  int64_t begin = 0;
  for (int ph = 0; ph < 3; ++ph) {
    a.items = plan->d_items + begin;
    a.n_items = plan->phase_end[ph] - begin;
    a.head = plan->d_ctl + ph;
    begin = plan->phase_end[ph];
    if (a.n_items > 0) {
      const unsigned g = (unsigned)std::min<int64_t>(plan->grid, a.n_items);
      CCL_LAUNCH(names[ph], k_batched, g, plan->tuning.block_threads, ph == 0 ? lds : 0, s, a);
    }
    if (tiled && plan->n_tiles > 0 && ph == 0) {
      if (occupied)
        CCL_LAUNCH("ccl_batched_tile", k_batched_tile<true>, (unsigned)plan->n_tiles, kBatchBlock, 0, s, ta);
      else
        CCL_LAUNCH("ccl_batched_tile", k_batched_tile<false>, (unsigned)plan->n_tiles, kBatchBlock, 0, s, ta);
    }
    if (tiled && plan->n_tiles > 0 && ph == 1)
      CCL_LAUNCH("ccl_batched_cross", k_batched_cross, (unsigned)plan->n_tiles, 512, 0, s, ta);
  }
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
