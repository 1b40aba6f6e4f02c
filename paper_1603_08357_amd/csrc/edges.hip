// Edge-list labeling: init (step i), bond-parallel merge (step iii,
// Algorithm 1), flatten (step iv).  Paper, section 3.
#include "common.hpp"
#include "mem.hpp"
#include "philox.hpp"
#include "uf.hpp"

namespace ccl {

constexpr int kBlock = 256;

// Step (i) with every residual list taken as empty: label[i] = i.
// VEC: label is 16-byte aligned and written four ids at a time.
template <bool VEC>
__global__ void __launch_bounds__(kBlock) k_init(int32_t* __restrict__ label, int64_t n) {
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t done = 0;
  if (VEC) {
    // device-scope 16-byte stores through a resource based at the
    // workgroup's first group of each step (wavefront-uniform)
    const int64_t n4 = n >> 2;
    for (int64_t q0 = (int64_t)blockIdx.x * kBlock; q0 < n4; q0 += stride) {
      const int64_t q = q0 + threadIdx.x;
      const int32_t b = (int32_t)(q << 2);
      const __amdgpu_buffer_rsrc_t r = make_rsrc(label + 4 * q0, 16u * (uint32_t)min<int64_t>(kBlock, n4 - q0));
      st_dev4(r, 16u * threadIdx.x, make_int4(b, b + 1, b + 2, b + 3));
    }
    done = n4 << 2;
  }
  for (int64_t i = done + tid; i < n; i += stride) st_dev(label + i, (int32_t)i);
}

// Step (iii): roots of both ends of every occupied bond, then the atomicMin
// loop of Algorithm 1; unoccupied and same-root bonds issue nothing.  VEC:
// src/dst are 16-byte aligned and a lane takes four consecutive bonds with
// 16-byte loads (occ 4-byte aligned: one 4-byte load), then requests the first parent of
// all eight ends before chasing any of them.
// OCC: every bond occupied (0), read from the mask (1), or drawn as word b of
// the Philox stream for bond b (2; the mask ccl_bernoulli would write).
constexpr int kEdgeOccAll = 0, kEdgeOccMask = 1, kEdgeOccDraw = 2;

template <bool VEC, int OCC>
__global__ void __launch_bounds__(kBlock)
    k_merge_edges(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                  const uint8_t* __restrict__ occ, int64_t m, int32_t* label, PhiloxOcc rng) {
  constexpr bool HAS_OCC = OCC == kEdgeOccMask, DRAW = OCC == kEdgeOccDraw;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t done = 0;
  if (VEC) {
    const int64_t m4 = m >> 2;
    for (int64_t q = tid; q < m4; q += stride) {
      const int4 u4 = reinterpret_cast<const int4*>(src)[q];
      const int4 v4 = reinterpret_cast<const int4*>(dst)[q];
      uint32_t o4 = 0x01010101u;
      if (HAS_OCC) o4 = reinterpret_cast<const uint32_t*>(occ)[q];  // byte j = bond 4q + j
      if (DRAW) o4 = philox_occ4(rng, 4 * (uint64_t)q);            // one Philox block
      const int32_t u[4] = {u4.x, u4.y, u4.z, u4.w};
      const int32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
      int32_t pu[4], pv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool on = (o4 >> (8 * j)) & 0xFFu;
        pu[j] = on ? lab_ld(label + u[j]) : u[j];
        pv[j] = on ? lab_ld(label + v[j]) : v[j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (((o4 >> (8 * j)) & 0xFFu) == 0) continue;
        const int32_t r1 = find_root_halving_from(label, u[j], pu[j]);
        const int32_t r2 = find_root_halving_from(label, v[j], pv[j]);
        if (r1 != r2) join_roots(label, r1, r2);
      }
    }
    done = m4 << 2;
  }
  for (int64_t b = done + tid; b < m; b += stride) {
    if ((HAS_OCC && occ[b] == 0) || (DRAW && !philox_occupied(rng, (uint64_t)b))) continue;
    unite(label, src[b], dst[b]);
  }
}

// Step (iv): every site follows its label to the root and stores it, four
// sites per lane (16-byte loads and stores when aligned).  Workgroups own
// contiguous site ranges, renumbered so that each XCD's L2 holds one region
// of the array.  Every store in this step is a root: the owner of a site
// stores its root, and a chase that started at a site's parent p also stores
// the root into p, so the many sites sharing p find it in one step.  Both are
// final values (every writer of p stores the same root), whereas a shortcut
// to a non-root ancestor could land after the owner's final store and leave a
// non-root label behind -- so the chase itself stores nothing else.
template <bool VEC>
__global__ void __launch_bounds__(kBlock) k_flatten(int32_t* label, int64_t n) {
  constexpr int G = 4;  // 16-byte groups per lane per iteration
  const int64_t groups = (n + 3) >> 2;
  const int64_t per = (groups + gridDim.x - 1) / gridDim.x;
  const int64_t g0 = (int64_t)xcd_block_id() * per;
  const int64_t g1 = min(g0 + per, groups);
  const int64_t full = VEC ? (n >> 2) : 0;  // groups with all four sites in range
  // the workgroup's groups [g0, min(g1, full)) for its 16-byte stores (at most
  // 2^18 groups, so the byte offsets fit 32 bits)
  const __amdgpu_buffer_rsrc_t rl =
      make_rsrc(label + 4 * g0, 16u * (uint32_t)max<int64_t>(0, min(g1, full) - g0));
  for (int64_t gb = g0; gb < g1; gb += G * kBlock) {
    int4 v[G];
    int32_t q[G][4];
    // the lane's groups gb + j*kBlock + tid, then all sixteen parents' labels
#pragma unroll
    for (int j = 0; j < G; ++j) {
      // clamped index keeps the loads unconditional; groups outside the
      // vector range are replaced by the identity (nothing to do)
      const int64_t g = gb + j * kBlock + threadIdx.x;
      int4 ld = make_int4(0, 0, 0, 0);
      if (full > 0) ld = reinterpret_cast<const int4*>(label)[min(g, full - 1)];  // uniform branch
      const bool in = g < g1 && g < full;
      v[j] = in ? ld : make_int4((int32_t)(4 * g), (int32_t)(4 * g + 1), (int32_t)(4 * g + 2),
                                 (int32_t)(4 * g + 3));
    }
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int32_t* c = reinterpret_cast<const int32_t*>(&v[j]);
      const int64_t i0 = (gb + j * kBlock + threadIdx.x) << 2;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        // unconditional load (index 0 when nothing is needed) keeps the
        // sixteen loads free of branches, so they are all in flight at once
        const bool need = c[t] != (int32_t)(i0 + t);
        const int32_t got = lab_ld(label + (need ? c[t] : 0));
        q[j][t] = need ? got : c[t];
      }
    }
    // chases that remain (the parent is not a root) advance one link per
    // round, all sixteen at once, while any lane of the wavefront has one
    int32_t x[G][4], px[G][4];
    uint32_t open = 0;  // bit 4j+t: site t of group j is still chasing
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int64_t g = gb + j * kBlock + threadIdx.x;
      const int32_t* c = reinterpret_cast<const int32_t*>(&v[j]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool need = g < g1 && g < full && c[t] != (int32_t)((g << 2) + t) && q[j][t] != c[t];
        open |= (uint32_t)need << (4 * j + t);
        x[j][t] = q[j][t];
        px[j][t] = lab_ld(label + (need ? x[j][t] : 0));
      }
    }
    const uint32_t needed = open;
    for (;;) {
#pragma unroll
      for (int j = 0; j < G; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (px[j][t] == x[j][t]) open &= ~(1u << (4 * j + t));
      if (!__any(open != 0)) break;
#pragma unroll
      for (int j = 0; j < G; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          // unconditional load (index 0 when idle); an idle chase keeps its value
          const bool go = (open >> (4 * j + t)) & 1u;
          x[j][t] = go ? px[j][t] : x[j][t];
          const int32_t nx = lab_ld(label + (go ? x[j][t] : 0));
          px[j][t] = go ? nx : px[j][t];
        }
    }
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int64_t g = gb + j * kBlock + threadIdx.x;
      if (g >= g1) continue;
      const int64_t i0 = g << 2;
      if (g < full) {
        int32_t* c = reinterpret_cast<int32_t*>(&v[j]);
        if ((needed >> (4 * j)) & 0xFu) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (!((needed >> (4 * j + t)) & 1u)) continue;
            if (x[j][t] != q[j][t]) lab_st(label + c[t], x[j][t]);  // the parent's root
            c[t] = x[j][t];
          }
          st_dev4(rl, 16u * (uint32_t)(g - g0), v[j]);
        }
      } else {
        for (int64_t i = i0; i < min(i0 + 4, n); ++i) {
          const int32_t p = lab_ld(label + i);
          if (p == (int32_t)i) continue;
          const int32_t qq = lab_ld(label + p);
          if (qq == p) continue;
          const int32_t r = find_root(label, qq);
          if (r != qq) lab_st(label + p, r);
          lab_st(label + i, r);
        }
      }
    }
  }
}

ccl_status launch_init(int64_t n, int32_t* label, hipStream_t s, const DeviceInfo& d) {
  if (n == 0) return CCL_OK;
  const bool vec = (reinterpret_cast<uintptr_t>(label) & 15) == 0;
  const unsigned g = grid_for(vec ? (n + 3) / 4 : n, kBlock, 8, d);
  if (vec)
    CCL_LAUNCH("ccl_init", k_init<true>, g, kBlock, 0, s, label, n);
  else
    CCL_LAUNCH("ccl_init", k_init<false>, g, kBlock, 0, s, label, n);
  return CCL_OK;
}

ccl_status launch_flatten(int64_t n, int32_t* label, hipStream_t s, const DeviceInfo& d) {
  if (n == 0) return CCL_OK;
  const unsigned g = grid_for((n + 3) / 4, kBlock, 8, d);
  if ((reinterpret_cast<uintptr_t>(label) & 15) == 0)
    CCL_LAUNCH("ccl_flatten", k_flatten<true>, g, kBlock, 0, s, label, n);
  else
    CCL_LAUNCH("ccl_flatten", k_flatten<false>, g, kBlock, 0, s, label, n);
  return CCL_OK;
}

ccl_status launch_label_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              const uint8_t* occ, const PhiloxOcc* draw, int32_t* label,
                              hipStream_t s, const DeviceInfo& d) {
  ccl_status st = launch_init(n, label, s, d);
  if (st != CCL_OK) return st;
  if (m > 0) {
    // four bonds per lane only when that still fills the grid twice over: a
    // small graph needs every lane it can get to hide the chase latency
    const int64_t lanes = (int64_t)d.cu_count * 8 * kBlock;
    const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(occ) & 3) == 0 && m >= 8 * lanes;
    const unsigned g = grid_for(vec ? (m + 3) / 4 : m, kBlock, 8, d);
    const PhiloxOcc rng = draw != nullptr ? *draw : PhiloxOcc{0, 0, 0};
    if (vec && occ)
      CCL_LAUNCH("ccl_merge_edges", (k_merge_edges<true, kEdgeOccMask>), g, kBlock, 0, s, src, dst, occ,
                 m, label, rng);
    else if (vec && draw)
      CCL_LAUNCH("ccl_merge_edges", (k_merge_edges<true, kEdgeOccDraw>), g, kBlock, 0, s, src, dst, occ,
                 m, label, rng);
    else if (vec)
      CCL_LAUNCH("ccl_merge_edges", (k_merge_edges<true, kEdgeOccAll>), g, kBlock, 0, s, src, dst, occ,
                 m, label, rng);
    else if (occ)
      CCL_LAUNCH("ccl_merge_edges", (k_merge_edges<false, kEdgeOccMask>), g, kBlock, 0, s, src, dst, occ,
                 m, label, rng);
    else if (draw)
      CCL_LAUNCH("ccl_merge_edges", (k_merge_edges<false, kEdgeOccDraw>), g, kBlock, 0, s, src, dst, occ,
                 m, label, rng);
    else
      CCL_LAUNCH("ccl_merge_edges", (k_merge_edges<false, kEdgeOccAll>), g, kBlock, 0, s, src, dst, occ,
                 m, label, rng);
  }
  return launch_flatten(n, label, s, d);
}

// ---------------------------------------------------------------- checks

__global__ void __launch_bounds__(kBlock)
    k_validate_edges(int64_t n, int64_t m, const int32_t* __restrict__ src,
                     const int32_t* __restrict__ dst, unsigned long long* count) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  unsigned long long bad = 0;
  for (int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x; b < m; b += stride) {
    const int64_t u = src[b], v = dst[b];
    bad += (u < 0 || u >= n || v < 0 || v >= n) ? 1ull : 0ull;
  }
  if (bad) atomicAdd(count, bad);
}

ccl_status launch_validate_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                 unsigned long long* d_count, hipStream_t s, const DeviceInfo& d) {
  if (m == 0) return CCL_OK;
  CCL_LAUNCH("ccl_validate_edges", k_validate_edges, grid_for(m, kBlock, 8, d), kBlock, 0, s, n,
             m, src, dst, d_count);
  return CCL_OK;
}

// ---------------------------------------------------------------- probe

// Streaming copy: four 16-byte loads per lane in flight before the four
// stores, workgroups on contiguous XCD-local ranges; the tail byte by byte.
__global__ void __launch_bounds__(kBlock)
    k_probe_copy(const int4* __restrict__ in, int4* __restrict__ out, int64_t n16,
                 const uint8_t* __restrict__ in_b, uint8_t* __restrict__ out_b, int64_t tail) {
  constexpr int U = 4;
  const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)xcd_block_id() * per, hi = min(lo + per, n16);
  int64_t i = lo + threadIdx.x;
  for (; i + (U - 1) * kBlock < hi; i += U * kBlock) {
    int4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = in[i + u * kBlock];
#pragma unroll
    for (int u = 0; u < U; ++u) out[i + u * kBlock] = v[u];
  }
  for (; i < hi; i += kBlock) out[i] = in[i];
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (tid < tail) out_b[tid] = in_b[tid];
}

ccl_status launch_probe_copy(const void* in, void* out, size_t bytes, hipStream_t s,
                             const DeviceInfo& d) {
  if (bytes == 0) return CCL_OK;
  const int64_t n16 = (int64_t)(bytes / 16), tail = (int64_t)(bytes % 16);
  const uint8_t* ib = static_cast<const uint8_t*>(in) + n16 * 16;
  uint8_t* ob = static_cast<uint8_t*>(out) + n16 * 16;
  CCL_LAUNCH("ccl_probe_copy", k_probe_copy, grid_for(n16 > 0 ? n16 : 1, kBlock, 8, d), kBlock, 0,
             s, static_cast<const int4*>(in), static_cast<int4*>(out), n16, ib, ob, tail);
  return CCL_OK;
}

}  // namespace ccl
