// CSR labeling with tile-local joins in LDS.
//
// Sites are cut into tiles of kCsrTile (65536) consecutive ids; a tile owns its sites
// and the bonds stored in its rows.  Three kernels:
//   1. tile kernel, one workgroup per tile: step (i) for the tile in LDS
//      (par[t] = t, 16-bit tile-relative entries: 128 KB), step (iii) --
//      Algorithm 1 on LDS, its atomicMin a 32-bit compare-and-swap -- for every
//      occupied bond whose two ends lie in the tile, a root chase in LDS, and
//      one coalesced store of the tile's labels (each site's tile-local root,
//      the tile's minimum member of its local cluster; the grid tiles store
//      a near ancestor for the rare site deeper than their lockstep chase
//      reaches).  Occupied bonds that
//      leave the tile are appended, as (site, neighbour) pairs, to the tile's
//      own segment of the workspace (the segment has room for every bond of
//      the tile, so no global counter is needed);
//   2. cross kernel: step (iii) in global memory (Algorithm 1 with
//      device-scope atomicMin) over those pairs;
//   3. flatten: step (iv).
// Every value the tile kernel stores is a member of the site's cluster no
// larger than the site, so kernels 2-3 see a valid forest and finish the job
// exactly as the single-pass method would.
#include "common.hpp"
#include "mem.hpp"
#include "philox.hpp"
#include "tile.hpp"
#include "uf.hpp"

namespace ccl {

constexpr int kTileShift = 16;
constexpr int kRowsPerThread = 4;  // rows per thread per iteration (row path)
constexpr int kDegFast = 4;        // bonds per row kept in registers (row path)
constexpr int kChunkRows = kTileBlock * kRowsPerThread;
constexpr int kGroupsPerIter = 2;  // groups of four bonds per lane per step (affine path; 1, 3, 4 measured slower)
constexpr int kLeaveBits = 5;  // a lane leaves at most 16 bonds per step: 5-bit counts
static_assert(4 * kGroupsPerIter < (1 << kLeaveBits) && kRowsPerThread * kDegFast < (1 << kLeaveBits),
              "a lane's leaving bonds per step must fit a count of kLeaveBits bits");
static_assert((1 << kTileShift) == kCsrTile, "tile size");

// Tile-relative row of tile-relative bond e in an affine tile of degree d,
// as e * ceil(2^20 / d) >> 20 (exact for d <= 4 and e < 2^18, which a tile of
// 65536 rows of at most 4 bonds satisfies); `magic` is ceil(2^20 / d).
__device__ __forceinline__ int32_t affine_row(int32_t e, uint32_t magic) {
  return (int32_t)(((uint64_t)(uint32_t)e * magic) >> 20);
}

// Site column of bond e of a tile row of degree d <= 4, as e * ceil(2^16 / d)
// >> 16 with one 24-bit multiply: exact for e < 2^14 (a grid tile row of at
// most 4096 sites has at most 16384 bonds); `magic16` is ceil(2^16 / d).
__device__ __forceinline__ int32_t row_bond_site(int32_t e, uint32_t magic16) {
  return (int32_t)(__umul24((uint32_t)e, magic16) >> 16);
}

// Join bond (t, v) of the tile (t tile-relative, v global) in LDS, or, when v
// lies outside the tile, count it and return true (the caller records it).
__device__ __forceinline__ bool tile_bond(uint16_t* par, int32_t t, int32_t v, int64_t lo,
                                          int32_t cnt) {
  const int64_t vl = (int64_t)v - lo;
  if (vl >= 0 && vl < cnt) {
    lds16_unite(par, t, (int32_t)vl);
    return false;
  }
  return true;
}

// One workgroup per tile.  A tile whose bond count is d*cnt (1 <= d <= 4) is
// read as affine (row_ptr[lo + t] = e_begin + d*t): its bonds stream in
// groups of four, lane tid taking groups (G*k+u)*kTileBlock + tid (u < G =
// kGroupsPerIter) at step k with one 16-byte col load and one 4-byte occ load
// per group, both fully coalesced, and requesting step k+1's groups before
// joining step k's, so no barrier or wait on another wavefront is ever on
// the way.  The affine form is verified during the same stream (16 bytes of
// row_ptr per lane and step) and voted on at the end; a tile that fails
// starts over on the row path, as do all other CSR graphs: kRowsPerThread
// rows per lane, the first
//    kDegFast bonds of each row in one batch of buffer loads (longer rows in a
//    loop), the next rows' row_ptr requested ahead.
// Buffer resources are based at the tile's first row and first bond, so
// offsets stay small whatever the graph size; a tile with 2^30 or more bonds
// uses plain loads.
// Occupancy of the bonds: all occupied, read from a mask aligned with col, or
// drawn from the Philox stream on the fly (bond e is word e of the stream;
// the same draw ccl_bernoulli writes into a mask).
constexpr int kOccAll = 0, kOccMask = 1, kOccDraw = 2;

template <int OCC>
__global__ void __launch_bounds__(kTileBlock)
    k_csr_tile(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
               const uint8_t* __restrict__ occ, int32_t* __restrict__ label,
               int2* __restrict__ pairs, int2* __restrict__ seg, PhiloxOcc rng) {
  constexpr bool HAS_OCC = OCC == kOccMask, DRAW = OCC == kOccDraw;
  __shared__ uint16_t par[kCsrTile];  // tile-relative parents, 16 bits each
  __shared__ uint32_t stage[kTileBlock / 64][kStageCap];  // per-wavefront join staging
  __shared__ uint32_t n_out;
  const int wave = threadIdx.x >> 6;
  const int64_t lo = (int64_t)blockIdx.x << kTileShift;
  const int32_t cnt = (int32_t)min((int64_t)kCsrTile, n - lo);
  const int tid = threadIdx.x;
  const int32_t e0 = row_ptr[0];
  const int32_t e_begin = row_ptr[lo];
  const int32_t e_count = row_ptr[lo + cnt] - e_begin;
  const bool fast = e_count >= 0 && e_count < (1 << 30);
  // the tile's segment of the pair list: one slot per bond of the tile
  int2* my_pairs = pairs != nullptr ? pairs + (e_begin - e0) : nullptr;
  const int32_t deg = (fast && cnt > 0 && e_count % cnt == 0) ? e_count / cnt : 0;
  const bool affine_try =
      deg >= 1 && deg <= 4 &&
      (!HAS_OCC || ((reinterpret_cast<uintptr_t>(occ + e_begin) & 3) == 0));
  const uint32_t magic = deg > 0 ? ((1u << 20) + (uint32_t)deg - 1u) / (uint32_t)deg : 0u;
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(row_ptr + lo, (uint32_t)(cnt + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(col + e_begin, fast ? (uint32_t)e_count * 4u : 0u);
  const __amdgpu_buffer_rsrc_t ro =
      make_rsrc(HAS_OCC ? occ + e_begin : nullptr, fast && HAS_OCC ? (uint32_t)e_count : 0u);

  // the affine stream's first bond loads go out before the LDS is set up
  const int32_t nb = deg * cnt;
  const int32_t full = nb >> 2;  // groups of four bonds entirely inside the tile
  constexpr int G = kGroupsPerIter;
  const int32_t iters = (((nb + 3) >> 2) + G * kTileBlock - 1) / (G * kTileBlock);
  int4 c[G], cn[G];
  uint32_t o[G], on[G];
  auto load = [&](int32_t k, int u, int4& cv, uint32_t& ov) {
    const int32_t q = (G * k + u) * kTileBlock + tid;
    const uint32_t off = q < full ? 4u * (uint32_t)q : kOffNone;
    cv = buf_i32x4(rc, off * 4u);
    ov = HAS_OCC ? buf_u32(ro, off)
                 : (off == kOffNone ? 0u : (DRAW ? philox_occ4(rng, (uint64_t)e_begin + off) : 0x01010101u));
  };
  if (affine_try) {
#pragma unroll
    for (int u = 0; u < G; ++u) load(0, u, c[u], o[u]);
  }

  auto init_par = [&]() {
    for (int w = tid; w < kCsrTile / 8; w += kTileBlock) {  // par[t] = t, 16 bytes at a time
      const uint32_t t = 8u * (uint32_t)w;
      reinterpret_cast<uint4*>(par)[w] =
          make_uint4(t | ((t + 1) << 16), (t + 2) | ((t + 3) << 16), (t + 4) | ((t + 5) << 16),
                     (t + 6) | ((t + 7) << 16));
    }
    if (tid == 0) n_out = 0;
  };
  init_par();
  __syncthreads();

  // ---- B, affine, speculatively: bond groups of four, read as if row_ptr
  // were e_begin + deg*r.  The rows are checked against that on the way (16
  // bytes of row_ptr per lane and step, in flight with the bond loads); a
  // tile that fails the check starts again on the row path, which rewrites
  // the tile's leaving pairs from the start of its segment.  Every index the
  // affine reading forms stays inside the tile and its resources either way.
  bool affine = false;
  if (affine_try) {
    const int32_t g4 = cnt >> 2;  // groups of four rows
    auto rp_load = [&](int32_t g) { return buf_i32x4(rp, g < g4 ? 16u * (uint32_t)g : kOffNone * 4u); };
    auto rp_ok = [&](int32_t g, const int4& v) {
      const int32_t r0 = e_begin + deg * 4 * g;
      return g >= g4 || (v.x == r0 && v.y == r0 + deg && v.z == r0 + 2 * deg && v.w == r0 + 3 * deg);
    };
    bool ok = true;
    int4 rv = rp_load(tid), rvn;
    uint32_t staged = 0;  // entries on this wavefront's staging stack
    for (int32_t k = 0; k < iters; ++k) {
#pragma unroll
      for (int u = 0; u < G; ++u) load(k + 1, u, cn[u], on[u]);
      rvn = rp_load((k + 1) * kTileBlock + tid);
      ok = rp_ok(k * kTileBlock + tid, rv) && ok;
      uint32_t leave = 0;  // bit 4u+j: bond j of group u leaves the tile
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int32_t e = 4 * ((G * k + u) * kTileBlock + tid);
        const int32_t c4[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
        uint32_t act = 0;  // bit j: bond j of the group is occupied and inside the tile
        uint32_t packed[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool on = ((o[u] >> (8 * j)) & 0xFFu) != 0;
          const uint32_t vl = (uint32_t)c4[j] - (uint32_t)lo;  // lo + cnt <= 2^31
          const bool inside = vl < (uint32_t)cnt;
          if (on && !inside) leave |= 1u << (4 * u + j);
          act |= (uint32_t)(on && inside) << j;
          packed[j] = ((uint32_t)affine_row(e + j, magic) << 16) | (vl & 0xFFFFu);
        }
        tile_join_compact(par, stage[wave], staged, act, packed);
      }
      uint32_t slot = reserve_slots<kLeaveBits>(__popc(leave), &n_out);
      if (leave) {  // static indices only: the register arrays must not spill
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int32_t e = 4 * ((G * k + u) * kTileBlock + tid);
          const int32_t c4[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if ((leave >> (4 * u + j)) & 1u)
              st_dev2(my_pairs + slot++, make_int2((int32_t)(lo + affine_row(e + j, magic)), c4[j]));
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        c[u] = cn[u];
        o[u] = on[u];
      }
      rv = rvn;
    }
    // row groups past the loop's steps, then the last cnt mod 4 rows (the
    // entry at lo+cnt is e_begin + deg*cnt by the choice of deg)
    for (int32_t g = iters * kTileBlock + tid; g < g4; g += kTileBlock) ok = rp_ok(g, rp_load(g)) && ok;
    for (int32_t t = 4 * g4 + tid; t < cnt; t += kTileBlock)
      ok = buf_i32(rp, 4u * (uint32_t)t) == e_begin + deg * t && ok;
    drain_joins(par, stage[wave], staged);  // what is left on the stack
    affine = __syncthreads_and(ok) != 0;
    if (!affine) {
      init_par();
      __syncthreads();
    }
  }
  if (affine) {
    // the last group, when it straddles the end of the tile
    if (tid == 0 && full * 4 < nb) {
      for (int32_t x = 4 * full; x < nb; ++x) {
        const int64_t ge = (int64_t)e_begin + x;
        if ((HAS_OCC && occ[ge] == 0) || (DRAW && !philox_occupied(rng, (uint64_t)ge))) continue;
        const int32_t v = col[ge];
        if (tile_bond(par, affine_row(x, magic), v, lo, cnt)) {
          const uint32_t sl =
              __hip_atomic_fetch_add(&n_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          st_dev2(my_pairs + sl, make_int2((int32_t)(lo + affine_row(x, magic)), v));
        }
      }
    }
  } else {
    // ---- B, rows
    int32_t ra[kRowsPerThread], rb[kRowsPerThread];
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const uint32_t t = (uint32_t)(k * kTileBlock + tid);
      ra[k] = buf_i32(rp, 4u * t) - e_begin;
      rb[k] = buf_i32(rp, 4u * (t + 1)) - e_begin;
    }
    for (int base = 0; base < cnt; base += kChunkRows) {
      int32_t cv[kRowsPerThread][kDegFast];
      uint32_t ov[kRowsPerThread][kDegFast];
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k)
#pragma unroll
        for (int j = 0; j < kDegFast; ++j) {
          const int32_t e = ra[k] + j;
          const uint32_t off =
              (fast && e < rb[k] && base + k * kTileBlock + tid < cnt) ? (uint32_t)e : kOffNone;
          cv[k][j] = buf_i32(rc, off * 4u);
          ov[k][j] = HAS_OCC ? buf_u8(ro, off)
                             : (off == kOffNone ? 0u
                                                : (DRAW ? (philox_occupied(rng, (uint64_t)e_begin + off) ? 1u : 0u)
                                                        : 1u));
        }
      int32_t na[kRowsPerThread], nb[kRowsPerThread];
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
        const uint32_t t = (uint32_t)(base + kChunkRows + k * kTileBlock + tid);
        na[k] = buf_i32(rp, 4u * t) - e_begin;
        nb[k] = buf_i32(rp, 4u * (t + 1)) - e_begin;
      }
      uint32_t leave = 0;  // bit kDegFast*k+j: register bond (k, j) leaves the tile
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {  // one row's bonds per lockstep join
        int32_t ja[kDegFast], jb[kDegFast];
        const int t = base + k * kTileBlock + tid;
#pragma unroll
        for (int j = 0; j < kDegFast; ++j) {
          const bool on = t < cnt && ov[k][j] != 0;
          const uint32_t vl = (uint32_t)cv[k][j] - (uint32_t)lo;  // lo + cnt <= 2^31
          const bool inside = vl < (uint32_t)cnt;
          if (on && !inside) leave |= 1u << (kDegFast * k + j);
          ja[j] = on && inside ? t : 0;
          jb[j] = on && inside ? (int32_t)vl : 0;
        }
        lds16_unite_lockstep<kDegFast, kLdsRounds>(par, ja, jb);
      }
      uint32_t slot = reserve_slots<kLeaveBits>(__popc(leave), &n_out);
      if (leave) {  // static indices only: the register arrays must not spill
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k)
#pragma unroll
          for (int j = 0; j < kDegFast; ++j)
            if ((leave >> (kDegFast * k + j)) & 1u)
              st_dev2(my_pairs + slot++, make_int2((int32_t)(lo + base + k * kTileBlock + tid), cv[k][j]));
      }
      // rows longer than kDegFast: the rest of their bonds one by one
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
        const int t = base + k * kTileBlock + tid;
        if (t >= cnt) continue;
        for (int32_t e = ra[k] + (fast ? kDegFast : 0); e < rb[k]; ++e) {
          const int64_t ge = (int64_t)e_begin + e;
          if ((HAS_OCC && occ[ge] == 0) || (DRAW && !philox_occupied(rng, (uint64_t)ge))) continue;
          const int32_t v = col[ge];
          if (tile_bond(par, t, v, lo, cnt)) {
            const uint32_t sl =
                __hip_atomic_fetch_add(&n_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            st_dev2(my_pairs + sl, make_int2((int32_t)(lo + t), v));
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
        ra[k] = na[k];
        rb[k] = nb[k];
      }
    }
  }
  __syncthreads();
  // the tile's labels: each site's tile-local root (its cluster's minimum in
  // the tile), eight sites per lane resolved together and stored 16 bytes at
  // a time when the label array allows it
  const int32_t n4 = ((reinterpret_cast<uintptr_t>(label + lo) & 15) == 0) ? (cnt >> 2) : 0;
  const __amdgpu_buffer_rsrc_t rl = make_rsrc(label + lo, 16u * (uint32_t)n4);
  for (int32_t q0 = 0; q0 < n4; q0 += 2 * kTileBlock) {
    int32_t x[8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t q = q0 + h * kTileBlock + tid;
      const uint2 w = reinterpret_cast<const uint2*>(par)[q < n4 ? q : 0];  // parents of 4q..4q+3
      x[4 * h + 0] = (int32_t)(w.x & 0xFFFFu);
      x[4 * h + 1] = (int32_t)(w.x >> 16);
      x[4 * h + 2] = (int32_t)(w.y & 0xFFFFu);
      x[4 * h + 3] = (int32_t)(w.y >> 16);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = lds16_ld(par + x[k]);  // a root reads itself
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int32_t p = lds16_ld(par + x[k]);
      if (p != x[k]) x[k] = lds16_find(par, x[k]);  // the rare longer chain
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t q = q0 + h * kTileBlock + tid;
      const int32_t b = (int32_t)lo;
      if (q < n4)
        st_dev4(rl, 16u * (uint32_t)q,
                make_int4(b + x[4 * h], b + x[4 * h + 1], b + x[4 * h + 2], b + x[4 * h + 3]));
    }
  }
  for (int t = 4 * n4 + tid; t < cnt; t += kTileBlock) st_dev(label + lo + t, (int32_t)(lo + lds16_find(par, t)));
  if (tid == 0 && seg != nullptr) st_dev2(seg + blockIdx.x, make_int2(e_begin - e0, (int32_t)n_out));
}

// ---------------------------------------------------------------- 2-D tiles
//
// Grid tiles.  When the site ids number a grid row by row (site y*W + x,
// e.g. a lattice of row length W), a tile of 65536 consecutive ids is a slab
// of 65536/W rows whose two long edges cross up to 2W bonds each way: on the
// 8192-wide triangular lattice a quarter of the sites sit on a slab edge and
// the cross kernel gets 5.8 M leaving bonds at p_c.  A grid tile is instead
// kGridTh rows of kGridTw columns (32 x 2048): a quarter of the edge per
// site, so a quarter of the leaving bonds.  Taller tiles hold larger
// clusters, whose LDS joins cost more; on MI355X the 32 x 2048 tile was the
// fastest whole path (tile kernel 0.518 ms, cross 0.082, flatten 0.173 on
// the 8192^2 triangular lattice at p_c, against 0.469 / 0.145 / 0.187 for
// 16 x 4096 and 0.560 / 0.056 / 0.162 for 64 x 1024).  Any CSR graph is
// labelled correctly with any W; W only changes which bonds stay inside a
// tile.  Tile (ty, tx) holds rows [32 ty, 32 ty + 32) and columns
// [2048 tx, 2048 tx + cw); tile-relative slot t = (row << 11) | column, so
// slot order is id order and the LDS roots are still the tile minima.
// Tile-row ty's bonds form one contiguous range of the CSR, and tile tx of
// that row takes the slots [start + bonds of columns < 2048 tx in each of its
// rows, + its own bonds) of the pair list: the tiles' regions are disjoint
// and exactly as large as their bond counts, for any CSR.
constexpr int kGridTwShift = 11;
constexpr int kGridTw = 1 << kGridTwShift;
constexpr int kGridTh = kCsrTile / kGridTw;
static_assert(kGridTh <= 64, "one lane per tile row in the header loads");
static_assert(kGridTw >= kTileBlock && (4 * kTileBlock) % kGridTw == 0, "the epilogue's runs cover whole rows");
constexpr int kEpiRuns = 2;    // runs of 4 kTileBlock slots per epilogue pass
constexpr int kEpiRounds = 3;  // lockstep LDS rounds of the epilogue's chases

struct GridGeo {
  int64_t n;        // sites
  int64_t w;        // row length of the id grid
  int64_t h;        // rows, ceil(n / w)
  int32_t tiles_x;  // tiles per tile-row, ceil(w / kGridTw)
  float inv_w;      // 1 / w
  int32_t w_shift;  // log2(w) when w is a power of two
};

// Sum over the 64 lanes of a wavefront.
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <int OCC, bool POW2>
__global__ void __launch_bounds__(kTileBlock)
    k_csr_tile_grid(GridGeo geo, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                    const uint8_t* __restrict__ occ, int32_t* __restrict__ label,
                    int2* __restrict__ pairs, int2* __restrict__ seg, PhiloxOcc rng) {
  constexpr bool HAS_OCC = OCC == kOccMask, DRAW = OCC == kOccDraw;
  __shared__ uint16_t par[kCsrTile];  // tile-relative parents, 16 bits each
  __shared__ uint32_t stage[kTileBlock / 64][kStageCap];  // per-wavefront join staging
  __shared__ uint32_t n_out;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  // Workgroup-uniform values are kept in scalar registers (readfirstlane):
  // a buffer resource or loop bound the compiler took for divergent would
  // cost a waterfall loop around every load and vector registers the stream
  // needs.
  auto uni = [](int32_t v) { return __builtin_amdgcn_readfirstlane(v); };
  auto uni64 = [&](int64_t v) {
    return (int64_t)(((uint64_t)(uint32_t)uni((int32_t)(v >> 32)) << 32) | (uint32_t)uni((int32_t)v));
  };
  const int32_t ty = (int32_t)blockIdx.x / geo.tiles_x;
  const int32_t tx = (int32_t)blockIdx.x - ty * geo.tiles_x;
  const int64_t y0 = (int64_t)ty * kGridTh;
  const int64_t x0 = (int64_t)tx << kGridTwShift;
  const int32_t cw = (int32_t)min((int64_t)kGridTw, geo.w - x0);
  const int64_t u0 = y0 * geo.w + x0;
  // sites of tile row s: [u0 + s w, + len(s)); the last grid row may be partial
  auto seg_len = [&](int32_t s) -> int32_t {
    const int64_t r = geo.n - (u0 + (int64_t)s * geo.w);
    return r <= 0 ? 0 : (int32_t)min((int64_t)cw, r);
  };
  // rows of the tile-row, and those holding at least one site of this tile
  // (only the last grid row can be short)
  const int32_t rows_all = uni((int32_t)min((int64_t)kGridTh, geo.h - y0));
  const int32_t rows = uni(rows_all > 0 && seg_len(rows_all - 1) == 0 ? rows_all - 1 : rows_all);
  if (rows == 0) {  // no site of the partial last grid row falls in this tile
    if (threadIdx.x == 0) st_dev2(seg + blockIdx.x, make_int2(0, 0));
    return;
  }
  // header, computed by every wavefront on its own (lane s < rows: tile row s):
  // the first bond of the tile-row, of the row and of the tile's segment of
  // it, and the end of that segment
  int32_t ra = 0, rb = 0, rc_end = 0, len_l = 0;
  if (lane < rows_all) {
    const int64_t row0 = min((y0 + lane) * geo.w, geo.n);
    const int64_t us = min(row0 + x0, geo.n);
    len_l = seg_len(lane);
    ra = row_ptr[row0];
    rb = row_ptr[us];
    rc_end = row_ptr[us + len_l];
  }
  const int32_t e0 = row_ptr[0];
  const int32_t tile_row_start = uni(__shfl(ra, 0, 64));
  const int32_t e_first = uni(__shfl(rb, 0, 64));           // first bond of the tile
  const int32_t e_last = uni(__shfl(rc_end, rows - 1, 64));  // one past its last bond
  const int64_t before = uni64(wave_sum64(lane < rows_all ? (int64_t)(rb - ra) : 0));
  const int64_t mine = uni64(wave_sum64(lane < rows_all ? (int64_t)(rc_end - rb) : 0));  // the tile's bonds
  const int64_t tile_sites = uni64(wave_sum64((int64_t)len_l));
  const int64_t region = (int64_t)(tile_row_start - e0) + before;  // the tile's pair-list slots
  int2* my_pairs = pairs + region;
  const int32_t len0 = uni(seg_len(0));
  const int32_t len_last = uni(seg_len(rows - 1));  // every other tile row has cw sites
  auto row_len = [&](int32_t s) { return s == rows - 1 ? len_last : (s < rows ? cw : 0); };
  const int64_t span_sites = uni64((int64_t)(rows - 1) * geo.w + len_last);  // u0 .. last site + 1
  const int32_t span_bonds = e_last - e_first;
  const bool fast = uni(span_bonds >= 0 && span_bonds < (1 << 30) && span_sites < (1 << 29)) != 0;
  // affine: row_ptr[u] = e_first + deg (u - u0) on every site of the tile.
  // Tried when the first row, the whole span and the tile's own bonds all
  // fit that degree (so the speculative pass never records more leaving
  // bonds than the tile's region holds), then verified entry by entry.
  const int32_t seg0_bonds = uni(__shfl(rc_end, 0, 64)) - e_first;
  const int32_t deg = uni((fast && len0 > 0 && seg0_bonds % len0 == 0) ? seg0_bonds / len0 : 0);
  const bool affine_try =
      deg >= 1 && deg <= 4 && (int64_t)span_bonds == (int64_t)deg * span_sites &&
      mine == (int64_t)deg * tile_sites &&
      ((int64_t)deg * geo.w) % 4 == 0 &&
      (!HAS_OCC || ((reinterpret_cast<uintptr_t>(occ + e_first) & 3) == 0));
  const uint32_t magic16 = deg > 0 ? ((1u << 16) + (uint32_t)deg - 1u) / (uint32_t)deg : 0u;
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(row_ptr + u0, fast ? (uint32_t)(span_sites + 1) * 4u : 0u);
  const __amdgpu_buffer_rsrc_t rcol = make_rsrc(col + e_first, fast ? (uint32_t)span_bonds * 4u : 0u);
  const __amdgpu_buffer_rsrc_t ro =
      make_rsrc(HAS_OCC ? occ + e_first : nullptr, fast && HAS_OCC ? (uint32_t)span_bonds : 0u);
  const int32_t w32 = (int32_t)min(geo.w, (int64_t)INT32_MAX);
  const int32_t row_base = (int32_t)(y0 * geo.w);  // < n <= 2^31 - 1
  const uint32_t lim = (uint32_t)min((int64_t)rows * geo.w, (int64_t)UINT32_MAX);

  // Tile slot of site v, or -1 when v lies outside the tile.  POW2: bit
  // fields (below); otherwise a float quotient corrected by one step (exact:
  // the row index within reach is below kGridTh).
  // With w = 2^w_shift (>= 2 kGridTw), an id is (row, column) in bit fields,
  // the tile is the ids whose bits above the low 11 of the column and above
  // the low 5 of the row equal the tile's (mask pow2_m, pattern pow2_b), and
  // the slot is those low bits side by side.
  const uint32_t pow2_m = POW2 ? ~((uint32_t)(kGridTw - 1) | ((uint32_t)(kGridTh - 1) << geo.w_shift)) : 0u;
  const uint32_t pow2_b = POW2 ? ((uint32_t)x0 | (uint32_t)(y0 << geo.w_shift)) : 0u;
  auto slot_of = [&](int32_t v) -> int32_t {
    if (POW2) {
      const uint32_t uv = (uint32_t)v;
      const uint32_t t = (((uv >> geo.w_shift) & (uint32_t)(kGridTh - 1)) << kGridTwShift) |
                         (uv & (uint32_t)(kGridTw - 1));
      return (uv & pow2_m) == pow2_b ? (int32_t)t : -1;
    }
    const uint32_t vr = (uint32_t)(v - row_base);
    if (vr >= lim) return -1;
    int32_t vs = (int32_t)((float)vr * geo.inv_w);
    int32_t r = (int32_t)vr - vs * w32;
    if (r < 0) {
      --vs;
      r += w32;
    } else if (r >= w32) {
      ++vs;
      r -= w32;
    }
    const uint32_t vc = (uint32_t)(r - (int32_t)x0);
    return vc < (uint32_t)cw ? (vs << kGridTwShift) | (int32_t)vc : -1;
  };

  // ---- the affine stream.  A tile row's bonds are [e_first + deg s w,
  // + deg len(s)), read relative to the tile's first bond in groups of four;
  // each row is padded to whole slots of kTileBlock groups (spr slots per
  // row), so a slot -- one group per lane -- lies in a single row and its
  // row index is a scalar.  Slot (k, u) of step k is G k + u.
  const int32_t gps = (deg * cw + 3) >> 2;                        // groups per row
  const int32_t spr = max(1, (gps + kTileBlock - 1) / kTileBlock);  // slots per row
  const int32_t n_slots = rows * spr;
  constexpr int G = kGroupsPerIter;
  const int32_t iters = (n_slots + G - 1) / G;
  int4 c[G], cn[G];
  uint32_t o[G], on[G];
  // a slot position (row s, slot r of the row), advanced without division
  struct SlotPos {
    int32_t s, r;
  };
  auto advance = [&](SlotPos p, int32_t by) {  // by <= G
#pragma unroll
    for (int i = 0; i < G; ++i)
      if (i < by && ++p.r == spr) {
        p.r = 0;
        ++p.s;
      }
    return p;
  };
  auto group = [&](SlotPos p) { return p.r * kTileBlock + tid; };
  auto load = [&](SlotPos p, int4& cv, uint32_t& ov) {
    const int32_t g = group(p);
    const bool in = p.s < rows && 4 * g < deg * row_len(p.s);
    const uint32_t off = in ? (uint32_t)(deg * p.s * w32 + 4 * g) : kOffNone;
    cv = buf_i32x4(rcol, off * 4u);
    ov = HAS_OCC ? buf_u32(ro, off)
                 : (!in ? 0u : (DRAW ? philox_occ4(rng, (uint64_t)e_first + off) : 0x01010101u));
  };
  SlotPos next{0, 0};  // the slot of the next load
  if (affine_try) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      load(next, c[u], o[u]);
      next = advance(next, 1);
    }
  }

  auto init_par = [&]() {
    for (int w = tid; w < kCsrTile / 8; w += kTileBlock) {  // par[t] = t, 16 bytes at a time
      const uint32_t t = 8u * (uint32_t)w;
      reinterpret_cast<uint4*>(par)[w] =
          make_uint4(t | ((t + 1) << 16), (t + 2) | ((t + 3) << 16), (t + 4) | ((t + 5) << 16),
                     (t + 6) | ((t + 7) << 16));
    }
    if (tid == 0) n_out = 0;
  };
  init_par();
  __syncthreads();

  bool affine = false;
  if (affine_try) {
    // verification: every row_ptr entry of every tile row equals e_first +
    // deg (u - u0): entries [0, len(s)) of row s in groups of four, one group
    // per lane, vslots per row, one vslot per step (requested a step ahead,
    // like the bonds, so no wait for it stands between a step's loads and its
    // joins), the rest after the loop; then the end entry of each row
    const int32_t rgps = (cw + 3) >> 2;
    const int32_t vspr = max(1, (rgps + kTileBlock - 1) / kTileBlock);
    const int32_t n_vslots = rows * vspr;
    auto rp_at = [&](int32_t vslot, int32_t& rel, int32_t& n_ok) {
      const int32_t s = vslot / vspr;  // scalar
      const int32_t i = 4 * ((vslot - s * vspr) * kTileBlock + tid);
      n_ok = vslot < n_vslots ? row_len(s) - i : 0;
      rel = s * w32 + i;  // site offset from u0
    };
    auto rp_load = [&](int32_t vslot) {
      int32_t rel, n_ok;
      rp_at(vslot, rel, n_ok);
      return buf_i32x4(rp, n_ok > 0 ? 4u * (uint32_t)rel : kOffNone * 4u);
    };
    auto rp_ok = [&](int32_t vslot, const int4& v) {
      int32_t rel, n_ok;
      rp_at(vslot, rel, n_ok);
      const int32_t want = (int32_t)((uint32_t)e_first + (uint32_t)deg * (uint32_t)rel);
      return n_ok <= 0 ||
             ((v.x == want) && (n_ok < 2 || v.y == want + deg) && (n_ok < 3 || v.z == want + 2 * deg) &&
              (n_ok < 4 || v.w == want + 3 * deg));
    };
    bool ok = true;
    uint32_t staged = 0;  // entries on this wavefront's staging stack
    int4 rv = rp_load(0), rvn;
    SlotPos cur{0, 0};  // the slot of this step's first group
    for (int32_t k = 0; k < iters; ++k) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        load(next, cn[u], on[u]);
        next = advance(next, 1);
      }
      rvn = rp_load(k + 1);
      ok = rp_ok(k, rv) && ok;
      uint32_t leave = 0;  // bit 4u+j: bond j of group u leaves the tile
      SlotPos at = cur;
#pragma unroll
      for (int u = 0; u < G; ++u, at = advance(at, 1)) {
        const int32_t s = at.s;
        const int32_t g = group(at);
        const int32_t c4[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
        uint32_t act = 0;  // bit j: bond j of the group is occupied and inside the tile
        uint32_t packed[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool on = ((o[u] >> (8 * j)) & 0xFFu) != 0;
          const int32_t vt = slot_of(c4[j]);
          if (on && vt < 0) leave |= 1u << (4 * u + j);
          act |= (uint32_t)(on && vt >= 0) << j;
          const uint32_t ut = ((uint32_t)s << kGridTwShift) | (uint32_t)row_bond_site(4 * g + j, magic16);
          packed[j] = (ut << 16) | ((uint32_t)vt & 0xFFFFu);
        }
        tile_join_compact(par, stage[wave], staged, act, packed);
      }
      uint32_t pslot = reserve_slots<kLeaveBits>(__popc(leave), &n_out);
      if (leave) {  // static indices only: the register arrays must not spill
        at = cur;
#pragma unroll
        for (int u = 0; u < G; ++u, at = advance(at, 1)) {
          const int32_t s = at.s;
          const int32_t g = group(at);
          const int32_t c4[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if ((leave >> (4 * u + j)) & 1u) {
              const int64_t site = u0 + (int64_t)s * geo.w + row_bond_site(4 * g + j, magic16);
              st_dev2(my_pairs + pslot++, make_int2((int32_t)site, c4[j]));
            }
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        c[u] = cn[u];
        o[u] = on[u];
      }
      rv = rvn;
      cur = advance(cur, G);
    }
    ok = rp_ok(iters, rv) && ok;  // requested by the last step
    for (int32_t vs = iters + 1; vs < n_vslots; ++vs) ok = rp_ok(vs, rp_load(vs)) && ok;
    if (tid < rows) {  // the end entry of each row (the last site's bond range)
      const int32_t rel = tid * w32 + row_len(tid);
      ok = buf_i32(rp, 4u * (uint32_t)rel) == (int32_t)((uint32_t)e_first + (uint32_t)deg * (uint32_t)rel) && ok;
    }
    drain_joins(par, stage[wave], staged);  // what is left on the stack
    affine = __syncthreads_and(ok) != 0;
    if (!affine) {
      init_par();
      __syncthreads();
    }
  }
  if (!affine) {
    // ---- rows: one tile row per pass, kGridTw / kTileBlock sites per lane,
    // every bond of a site in turn, read with plain loads
    for (int32_t s = 0; s < rows; ++s) {
      const int32_t len = seg_len(s);
      const int64_t us = u0 + (int64_t)s * geo.w;
#pragma unroll
      for (int k = 0; k < kGridTw / kTileBlock; ++k) {
        const int32_t cc = k * kTileBlock + tid;
        if (cc >= len) continue;
        const int64_t u = us + cc;
        const int32_t ut = (s << kGridTwShift) | cc;
        const int32_t b0 = row_ptr[u], b1 = row_ptr[u + 1];
        for (int32_t e = b0; e < b1; ++e) {
          if ((HAS_OCC && occ[e] == 0) || (DRAW && !philox_occupied(rng, (uint64_t)e))) continue;
          const int32_t v = col[e];
          const int32_t vt = slot_of(v);
          if (vt >= 0) {
            lds16_unite(par, ut, vt);
          } else {
            const uint32_t sl =
                __hip_atomic_fetch_add(&n_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            st_dev2(my_pairs + sl, make_int2((int32_t)u, v));
          }
        }
      }
    }
  }
  __syncthreads();
  // the tile's labels: each site's ancestor kEpiRounds + 1 links up its
  // tile-local tree -- its tile-local root for all but the rare deeper
  // chains, which the cross kernel and the flatten finish in global memory
  // (a check for them and a divergent chase to the root cost more here than
  // the few extra global steps they cause).  A pass takes kEpiRuns runs of
  // 4 kTileBlock consecutive slots, four per lane (a run covers whole tile
  // rows), all their chases in lockstep; 16-byte stores when the label array
  // and the row length allow it
  const bool vec = ((reinterpret_cast<uintptr_t>(label + u0) & 15) == 0) && (geo.w % 4 == 0);
  const __amdgpu_buffer_rsrc_t rl = make_rsrc(label + u0, vec && fast ? (uint32_t)span_sites * 4u : 0u);
  auto gid = [&](int32_t t) {
    return (int32_t)(u0 + (int64_t)(t >> kGridTwShift) * geo.w + (t & (kGridTw - 1)));
  };
  constexpr int32_t kRun = 4 * kTileBlock;  // slots per run
  constexpr int E = kEpiRuns;
  const int32_t n_runs = (rows * kGridTw + kRun - 1) / kRun;
  for (int32_t q0 = 0; q0 < n_runs; q0 += E) {
    int32_t x[4 * E];
#pragma unroll
    for (int h = 0; h < E; ++h) {
      const int32_t t = min(q0 + h, n_runs - 1) * kRun + 4 * tid;  // a missing run repeats the last
      const uint2 wv = reinterpret_cast<const uint2*>(par)[t >> 2];
      x[4 * h + 0] = (int32_t)(wv.x & 0xFFFFu);
      x[4 * h + 1] = (int32_t)(wv.x >> 16);
      x[4 * h + 2] = (int32_t)(wv.y & 0xFFFFu);
      x[4 * h + 3] = (int32_t)(wv.y >> 16);
    }
#pragma unroll
    for (int r = 0; r < kEpiRounds; ++r)
#pragma unroll
      for (int k = 0; k < 4 * E; ++k) x[k] = lds16_ld(par + x[k]);  // a root reads itself
#pragma unroll
    for (int h = 0; h < E; ++h) {
      if (q0 + h >= n_runs) continue;
      const int32_t t = (q0 + h) * kRun + 4 * tid;
      const int32_t s = t >> kGridTwShift, cc = t & (kGridTw - 1);
      const int32_t len = row_len(s);  // 0 past the last row
      if (cc >= len) continue;
      if (vec && fast && cc + 4 <= len) {
        st_dev4(rl, 4u * (uint32_t)(s * w32 + cc),
                make_int4(gid(x[4 * h]), gid(x[4 * h + 1]), gid(x[4 * h + 2]), gid(x[4 * h + 3])));
      } else {
        const int64_t us = u0 + (int64_t)s * geo.w;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (cc + k < len) st_dev(label + us + cc + k, gid(x[4 * h + k]));
      }
    }
  }
  if (tid == 0) st_dev2(seg + blockIdx.x, make_int2((int32_t)region, (int32_t)n_out));
}

// Cross kernel: one workgroup per tile (tiles renumbered so that each XCD
// takes a contiguous range of them and its L2 holds the neighbouring tiles
// those joins touch) walks the tile's leaving-bond pairs in chunks.  Before
// anything touches global atomics, a chunk is reduced in LDS:
//   1. every pair (u, v) is replaced by (label[u], label[v]) -- after the
//      tile kernel these are (nearly always) tile-local roots, so many pairs
//      coincide (a cluster crosses a tile boundary at many bonds);
//   2. those labels are entered in a hash table (open addressing; a chunk of
//      kCrossChunk pairs has at most 2 kCrossChunk distinct labels, so the
//      table of kCrossSlots never fills), and the pairs are joined there with
//      the LDS union-find on slot numbers;
//   3. every table entry that is not the root of its local component is
//      listed (compactly, so that every lane of the next step has work), and
//      each listed entry issues one global join, Algorithm 1 in global
//      memory, with the label at the component's root slot.
// The global joins are a spanning forest of the chunk's pairs, so the result
// is the same connectivity with far fewer global chases and atomics: above
// the threshold, where nearly every leaving bond belongs to the spanning
// cluster, a chunk reduces to a handful of joins instead of thousands of
// atomics on the same few addresses.
constexpr int kCrossBlock = 512;
constexpr int kCrossPer = 1;  // pairs (and later joins) a lane carries in lockstep
constexpr int kCrossJoinPer = 1;  // global joins a lane carries in lockstep
constexpr int kCrossSplit = 1;  // workgroups per tile, each taking every kCrossSplit-th chunk
constexpr int kCrossChunk = kCrossPer * kCrossBlock;
constexpr int kCrossSlots = 2 * kCrossChunk;
constexpr int32_t kEmpty = -1;
static_assert((kCrossSlots & (kCrossSlots - 1)) == 0 && kCrossSlots <= 65536, "slot ids are 16-bit");

// Table slots of the 2P labels a lane holds, inserting the absent ones:
// linear probing in lockstep, one compare-and-swap per label per round (a
// label already placed re-tries its own slot, which fails harmlessly), until
// every label of the wavefront has its slot.
template <int P>
__device__ __forceinline__ void slots_of(int32_t* keys, int32_t (&a)[P], int32_t (&b)[P]) {
  constexpr int kBits = __builtin_ctz(kCrossSlots);
  int32_t ka[P], kb[P];
  uint32_t open = 0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    ka[k] = a[k];
    kb[k] = b[k];
    a[k] = (int32_t)(((uint32_t)ka[k] * 0x9E3779B1u) >> (32 - kBits));
    b[k] = (int32_t)(((uint32_t)kb[k] * 0x9E3779B1u) >> (32 - kBits));
  }
  open = (1u << (2 * P)) - 1u;
  while (__any(open != 0)) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      int32_t sa = kEmpty, sb = kEmpty;
      __hip_atomic_compare_exchange_strong(keys + a[k], &sa, ka[k], __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_compare_exchange_strong(keys + b[k], &sb, kb[k], __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
      if ((open >> k) & 1u) {
        if (sa == kEmpty || sa == ka[k])
          open &= ~(1u << k);
        else
          a[k] = (a[k] + 1) & (kCrossSlots - 1);
      }
      if ((open >> (P + k)) & 1u) {
        if (sb == kEmpty || sb == kb[k])
          open &= ~(1u << (P + k));
        else
          b[k] = (b[k] + 1) & (kCrossSlots - 1);
      }
    }
  }
}

__global__ void __launch_bounds__(kCrossBlock)
    k_csr_cross(const int2* __restrict__ pairs, const int2* __restrict__ seg, int32_t* label) {
  __shared__ int32_t keys[kCrossSlots];
  __shared__ uint16_t lpar[kCrossSlots];
  // the join list: at most one per table entry less one per component, so
  // kCrossSlots - 1 entries; its last word is the list's length (this keeps
  // the kernel at 40 KB of LDS, four workgroups per CU)
  __shared__ uint32_t joins[kCrossSlots];
  uint32_t& n_join = joins[kCrossSlots - 1];
  constexpr int P = kCrossPer;
  const int tid = threadIdx.x;
  const uint32_t id = xcd_block_id();
  const uint32_t tile = id / kCrossSplit;
  const int2 sc = seg[tile];
  const int2* p = pairs + sc.x;
  const int32_t count = sc.y;
  bool unused = false;
  for (int32_t c0 = (int32_t)(id % kCrossSplit) * kCrossChunk; c0 < count; c0 += kCrossSplit * kCrossChunk) {
    for (int s = tid; s < kCrossSlots; s += kCrossBlock) keys[s] = kEmpty;
    if (tid == 0) n_join = 0;
    for (int w = tid; w < kCrossSlots / 2; w += kCrossBlock)
      reinterpret_cast<uint32_t*>(lpar)[w] = (uint32_t)(2 * w) | ((uint32_t)(2 * w + 1) << 16);
    __syncthreads();
    // 1. the chunk's pairs and their current labels (clamped loads: pairs past
    //    the end repeat the last one and are dropped below)
    int32_t a[P], b[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int2 e = p[min(c0 + k * kCrossBlock + tid, count - 1)];
      a[k] = e.x;
      b[k] = e.y;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      a[k] = lab_ld(label + a[k]);
      b[k] = lab_ld(label + b[k]);
    }
    // 2. table slots, joined in LDS (labels of pairs past the end are
    //    entered too, harmlessly: they repeat the chunk's last pair)
    bool in[P];
#pragma unroll
    for (int k = 0; k < P; ++k) in[k] = c0 + k * kCrossBlock + tid < count && a[k] != b[k];
    slots_of<P>(keys, a, b);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      a[k] = in[k] ? a[k] : 0;
      b[k] = in[k] ? b[k] : 0;
    }
    lds16_unite_lockstep<P, 1>(lpar, a, b);
    __syncthreads();
    // 3. the entries below their local root, listed compactly (slot and
    //    root slot, 16 bits each; one LDS atomic per wavefront and round)
    for (int s0 = 0; s0 < kCrossSlots; s0 += kCrossBlock) {
      const int s = s0 + tid;
      const int32_t r = keys[s] != kEmpty ? lds16_find(lpar, s) : s;
      const uint32_t slot = reserve_slots<1>(r != s ? 1u : 0u, &n_join);
      if (r != s) joins[slot] = ((uint32_t)s << 16) | (uint32_t)r;
    }
    __syncthreads();
    // 4. one global join per listed entry, kCrossJoinPer per lane in lockstep
    constexpr int J = kCrossJoinPer;
    const int32_t nj = (int32_t)n_join;
    for (int32_t j0 = 0; j0 < nj; j0 += J * kCrossBlock) {
      int32_t x[J], y[J];
#pragma unroll
      for (int k = 0; k < J; ++k) {
        const int32_t j = j0 + k * kCrossBlock + tid;
        const uint32_t e = joins[j < nj ? j : 0];
        x[k] = j < nj ? keys[e >> 16] : 0;
        y[k] = j < nj ? keys[e & 0xFFFFu] : 0;
      }
      unite_lockstep<J, 2, false>(label, x, y, unused);
    }
    __syncthreads();  // the table and the list are reset for the next chunk
  }
}

// Step (iv) for the CSR path: one workgroup per window of kFlatWin sites,
// staged in LDS with 16-byte loads.  After the tile and cross kernels a
// site's label is (nearly always) its tile-local root, often inside the same window, so
// the parent's label is an LDS read; only parents whose cluster was joined
// across tiles need a chase in global memory, and its result is cached in
// the window (every thread sharing that parent then finds the root in LDS).
// Every value written is the site's final root; the window goes back with
// 16-byte stores.  Windows are renumbered so each XCD takes a contiguous run.
// These are the only plain (not device-scope) label stores of the CSR path:
// they are the call's final values, no later kernel of the call writes or
// atomically updates these words, and every writer of a word stores the same
// root.  Device-scope stores here cost 0.035 ms on the 2^26-site lattice
// (write-through of lines the window has just read), and 0.14 ms more for
// the scattered parent stores.
constexpr int kFlatWin = 16384;
constexpr int kFlatBlock = 1024;
constexpr int kFlatPer = 4;  // sites a lane resolves in lockstep (2, 6, 8, 16 measured slower)

__global__ void __launch_bounds__(kFlatBlock) k_flatten_window(int32_t* label, int64_t n) {
  __shared__ int32_t w[kFlatWin];
  const int64_t w0 = (int64_t)xcd_block_id() * kFlatWin;
  const int32_t cnt = (int32_t)min((int64_t)kFlatWin, n - w0);
  const int tid = threadIdx.x;
  const int32_t cnt4 = cnt >> 2;
  const int4* src4 = reinterpret_cast<const int4*>(label + w0);
  for (int32_t t = tid; t < cnt4; t += kFlatBlock) reinterpret_cast<int4*>(w)[t] = src4[t];
  for (int32_t t = 4 * cnt4 + tid; t < cnt; t += kFlatBlock) w[t] = label[w0 + t];
  __syncthreads();
  // kFlatPer sites per lane in lockstep: their parents' labels are read
  // together (from the window when the parent lies inside it, else from
  // global memory), then the chases that remain advance one link per round,
  // all of them at once, while any lane of the wavefront still has one
  constexpr int K = kFlatPer;
  for (int32_t t0 = 0; t0 < cnt; t0 += K * kFlatBlock) {
    int32_t p[K], q[K], x[K], px[K];
    uint32_t pin[K];
    bool need[K];
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = lds_ld(w + min(t0 + k * kFlatBlock + tid, cnt - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      pin[k] = (uint32_t)((int64_t)p[k] - w0);  // parent's window slot (>= cnt: outside)
      const bool inside = pin[k] < (uint32_t)cnt;
      const int32_t ql = lds_ld(w + (inside ? pin[k] : 0u));
      const int32_t qg = lab_ld(label + (inside ? 0 : p[k]));
      q[k] = inside ? ql : qg;  // the parent's label
      x[k] = q[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int32_t t = t0 + k * kFlatBlock + tid;
      // a root, or a site whose parent is a root, is final already
      need[k] = t < cnt && p[k] != (int32_t)(w0 + t) && x[k] != p[k];
      px[k] = lab_ld(label + (need[k] ? x[k] : 0));
    }
    for (;;) {
      bool open = false;
#pragma unroll
      for (int k = 0; k < K; ++k) open = open || (need[k] && px[k] != x[k]);
      if (!__any(open)) break;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        // the load is unconditional (index 0 when idle); an idle chase keeps
        // its value
        const bool go = need[k] && px[k] != x[k];
        x[k] = go ? px[k] : x[k];
        const int32_t nx = lab_ld(label + (go ? x[k] : 0));
        px[k] = go ? nx : px[k];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!need[k]) continue;
      const int32_t t = t0 + k * kFlatBlock + tid;
      if (x[k] != q[k]) {  // the parent's final root, for the sites sharing it
        if (pin[k] < (uint32_t)cnt)
          lds_st(w + pin[k], x[k]);
        else
          label[p[k]] = x[k];  // a final root, as every writer of p stores
      }
      lds_st(w + t, x[k]);
    }
  }
  __syncthreads();
  int4* dst4 = reinterpret_cast<int4*>(label + w0);
  for (int32_t t = tid; t < cnt4; t += kFlatBlock) dst4[t] = reinterpret_cast<const int4*>(w)[t];
  for (int32_t t = 4 * cnt4 + tid; t < cnt; t += kFlatBlock) label[w0 + t] = w[t];
}

// Step (iv) for grid tiles.  After the tile and cross kernels a site's label
// is (nearly always) its tile-local root: the smallest id of its cluster
// inside its grid tile, so a site of the same tile rows or above and, for
// nearly every cluster, only a few hundred columns away.  A window of the full
// tile height (kGridTh rows) by kFlatCols columns, aligned with the tiles,
// therefore holds the parent of nearly every one of its sites (97% on the
// triangle lattice at p_c with 512 columns, against 22% for a window of two
// whole rows of 8192 sites).  One workgroup per window; a lane owns four
// 16-byte groups of a row (16 slots):
//   load     the groups into LDS; the lane notes its slots whose label lies
//            outside the window (a tile root joined across tiles, a parent
//            further away);
//   phase 1  without waiting for the other lanes, those slots are chased to
//            their roots in global memory, kFlatChase chases per lane in
//            flight, and marked final in LDS (bit 31: labels are below
//            2^31 - 1);
//   phase 2  every group is read back from LDS and each slot resolved:
//            marked, a root, or its parent's slot read -- after phase 1 an
//            unmarked label always lies inside the window, so this follows
//            labels in LDS only -- and the group goes to global memory at
//            once with a 16-byte store.
// Per slot this is a few LDS accesses and a dozen VALU operations; what the
// streaming passes do not hide is the latency of the phase-1 chases through
// the forest of joined tile roots.  The final values are plain stores, for
// the same reason as the windowed flatten above: no later kernel of the call
// touches these words.  On the 2^26-site triangle lattice this kernel takes
// 0.156 ms against 0.170 ms for the windowed flatten (0.107 ms with the two
// phases left out, 0.113 ms with phase 1 alone left out); 256-column
// windows of 512 or 256 lanes measured 0.185 / 0.255 ms.
constexpr int kFlatColsShift = 9;
constexpr int kFlatGridBlock = 1024;
constexpr int kFlatCols = 1 << kFlatColsShift;
constexpr int kFlatSlots = kGridTh * kFlatCols;
constexpr int kFlatGroups = kFlatSlots / (4 * kFlatGridBlock);  // 16-byte groups of one lane
constexpr int kFlatChase = 2;                                // global chases a lane keeps in flight (1, 4, 8 measured slower)
constexpr int32_t kFinal = INT32_MIN;                        // LDS mark: the slot holds its final root
static_assert(kGridTw % kFlatCols == 0, "windows must not straddle grid tiles");
static_assert(kFlatSlots % (4 * kFlatGridBlock) == 0 && 4 * kFlatGroups <= 32 && kFlatGroups % 2 == 0,
              "whole 16-byte groups per lane, pending slots in a 32-bit mask, groups in pairs");

template <bool POW2>
__global__ void __launch_bounds__(kFlatGridBlock) k_flatten_grid(int32_t* label, GridGeo geo, int32_t wins_x) {
  __shared__ int32_t w[kFlatSlots];
  const int tid = threadIdx.x;
  const int32_t b = (int32_t)xcd_block_id();
  const int32_t wy = b / wins_x, wx = b - wy * wins_x;
  const int64_t base64 = (int64_t)wy * kGridTh * geo.w + (int64_t)wx * kFlatCols;
  if (base64 >= geo.n) return;  // the partial last row ends left of this window: no site
  const uint32_t n = (uint32_t)geo.n;
  const uint32_t w32 = (uint32_t)geo.w;  // w < n <= 2^31 - 1
  const uint32_t rows = (uint32_t)min((int64_t)kGridTh, geo.h - (int64_t)wy * kGridTh);
  const uint32_t cw = min((uint32_t)kFlatCols, w32 - (uint32_t)wx * kFlatCols);  // a multiple of 4, as w is
  const uint32_t base = (uint32_t)base64;
  const uint32_t lim = rows * w32;  // <= kGridTh w < 2^32

  // Slot of site v, or -1 when v lies outside the window.  POW2: bit fields;
  // otherwise a float quotient corrected by one step (the row within reach
  // is below kGridTh).
  auto slot_of = [&](int32_t v) -> int32_t {
    const uint32_t d = (uint32_t)v - base;  // wraps to >= lim when v < base
    if (d >= lim) return -1;
    uint32_t r, c;
    if (POW2) {
      r = d >> geo.w_shift;
      c = d & (w32 - 1u);
    } else {
      int32_t q = (int32_t)((float)d * geo.inv_w);
      int32_t e = (int32_t)d - q * (int32_t)w32;
      if (e < 0) {
        --q;
        e += (int32_t)w32;
      } else if (e >= (int32_t)w32) {
        ++q;
        e -= (int32_t)w32;
      }
      r = (uint32_t)q;
      c = (uint32_t)e;
    }
    return c < cw ? (int32_t)((r << kFlatColsShift) | c) : -1;
  };

  // The lane's groups: group i is slots 4 (tid + i kFlatGridBlock) + 0..3, in
  // window row r0 + kRowStep i, columns c0 + 0..3 (with 512 columns and 1024
  // lanes: row (tid >> 7) + 8 i, columns 4 (tid & 127) + 0..3).
  const uint32_t c0 = (uint32_t)(tid & (kFlatCols / 4 - 1)) * 4u;
  const uint32_t r0 = (uint32_t)tid / (kFlatCols / 4);
  constexpr uint32_t kRowStep = kFlatGridBlock / (kFlatCols / 4);
  auto gsite = [&](int i) { return base + (r0 + kRowStep * i) * w32 + c0; };  // < 2^32: rows * w < n + w
  auto gvalid = [&](int i) { return r0 + kRowStep * i < rows && c0 < cw && gsite(i) < n; };
  auto gslot = [&](int i) { return 4 * (tid + i * kFlatGridBlock); };

  // ---- load
  uint32_t pend = 0;  // bit 4 i + j: slot j of group i needs a chase in global memory
#pragma unroll
  for (int i = 0; i < kFlatGroups; ++i) {
    if (!gvalid(i)) continue;
    const uint32_t g = gsite(i);
    int4 v;
    if (g + 4u <= n) {
      v = *reinterpret_cast<const int4*>(label + g);
    } else {  // the end of the last row
      v.x = label[g];
      v.y = g + 1u < n ? label[g + 1u] : (int32_t)g + 1;
      v.z = g + 2u < n ? label[g + 2u] : (int32_t)g + 2;
      v.w = g + 3u < n ? label[g + 3u] : (int32_t)g + 3;
    }
    *reinterpret_cast<int4*>(w + gslot(i)) = v;
    const int32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (g + (uint32_t)j < n && slot_of(vv[j]) < 0) pend |= 1u << (4 * i + j);
  }

  // ---- phase 1: labels outside the window, chased in global memory.  A
  // lane reads and marks only its own slots, so it starts as soon as its own
  // loads are in LDS.  A chase that took more than one step also stores the
  // root it found at the label it started from (a site outside the window,
  // usually a tile root): windows that reach that site later find the root
  // in one step.  Like the window's own stores this is a final value.
  {
    // per chase: its slot (-1: idle), the site it is at, the site it started
    // from and that site's label once read
    int32_t cs[kFlatChase], cx[kFlatChase], cfrom[kFlatChase], cnext[kFlatChase];
#pragma unroll
    for (int c = 0; c < kFlatChase; ++c) cs[c] = -1;
    for (;;) {
      bool busy = false;
#pragma unroll
      for (int c = 0; c < kFlatChase; ++c) {
        if (cs[c] < 0 && pend != 0) {
          const int k = __builtin_ctz(pend);
          pend &= pend - 1u;
          cs[c] = gslot(k >> 2) + (k & 3);
          cx[c] = lds_ld(w + cs[c]);
          cfrom[c] = cx[c];
          cnext[c] = cx[c];
        }
        busy = busy || cs[c] >= 0;
      }
      if (!__any(busy)) break;
      int32_t cy[kFlatChase];
#pragma unroll
      for (int c = 0; c < kFlatChase; ++c) cy[c] = lab_ld(label + (cs[c] >= 0 ? cx[c] : 0));
#pragma unroll
      for (int c = 0; c < kFlatChase; ++c) {
        const bool root = cs[c] >= 0 && cy[c] == cx[c];
        if (root) lds_st(w + cs[c], cx[c] | kFinal);
        if (root && cnext[c] != cx[c]) label[cfrom[c]] = cx[c];  // more than one step
        cnext[c] = cs[c] >= 0 && cnext[c] == cfrom[c] ? cy[c] : cnext[c];
        cx[c] = cs[c] >= 0 ? cy[c] : cx[c];
        cs[c] = root ? -1 : cs[c];
      }
    }
  }
  __syncthreads();

  // ---- phase 2: the other slots, in LDS; each group stored when resolved
#pragma unroll
  for (int i0 = 0; i0 < kFlatGroups; i0 += 2) {
    int32_t v[8], y[8], ps[8];
    bool todo[8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int4 t = gvalid(i0 + h) ? *reinterpret_cast<const int4*>(w + gslot(i0 + h)) : int4{-1, -1, -1, -1};
      v[4 * h] = t.x;
      v[4 * h + 1] = t.y;
      v[4 * h + 2] = t.z;
      v[4 * h + 3] = t.w;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int32_t id = (int32_t)(gsite(i0 + (k >> 2)) + (uint32_t)(k & 3));
      todo[k] = v[k] >= 0 && v[k] != id;  // not marked, not a root
      ps[k] = todo[k] ? slot_of(v[k]) : 0;  // inside the window: unmarked labels are, after phase 1
      y[k] = lds_ld(w + ps[k]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (!todo[k]) continue;
      int32_t x = v[k], yy = y[k];
      if (yy >= 0 && yy != x) {  // the parent is neither marked nor a root: follow on
        do {
          x = yy;
          yy = lds_ld(w + slot_of(x));
        } while (yy >= 0 && yy != x);
        // for the sites that share this parent
        lds_st(w + ps[k], (yy < 0 ? yy : x) | kFinal);
      }
      v[k] = yy < 0 ? yy : x;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!gvalid(i0 + h)) continue;
      const uint32_t g = gsite(i0 + h);
      const int4 t{v[4 * h] & INT32_MAX, v[4 * h + 1] & INT32_MAX, v[4 * h + 2] & INT32_MAX,
                   v[4 * h + 3] & INT32_MAX};
      if (g + 4u <= n) {
        *reinterpret_cast<int4*>(label + g) = t;
      } else {
        label[g] = t.x;
        if (g + 1u < n) label[g + 1u] = t.y;
        if (g + 2u < n) label[g + 2u] = t.z;
      }
    }
  }
}

// Tiles of the id grid of row length w: grid tiles when the rows are longer
// than a grid tile, w is a multiple of 4 and there are at least kGridTh rows,
// else slabs of kCsrTile consecutive ids (w <= 0: no grid).
static bool use_grid(int64_t n, int64_t w) {
  // w a multiple of 4 keeps every tile row's bonds on the same 4-byte
  // alignment of the occupancy mask as the tile's first bond
  return w > kGridTw && w < n && w % 4 == 0 && (n + w - 1) / w >= kGridTh;
}

static int64_t csr_tiles(int64_t n, int64_t w) {
  if (!use_grid(n, w)) return (n + kCsrTile - 1) / kCsrTile;
  const int64_t h = (n + w - 1) / w;
  return ((h + kGridTh - 1) / kGridTh) * ((w + kGridTw - 1) / kGridTw);
}

// The tile table is sized for any grid width: with at least kGridTh rows of
// more than kGridTw sites, ceil(h/kGridTh) ceil(w/kGridTw) <= 4 ceil(n/65536) + 2
// (kGridTh kGridTw = 65536).
static size_t csr_seg_bytes(int64_t n_sites) {
  const int64_t max_tiles = 4 * ((n_sites + kCsrTile - 1) / kCsrTile) + 2;
  return ((size_t)max_tiles * sizeof(int2) + 255) & ~(size_t)255;
}

size_t csr_workspace_bytes(int64_t n_sites, int64_t n_bonds) {
  if (n_sites <= kCsrTile) return 0;
  return csr_seg_bytes(n_sites) + (size_t)n_bonds * sizeof(int2);
}

ccl_status launch_label_csr(int64_t n, int64_t grid_w, const int32_t* row_ptr, const int32_t* col,
                            const uint8_t* occ, const PhiloxOcc* draw, int32_t* label,
                            void* workspace, hipStream_t s, const DeviceInfo& d) {
  if (n == 0) return CCL_OK;
  const bool grid = use_grid(n, grid_w);
  const int64_t n_tiles = csr_tiles(n, grid_w);
  if (n_tiles > 4 * ((n + kCsrTile - 1) / kCsrTile) + 2) return CCL_ERR_INVALID_VALUE;  // cannot happen
  int2* seg = nullptr;
  int2* pairs = nullptr;
  if (n_tiles > 1) {  // a single tile has no leaving bonds and needs no workspace
    seg = static_cast<int2*>(workspace);
    pairs = reinterpret_cast<int2*>(static_cast<char*>(workspace) + csr_seg_bytes(n));
  }
  const PhiloxOcc rng = draw != nullptr ? *draw : PhiloxOcc{0, 0, 0};
  GridGeo geo{};
  if (grid) {
    geo.n = n;
    geo.w = grid_w;
    geo.h = (n + grid_w - 1) / grid_w;
    geo.tiles_x = (int32_t)((grid_w + kGridTw - 1) / kGridTw);
    geo.inv_w = 1.0f / (float)grid_w;
    geo.w_shift = 0;
    while (((int64_t)1 << geo.w_shift) < grid_w) ++geo.w_shift;
  }
  if (grid) {
    const bool pow2 = ((int64_t)1 << geo.w_shift) == grid_w;
#define CCL_GRID_TILE(OCC)                                                                      \
  do {                                                                                          \
    if (pow2)                                                                                   \
      CCL_LAUNCH("ccl_csr_tile", (k_csr_tile_grid<OCC, true>), (unsigned)n_tiles, kTileBlock, 0, s, \
                 geo, row_ptr, col, occ, label, pairs, seg, rng);                               \
    else                                                                                        \
      CCL_LAUNCH("ccl_csr_tile", (k_csr_tile_grid<OCC, false>), (unsigned)n_tiles, kTileBlock, 0, s, \
                 geo, row_ptr, col, occ, label, pairs, seg, rng);                               \
  } while (0)
    if (occ != nullptr)
      CCL_GRID_TILE(kOccMask);
    else if (draw != nullptr)
      CCL_GRID_TILE(kOccDraw);
    else
      CCL_GRID_TILE(kOccAll);
#undef CCL_GRID_TILE
  } else if (occ != nullptr) {
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<kOccMask>, (unsigned)n_tiles, kTileBlock, 0, s, n,
               row_ptr, col, occ, label, pairs, seg, rng);
  } else if (draw != nullptr) {
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<kOccDraw>, (unsigned)n_tiles, kTileBlock, 0, s, n,
               row_ptr, col, occ, label, pairs, seg, rng);
  } else {
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<kOccAll>, (unsigned)n_tiles, kTileBlock, 0, s, n,
               row_ptr, col, occ, label, pairs, seg, rng);
  }
  if (n_tiles == 1 && !grid) return CCL_OK;  // one slab tile's labels are final (a grid has >= 2 tiles)
  CCL_LAUNCH("ccl_csr_cross", k_csr_cross, (unsigned)(n_tiles * kCrossSplit), kCrossBlock, 0, s, pairs, seg,
             label);
  if ((reinterpret_cast<uintptr_t>(label) & 15) != 0) return launch_flatten(n, label, s, d);
  if (grid) {
    const int32_t wins_x = (int32_t)((grid_w + kFlatCols - 1) / kFlatCols);
    const int64_t n_win = ((geo.h + kGridTh - 1) / kGridTh) * wins_x;
    if (((int64_t)1 << geo.w_shift) == grid_w)
      CCL_LAUNCH("ccl_flatten_grid", k_flatten_grid<true>, (unsigned)n_win, kFlatGridBlock, 0, s, label, geo, wins_x);
    else
      CCL_LAUNCH("ccl_flatten_grid", k_flatten_grid<false>, (unsigned)n_win, kFlatGridBlock, 0, s, label, geo, wins_x);
    return CCL_OK;
  }
  const unsigned n_win = (unsigned)((n + kFlatWin - 1) / kFlatWin);
  CCL_LAUNCH("ccl_flatten_window", k_flatten_window, n_win, kFlatBlock, 0, s, label, n);
  return CCL_OK;
}

// ---------------------------------------------------------------- checks

__global__ void __launch_bounds__(256)
    k_validate_csr(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                   int64_t n_col, unsigned long long* count) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long bad = 0;
  for (int64_t i = tid; i < n; i += stride) {
    const int32_t a = row_ptr[i], b = row_ptr[i + 1];
    bad += (b < a) ? 1ull : 0ull;
    bad += (i == 0 && a < 0) ? 1ull : 0ull;
    bad += (i == n - 1 && (int64_t)b > n_col) ? 1ull : 0ull;
  }
  for (int64_t e = tid; e < n_col; e += stride) {
    const int32_t v = col[e];
    bad += (v < 0 || (int64_t)v >= n) ? 1ull : 0ull;
  }
  if (bad) atomicAdd(count, bad);
}

ccl_status launch_validate_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                               int64_t n_col, unsigned long long* d_count, hipStream_t s,
                               const DeviceInfo& d) {
  const int64_t work = n > n_col ? n : n_col;
  if (work == 0) return CCL_OK;
  CCL_LAUNCH("ccl_validate_csr", k_validate_csr, grid_for(work, 256, 8, d), 256, 0, s, n, row_ptr,
             col, n_col, d_count);
  return CCL_OK;
}

}  // namespace ccl
