// CSR labeling with tile-local joins in LDS.
//
// Sites are cut into tiles of kCsrTile (65536) consecutive ids; a tile owns its sites
// and the bonds stored in its rows.  Three kernels:
//   1. tile kernel, one workgroup per tile: step (i) for the tile in LDS
//      (par[t] = t, 16-bit tile-relative entries: 128 KB), step (iii) --
//      Algorithm 1 on LDS, its atomicMin a 32-bit compare-and-swap -- for every
//      occupied bond whose two ends lie in the tile, a root chase in LDS, and
//      one coalesced store of the tile's labels (each site's tile-local root,
//      the tile's minimum member of its local cluster).  Occupied bonds that
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
#include "uf.hpp"

namespace ccl {

constexpr int kTileBlock = 1024;
constexpr int kTileShift = 16;
constexpr int kRowsPerThread = 4;  // rows per thread per iteration (row path)
constexpr int kDegFast = 4;        // bonds per row kept in registers (row path)
constexpr int kChunkRows = kTileBlock * kRowsPerThread;
constexpr int kGroupsPerIter = 3;  // groups of four bonds per lane per step (affine path)
constexpr int kLeaveBits = 5;  // a lane leaves at most 16 bonds per step: 5-bit counts
static_assert(4 * kGroupsPerIter < (1 << kLeaveBits) && kRowsPerThread * kDegFast < (1 << kLeaveBits),
              "a lane's leaving bonds per step must fit a count of kLeaveBits bits");
constexpr int kLdsRounds = 4;  // lockstep pointer-following rounds in LDS before the fallbacks
static_assert((1 << kTileShift) == kCsrTile, "tile size");

// Tile-relative row of tile-relative bond e in an affine tile of degree d,
// as e * ceil(2^20 / d) >> 20 (exact for d <= 4 and e < 2^18, which a tile of
// 65536 rows of at most 4 bonds satisfies); `magic` is ceil(2^20 / d).
__device__ __forceinline__ int32_t affine_row(int32_t e, uint32_t magic) {
  return (int32_t)(((uint64_t)(uint32_t)e * magic) >> 20);
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

// Joins of the affine tile path, compacted across the wavefront: each group
// of four bonds per lane appends its occupied in-tile bonds (bit j of `act`;
// `packed` holds the tile-relative ends, 16 bits each) to the wavefront's
// staging stack -- positions from a prefix count done with three ballots,
// since each lane has at most four -- and whenever the stack holds a full
// batch, the top kJoinPer * 64 entries are joined kJoinPer per lane in
// lockstep.  So the unoccupied majority of bond slots costs no join work and
// every lockstep join is full; `staged` (wavefront-uniform) carries the rest
// to the next group.  The stack is private to the wavefront, whose LDS
// accesses complete in order.
constexpr int kJoinPer = 1;  // joins per lane per batch (one measured fastest with the masked-or link)
constexpr int kJoinBatch = 64 * kJoinPer;
constexpr int kStageCap = kJoinBatch - 1 + 256;  // leftover + one group of 64 x 4

__device__ __forceinline__ void join_batch(uint16_t* par, const uint32_t* stage, uint32_t base,
                                           uint32_t limit) {
  const uint32_t lane = threadIdx.x & 63u;
  int32_t a[kJoinPer], b[kJoinPer];
#pragma unroll
  for (int h = 0; h < kJoinPer; ++h) {
    const uint32_t i = base + 64u * h + lane;
    const uint32_t v = i < limit ? stage[i] : 0u;  // (0, 0): a no-op bond
    a[h] = (int32_t)(v >> 16);
    b[h] = (int32_t)(v & 0xFFFFu);
  }
  lds16_unite_lockstep<kJoinPer, kLdsRounds>(par, a, b);
}

__device__ __forceinline__ void tile_join_compact(uint16_t* par, uint32_t* stage, uint32_t& staged,
                                                  uint32_t act, const uint32_t (&packed)[4]) {
  const uint32_t mine = __popc(act);
  const uint64_t b0 = __ballot(mine & 1u), b1 = __ballot(mine & 2u), b2 = __ballot(mine & 4u);
  auto below = [](uint64_t m) {  // set bits of m in lanes below this one
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  };
  uint32_t pos = staged + below(b0) + 2u * below(b1) + 4u * below(b2);
  staged += (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1) + 4u * (uint32_t)__popcll(b2);
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if ((act >> j) & 1u) stage[pos++] = packed[j];
  while (staged >= (uint32_t)kJoinBatch) {
    staged -= kJoinBatch;
    join_batch(par, stage, staged, staged + kJoinBatch);
  }
}

// Reserve `mine` (< 2^BITS) consecutive slots of a list for this lane: the
// lane's offset is a prefix count over the wavefront done with BITS ballots,
// and one LDS atomic per wavefront takes the wavefront's total.  Returns the
// lane's first slot.
template <int BITS>
__device__ __forceinline__ uint32_t reserve_slots(uint32_t mine, uint32_t* n_out) {
  uint32_t below = 0, total = 0;
#pragma unroll
  for (int i = 0; i < BITS; ++i) {
    const uint64_t m = __ballot((mine >> i) & 1u);
    below += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << i;
    total += (uint32_t)__popcll(m) << i;
  }
  uint32_t base = 0;
  if (total != 0) {  // wavefront-uniform
    if ((threadIdx.x & 63u) == 0)
      base = __hip_atomic_fetch_add(n_out, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
  }
  return base + below;
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
    if (staged > 0) join_batch(par, stage[wave], 0, staged);  // what is left on the stack
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

// Cross kernel: one workgroup per tile (tiles renumbered so that each XCD
// takes a contiguous range of them and its L2 holds the neighbouring tiles
// those joins touch) walks the tile's leaving-bond pairs in chunks.  Before
// anything touches global atomics, a chunk is reduced in LDS:
//   1. every pair (u, v) is replaced by (label[u], label[v]) -- after the
//      tile kernel these are tile-local roots, so many pairs coincide (a
//      cluster crosses a tile boundary at many bonds);
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
// site's label is its tile-local root, usually inside the same window, so
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
constexpr int kFlatPer = 8;  // sites a lane resolves in lockstep

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

size_t csr_workspace_bytes(int64_t n_sites, int64_t n_bonds) {
  if (n_sites <= kCsrTile) return 0;
  const int64_t n_tiles = (n_sites + kCsrTile - 1) / kCsrTile;
  const size_t seg = ((size_t)n_tiles * sizeof(int2) + 255) & ~(size_t)255;
  return seg + (size_t)n_bonds * sizeof(int2);
}

ccl_status launch_label_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                            const uint8_t* occ, const PhiloxOcc* draw, int32_t* label,
                            void* workspace, hipStream_t s, const DeviceInfo& d) {
  if (n == 0) return CCL_OK;
  const int64_t n_tiles = (n + kCsrTile - 1) / kCsrTile;
  int2* seg = nullptr;
  int2* pairs = nullptr;
  if (n_tiles > 1) {  // a single tile has no leaving bonds and needs no workspace
    seg = static_cast<int2*>(workspace);
    pairs = reinterpret_cast<int2*>(static_cast<char*>(workspace) +
                                    (((size_t)n_tiles * sizeof(int2) + 255) & ~(size_t)255));
  }
  const PhiloxOcc rng = draw != nullptr ? *draw : PhiloxOcc{0, 0, 0};
  if (occ != nullptr)
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<kOccMask>, (unsigned)n_tiles, kTileBlock, 0, s, n,
               row_ptr, col, occ, label, pairs, seg, rng);
  else if (draw != nullptr)
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<kOccDraw>, (unsigned)n_tiles, kTileBlock, 0, s, n,
               row_ptr, col, occ, label, pairs, seg, rng);
  else
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<kOccAll>, (unsigned)n_tiles, kTileBlock, 0, s, n,
               row_ptr, col, occ, label, pairs, seg, rng);
  if (n_tiles == 1) return CCL_OK;
  CCL_LAUNCH("ccl_csr_cross", k_csr_cross, (unsigned)(n_tiles * kCrossSplit), kCrossBlock, 0, s, pairs, seg,
             label);
  if ((reinterpret_cast<uintptr_t>(label) & 15) != 0) return launch_flatten(n, label, s, d);
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
