// Tile-local joins in LDS, shared by the CSR tile kernels and the batched
// tile items: a tile of up to 65536 sites keeps 16-bit tile-relative
// parents in LDS; each wavefront stages its occupied in-tile bonds and joins
// them in full batches of 64 (Algorithm 1 on the LDS forest); bonds that leave
// the tile get list slots reserved with ballots and one LDS atomic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uf.hpp"

namespace ccl {

constexpr int kTileBlock = 1024;
constexpr int kLdsRounds = 4;  // lockstep pointer-following rounds in LDS before the fallbacks

// Joins of the tile paths, compacted across the wavefront: each group of
// four bonds per lane appends its occupied in-tile bonds (bit j of `act`;
// `packed` holds the tile-relative ends, 16 bits each) to the wavefront's
// staging stack -- positions from a prefix count done with three ballots,
// since each lane has at most four -- and whenever the stack holds a full
// batch of 64, the top 64 entries are joined one per lane.  So the
// unoccupied majority of bond slots costs no join work and every batch is
// full; `staged` (wavefront-uniform) carries the rest to the next group.
// The stack is private to the wavefront, whose LDS accesses complete in
// order.
//
// A batch costs a fixed three LDS round trips: both ends' parents, one
// pointer-following step (with path halving), one masked-or link.  A pair
// that is not at two roots by then, or whose link found the higher root
// already linked, goes back on the stack as an equivalent pair -- the ends'
// current ancestors, or (previous parent, lower root), the pair Algorithm 1
// continues with -- and is finished by a later batch.  A lane waiting for a
// deep chase or a contended link thus holds up no other lane; the
// lockstep-to-the-slowest form needed eight to eleven round trips per batch
// on critical lattices.  Each pair that goes back has a strictly smaller sum
// of ends (parents are always below their children, and a displaced link's
// parent is below the root it hung under), so the stack drains.
constexpr int kJoinPer = 1;  // entries a lane joins per batch, their round trips shared
constexpr int kJoinBatch = 64 * kJoinPer;
constexpr int kStageCap = kJoinBatch - 1 + 256;  // leftover + one group of 64 x 4

// Joins stage[base, limit) (limit - base <= kJoinBatch), kJoinPer entries
// per lane; pairs that are not finished are written back from stage[base]
// on.  Returns how many.
__device__ __forceinline__ uint32_t join_batch(uint16_t* par, uint32_t* stage, uint32_t base,
                                               uint32_t limit) {
  constexpr int J = kJoinPer;
  const uint32_t lane = threadIdx.x & 63u;
  int32_t pa[J], pb[J], ga[J], gb[J];
#pragma unroll
  for (int k = 0; k < J; ++k) {
    const uint32_t i = base + 64u * k + lane;
    const uint32_t e = i < limit ? stage[i] : 0u;  // (0, 0): a no-op pair
    pa[k] = (int32_t)(e >> 16);
    pb[k] = (int32_t)(e & 0xFFFFu);
  }
  int32_t a[J], b[J];
#pragma unroll
  for (int k = 0; k < J; ++k) {
    a[k] = pa[k];
    b[k] = pb[k];
    pa[k] = lds16_ld(par + a[k]);
    pb[k] = lds16_ld(par + b[k]);
  }
#pragma unroll
  for (int k = 0; k < J; ++k) {
    ga[k] = lds16_ld(par + pa[k]);
    gb[k] = lds16_ld(par + pb[k]);
  }
  bool roots[J], go[J];
  int32_t hi[J], lo[J];
  uint32_t sh[J], off[J], msk[J], bits[J], ret[J];
#pragma unroll
  for (int k = 0; k < J; ++k) {
    if (ga[k] != pa[k]) lds16_st(par + a[k], ga[k]);  // halving: a now hangs under its grandparent
    if (gb[k] != pb[k]) lds16_st(par + b[k], gb[k]);
    roots[k] = ga[k] == pa[k] && gb[k] == pb[k];
    hi[k] = max(pa[k], pb[k]);
    lo[k] = min(pa[k], pb[k]);
    go[k] = roots[k] && hi[k] != lo[k];
    // the link: hi's 16-bit half of its word takes lo; a lane with nothing
    // to link issues an empty mask on the word of its own end
    sh[k] = (uint32_t)(hi[k] & 1) * 16u;
    off[k] = (uint32_t)reinterpret_cast<uintptr_t>(par) + 4u * (uint32_t)(hi[k] >> 1);
    msk[k] = go[k] ? 0xFFFFu << sh[k] : 0u;
    bits[k] = go[k] ? (uint32_t)lo[k] << sh[k] : 0u;
  }
  lds_mskor<J>(ret, off, msk, bits);
  uint32_t pos = base, total = 0;
#pragma unroll
  for (int k = 0; k < J; ++k) {
    const int32_t old = (int32_t)((ret[k] >> sh[k]) & 0xFFFFu);
    const bool displaced = go[k] && old != hi[k] && old != lo[k];
    const bool again = !roots[k] || displaced;
    const uint32_t back = !roots[k] ? ((uint32_t)ga[k] << 16) | (uint32_t)gb[k]
                                    : ((uint32_t)old << 16) | (uint32_t)lo[k];
    const uint64_t m = __ballot(again);
    if (again)
      stage[pos + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = back;
    const uint32_t c = (uint32_t)__popcll(m);
    pos += c;
    total += c;
  }
  return total;
}

// Joins everything left on the stack (at the end of a tile's bond stream).
__device__ __forceinline__ void drain_joins(uint16_t* par, uint32_t* stage, uint32_t staged) {
  while (staged > 0) {  // wavefront-uniform
    const uint32_t take = staged < (uint32_t)kJoinBatch ? staged : (uint32_t)kJoinBatch;
    staged -= take;
    staged += join_batch(par, stage, staged, staged + take);
  }
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
    staged += join_batch(par, stage, staged, staged + kJoinBatch);
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

}  // namespace ccl
