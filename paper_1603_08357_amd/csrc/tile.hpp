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
constexpr int kJoinBatch = 64;
constexpr int kStageCap = kJoinBatch - 1 + 256;  // leftover + one group of 64 x 4

// Joins stage[base, limit) (limit - base <= 64), one entry per lane; pairs
// that are not finished are written back from stage[base] on.  Returns how
// many.
__device__ __forceinline__ uint32_t join_batch(uint16_t* par, uint32_t* stage, uint32_t base,
                                               uint32_t limit) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t i = base + lane;
  const uint32_t e = i < limit ? stage[i] : 0u;  // (0, 0): a no-op pair
  int32_t a = (int32_t)(e >> 16), b = (int32_t)(e & 0xFFFFu);
  int32_t pa = lds16_ld(par + a), pb = lds16_ld(par + b);
  const int32_t ga = lds16_ld(par + pa), gb = lds16_ld(par + pb);
  if (ga != pa) lds16_st(par + a, ga);  // halving: a now hangs under its grandparent
  if (gb != pb) lds16_st(par + b, gb);
  const bool roots = ga == pa && gb == pb;
  const int32_t hi = max(pa, pb), lo = min(pa, pb);
  const bool go = roots && hi != lo;
  // the link: hi's 16-bit half of its word takes lo; a lane with nothing to
  // link issues an empty mask on the word of its own end
  const uint32_t sh = (uint32_t)(hi & 1) * 16u;
  uint32_t ret[1];
  const uint32_t off[1] = {(uint32_t)reinterpret_cast<uintptr_t>(par) + 4u * (uint32_t)(hi >> 1)};
  const uint32_t msk[1] = {go ? 0xFFFFu << sh : 0u};
  const uint32_t bits[1] = {go ? (uint32_t)lo << sh : 0u};
  lds_mskor<1>(ret, off, msk, bits);
  const int32_t old = (int32_t)((ret[0] >> sh) & 0xFFFFu);
  const bool displaced = go && old != hi && old != lo;
  const bool again = !roots || displaced;
  const uint32_t back = !roots ? ((uint32_t)ga << 16) | (uint32_t)gb : ((uint32_t)old << 16) | (uint32_t)lo;
  const uint64_t m = __ballot(again);
  if (again) {
    const uint32_t pos = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    stage[pos] = back;
  }
  return (uint32_t)__popcll(m);
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
