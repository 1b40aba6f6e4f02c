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

}  // namespace ccl
