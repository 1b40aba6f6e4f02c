// Bond occupancy drawn on the device: Philox4x32-10, the counter-based
// generator of Salmon, Moraes, Dror and Shaw (SC'11), written here from its
// published definition (ten rounds of two 32x32->64-bit products, the key
// bumped by the Weyl constants between rounds).  Word j of block b of stream
// s under seed K is output word j of Philox4x32-10 with counter
// (b mod 2^32, b div 2^32, s, 0) and key (K mod 2^32, K div 2^32); word w of
// the stream is word w mod 4 of block w div 4.  A bond with word u is
// occupied when u < floor(p 2^32) (p >= 1: always).  This replaces the
// paper's cuRAND draws (section 4) so that a Monte-Carlo loop never moves a
// mask across PCIe.
#include "common.hpp"
#include "mem.hpp"
#include "philox.hpp"

namespace ccl {

constexpr int kRngBlock = 256;

// One Philox block per lane: the words of block b that fall in
// [first, first + n) are written (as words, or as occupancy bytes; packed:
// first is a multiple of four and out 4-byte aligned, so a block wholly in
// range writes its four bytes with one 4-byte store).
template <bool BYTES>
__global__ void __launch_bounds__(kRngBlock)
    k_philox(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n, uint64_t threshold,
             void* __restrict__ out, bool packed) {
  const uint64_t b0 = first >> 2, b1 = (first + (uint64_t)n - 1) >> 2;
  const uint64_t stride = (uint64_t)gridDim.x * kRngBlock;
  for (uint64_t b = b0 + (uint64_t)blockIdx.x * kRngBlock + threadIdx.x; b <= b1; b += stride) {
    const uint4 w = philox_block(seed, stream_id, b);
    const uint32_t word[4] = {w.x, w.y, w.z, w.w};
    const uint64_t lo = b << 2;
    if (BYTES && packed && lo >= first && lo + 4 <= first + (uint64_t)n) {
      // the whole block is in range and its four bytes share one aligned word
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) v |= (uint32_t)((uint64_t)word[j] < threshold) << (8 * j);
      st_dev(reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(out) + (lo - first)), v);
      continue;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t idx = (b << 2) + (uint64_t)j;
      if (idx < first || idx >= first + (uint64_t)n) continue;
      if (BYTES)
        st_dev(static_cast<uint8_t*>(out) + (idx - first), (uint8_t)((uint64_t)word[j] < threshold ? 1 : 0));
      else
        st_dev(static_cast<uint32_t*>(out) + (idx - first), word[j]);
    }
  }
}

ccl_status launch_philox(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n,
                         uint64_t threshold, bool bytes, void* out, hipStream_t s,
                         const DeviceInfo& d) {
  const int64_t blocks = (int64_t)(((first + (uint64_t)n - 1) >> 2) - (first >> 2)) + 1;
  const unsigned g = grid_for(blocks, kRngBlock, 8, d);
  const bool packed = (first & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 3) == 0;
  if (bytes)
    CCL_LAUNCH("ccl_bernoulli", k_philox<true>, g, kRngBlock, 0, s, seed, stream_id, first, n,
               threshold, out, packed);
  else
    CCL_LAUNCH("ccl_philox_u32", k_philox<false>, g, kRngBlock, 0, s, seed, stream_id, first, n,
               threshold, out, packed);
  return CCL_OK;
}

}  // namespace ccl
