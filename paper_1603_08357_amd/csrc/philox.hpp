// Philox4x32-10 on the device (Salmon, Moraes, Dror, Shaw, SC'11), written
// from its published definition: ten rounds, each two 32x32->64-bit products
// of counter words with the round multipliers, the key bumped by the Weyl
// constants between rounds.  Used to draw bond occupancy on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // both halves of each 32x32 product from one 64-bit product
    const uint64_t pa = (uint64_t)kPhiloxMulA * c.x, pb = (uint64_t)kPhiloxMulB * c.z;
    c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb, (uint32_t)(pa >> 32) ^ c.w ^ k1,
                   (uint32_t)pa);
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  return c;
}

// Block b of stream `sid` under `seed`: counter (b mod 2^32, b div 2^32, sid, 0).
__device__ __forceinline__ uint4 philox_block(uint64_t seed, uint32_t sid, uint64_t b) {
  return philox4x32_10(make_uint4((uint32_t)b, (uint32_t)(b >> 32), sid, 0u), (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// Occupancy of bond w of the stream: word w below the threshold floor(p 2^32).
struct PhiloxOcc {
  uint64_t seed;
  uint32_t sid;
  uint64_t threshold;  // 2^32: every bond occupied
};

__device__ __forceinline__ bool philox_occupied(const PhiloxOcc& r, uint64_t w) {
  const uint4 v = philox_block(r.seed, r.sid, w >> 2);
  const uint32_t j = (uint32_t)(w & 3);  // selects, not a lane-private array
  const uint32_t u = j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
  return (uint64_t)u < r.threshold;
}

// Occupancy bytes (byte j = bond w0 + j) of the four bonds starting at w0.
__device__ __forceinline__ uint32_t philox_occ4(const PhiloxOcc& r, uint64_t w0) {
  const uint4 a = philox_block(r.seed, r.sid, w0 >> 2);
  // bit k: word k of the block pair (w0 >> 2, (w0 >> 2) + 1) is occupied
  uint32_t bits = (uint32_t)((uint64_t)a.x < r.threshold) | (uint32_t)((uint64_t)a.y < r.threshold) << 1 |
                  (uint32_t)((uint64_t)a.z < r.threshold) << 2 | (uint32_t)((uint64_t)a.w < r.threshold) << 3;
  const uint32_t s = (uint32_t)(w0 & 3);
  if (s != 0) {  // the four bonds straddle two blocks
    const uint4 b = philox_block(r.seed, r.sid, (w0 >> 2) + 1);
    bits |= (uint32_t)((uint64_t)b.x < r.threshold) << 4 | (uint32_t)((uint64_t)b.y < r.threshold) << 5 |
            (uint32_t)((uint64_t)b.z < r.threshold) << 6;
  }
  // the four bits from bit s, spread to the low bit of each byte
  return (((bits >> s) & 0xFu) * 0x00204081u) & 0x01010101u;
}

}  // namespace ccl
