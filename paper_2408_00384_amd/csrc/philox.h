// Device Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), written for gfx950.
//
// Each of the ten rounds multiplies counter words 0 and 2 by two fixed odd
// 64-bit constants, keeps both 64-bit halves of each product, mixes the high
// halves with the other two counter words and the key, and then the key is
// advanced by two Weyl increments (golden-ratio and sqrt(3) fractions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cliff {

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMulB = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t loA = kMulA * c[0], hiA = __umul64hi(kMulA, c[0]);
    const uint64_t loB = kMulB * c[2], hiB = __umul64hi(kMulB, c[2]);
    const uint64_t n0 = hiB ^ c[1] ^ k0;
    const uint64_t n2 = hiA ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = loB;
    c[2] = n2;
    c[3] = loA;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
}

// Outcome bit of a random measurement: key (seed, 0), counter (m, shot, circuit, 0).
__device__ __forceinline__ uint32_t outcome_bit(uint64_t seed, uint64_t circuit, uint64_t shot,
                                                uint64_t m) {
  uint64_t c[4] = {m, shot, circuit, 0};
  philox4x64_10(c, seed, 0);
  return uint32_t(c[0] & 1u);
}

}  // namespace cliff
