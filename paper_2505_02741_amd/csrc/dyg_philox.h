// Philox-4x32-10 counter-based generator for the walk kernels, written from
// its published definition (Salmon, Moraes, Dror, Shaw, "Parallel Random
// Numbers: As Easy as 1, 2, 3", SC'11, Sec. 4): ten rounds, each multiplying
// counter words 0 and 2 by two fixed odd constants, swapping the halves of the
// products into the other words with the round key XORed in, and advancing
// the two key words by Weyl increments between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dyg {

struct Philox4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p = uint64_t(0xD2511F53u) * c0;  // multiplier of word 0
    const uint64_t r = uint64_t(0xCD9E8D57u) * c2;  // multiplier of word 2
    const uint32_t n0 = uint32_t(r >> 32) ^ c1 ^ k0;
    const uint32_t n1 = uint32_t(r);
    const uint32_t n2 = uint32_t(p >> 32) ^ c3 ^ k1;
    const uint32_t n3 = uint32_t(p);
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;  // golden-ratio Weyl increment
    k1 += 0xBB67AE85u;  // sqrt(3)-1 Weyl increment
  }
  return Philox4{c0, c1, c2, c3};
}

}  // namespace dyg
