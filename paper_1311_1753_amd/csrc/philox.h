// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011) and the per-event uniform stream of the toy
// generators: uniform number m of event i comes from the block with counter
// (i mod 2^32, i div 2^32, m div 2, 0) under the key (seed low word, seed
// high word), words 0-1 for even m and 2-3 for odd m, as
// u = (floor((w_a 2^32 + w_b) / 2^11) + 1/2) 2^-53 in (0, 1).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hf {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = kPhiloxM0 * c[0], hi0 = __umulhi(kPhiloxM0, c[0]);
    const uint32_t lo1 = kPhiloxM1 * c[2], hi1 = __umulhi(kPhiloxM1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// The uniforms of one event, in order; a block's second pair is kept for the
// next number.
struct EventStream {
  uint32_t i0, i1, k0, k1;
  uint32_t m = 0, w2 = 0, w3 = 0;
  __device__ __forceinline__ double next() {
    uint32_t a, b;
    if ((m & 1u) == 0) {
      uint32_t c[4] = {i0, i1, m >> 1, 0u};
      philox4x32_10(c, k0, k1);
      a = c[0];
      b = c[1];
      w2 = c[2];
      w3 = c[3];
    } else {
      a = w2;
      b = w3;
    }
    ++m;
    const uint64_t bits = (((uint64_t)a << 32) | (uint64_t)b) >> 11;
    return ((double)bits + 0.5) * 0x1.0p-53;
  }
};


}  // namespace hf
