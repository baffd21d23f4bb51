// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// written from the published description: ten rounds, each multiplying counter
// words 0 and 2 by the round multipliers, XOR-ing the 64-bit products' high
// halves with the other words and the key, the key advancing by the two Weyl
// constants between rounds.  Used on the host (trajectory pre-sampling) and on
// the device (shot draws).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ptsbe {

struct Philox4 {
  uint32_t w[4];
};

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  Philox4 r;
  r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
  return r;
}

// Stream key: (lo32(seed), hi32(seed) XOR tag * 0x9E3779B9); tags: 1 trajectory
// pre-sampling, 2 shot draws, 3 extra draws.
__host__ __device__ inline void philox_key(uint64_t seed, uint32_t tag, uint32_t& k0, uint32_t& k1) {
  k0 = (uint32_t)seed;
  k1 = (uint32_t)(seed >> 32) ^ (uint32_t)(tag * 0x9E3779B9u);
}

// u in [0, 1): top 53 bits of (w1 << 32 | w0).
__host__ __device__ inline double philox_uniform(uint64_t seed, uint32_t tag, uint32_t c0, uint32_t c1,
                                                 uint32_t c2, uint32_t c3) {
  uint32_t k0, k1;
  philox_key(seed, tag, k0, k1);
  Philox4 r = philox4x32_10(c0, c1, c2, c3, k0, k1);
  uint64_t v = ((uint64_t)r.w[1] << 32) | r.w[0];
  return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace ptsbe
