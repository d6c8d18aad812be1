// Device generator of the Gaussian test matrices (Alg. 1's first step).
//
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key;
// each of the 10 rounds multiplies counter words 0 and 2 by 0xD2511F53 and
// 0xCD9E8D57 and mixes the high halves of the products with the other two
// words and the round key; the key is bumped by the Weyl constants
// (0x9E3779B9, 0xBB67AE85) before every round but the first.
// The Box-Muller transform (Box and Muller, 1958) turns the two 53-bit
// uniforms of one output into two independent N(0, 1) values.
//
// Matrix recipe: entry (i, j) of test matrix `id` under `seed` comes from
// the counter (j / 2, i, id, 0) with the key (low, high 32 bits of seed);
// u1 = ((x1:x0 >> 11) + 1) 2^-53 in (0, 1], u2 = (x3:x2 >> 11) 2^-53 in
// [0, 1), rho = sqrt(-2 ln u1), and the entry is rho cos(2 pi u2) for even j,
// rho sin(2 pi u2) for odd j.  Ids used by the library: 0 Omega_L (n x k),
// 1 Omega_R (m x k), 16 + ... completion columns of the orthonormalisation.
#pragma once

#include "cnmf_internal.hpp"

namespace cnmf {

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// The N(0, 1) pair of entries (row, 2 pair) and (row, 2 pair + 1).
__device__ __forceinline__ void gauss_pair(uint64_t seed, uint32_t id, uint32_t row, uint32_t pair, double& z0,
                                           double& z1) {
  uint32_t c0 = pair, c1 = row, c2 = id, c3 = 0;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((((uint64_t)c1) << 32) | c0) >> 11;
  const uint64_t b = ((((uint64_t)c3) << 32) | c2) >> 11;
  const double u1 = (double)(a + 1) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double rho = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586 * u2;
  z0 = rho * cos(th);
  z1 = rho * sin(th);
}

// One entry (row, col) of test matrix `id`.
__device__ __forceinline__ double gauss_entry(uint64_t seed, uint32_t id, uint32_t row, uint32_t col) {
  double z0, z1;
  gauss_pair(seed, id, row, col >> 1, z0, z1);
  return (col & 1) ? z1 : z0;
}

}  // namespace cnmf
