// Counter-based generator for the method's own draws: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller
// transform, one complex standard normal per Philox block. Shared by the device code
// of the single-problem and batched paths.
#pragma once

#include "qfs_internal.h"

namespace qfs {

struct Philox4 {
  uint32_t w[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
    const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
    const uint32_t n0 = hiB ^ c1 ^ k0;
    const uint32_t n2 = hiA ^ c3 ^ k1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// Complex normal with E|z|^2 = 1: |z|^2 = -ln(u1) ~ Exp(1), arg z = 2 pi u2; counter
// words (index lo, index hi, role, stream), key = the 64-bit seed.
__device__ __forceinline__ c128 complex_normal(uint64_t seed, uint32_t role, uint32_t stream,
                                               uint64_t idx) {
  const Philox4 x = philox4x32_10((uint32_t)idx, (uint32_t)(idx >> 32), role, stream,
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t m1 = ((((uint64_t)x.w[1]) << 32) | x.w[0]) >> 11;  // 53 bits
  const uint64_t m2 = ((((uint64_t)x.w[3]) << 32) | x.w[2]) >> 11;
  const double u1 = ((double)m1 + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)m2 * 0x1.0p-53;          // [0, 1)
  const double radius = sqrt(-log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  return cmake<double>(radius * cs, radius * sn);
}

}  // namespace qfs
