// Packet access, bit deposit, constant-address-space views and gate loads shared by
// the streaming sweep kernels (sweep.hip, group.hip).
#pragma once

#include "qfs_internal.h"

namespace qfs {

template <typename R>
struct Pk;  // 16-byte packet of samples
template <>
struct Pk<float> {
  static constexpr int V = 2;
  static constexpr int LOGV = 1;
  c64 v[2];
};
template <>
struct Pk<double> {
  static constexpr int V = 1;
  static constexpr int LOGV = 0;
  c128 v[1];
};

__device__ __forceinline__ Pk<float> ld_pk(const c64 *p) {
  const float4 x = *reinterpret_cast<const float4 *>(p);
  Pk<float> r;
  r.v[0] = cmake(x.x, x.y);
  r.v[1] = cmake(x.z, x.w);
  return r;
}
__device__ __forceinline__ Pk<double> ld_pk(const c128 *p) {
  const double2 x = *reinterpret_cast<const double2 *>(p);
  Pk<double> r;
  r.v[0] = cmake(x.x, x.y);
  return r;
}
__device__ __forceinline__ void st_pk(c64 *p, const Pk<float> &r) {
  *reinterpret_cast<float4 *>(p) = make_float4(r.v[0].re, r.v[0].im, r.v[1].re, r.v[1].im);
}
__device__ __forceinline__ void st_pk(c128 *p, const Pk<double> &r) {
  *reinterpret_cast<double2 *>(p) = make_double2(r.v[0].re, r.v[0].im);
}

// Insert a zero bit at each of the t ascending positions.
__device__ __forceinline__ uint32_t deposit(uint32_t r, const int *sorted_pos, int t) {
  for (int m = 0; m < t; ++m) {
    const int p = sorted_pos[m];
    const uint32_t low = r & ((1u << p) - 1u);
    r = ((r >> p) << (p + 1)) | low;
  }
  return r;
}

// Read-only kernel inputs through the constant address space: uniform loads from it are
// scalar loads (counted by lgkmcnt), so reading the next gate never waits for the vector
// stores still in flight, however the surrounding code looks to alias analysis.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

template <typename R, typename P>
__device__ __forceinline__ void load_gate(P src, cx<R> (&u)[16], bool dagger) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = dagger ? p * 4 + q : q * 4 + p;
      const cx<R> x = cmake<R>(src[i].re, src[i].im);  // (also from the constant address space)
      u[q * 4 + p] = dagger ? cconj(x) : x;
    }
}

}  // namespace qfs
