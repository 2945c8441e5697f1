// Packet access, bit deposit, constant-address-space views and gate loads shared by
// the streaming sweep kernels (sweep.hip, group.hip).
#pragma once

#include "qfs_internal.h"

namespace qfs {

// Work-group barrier for hand-offs through LDS only: it waits for the wave's own LDS
// operations, not for its global loads and stores (which __syncthreads also drains), so
// prefetches and stores stay in flight across it. The memory clobber keeps the compiler
// from moving memory operations across it.
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

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

// A 4x4 complex64 gate applied by the matrix cores to each lane's own four amplitudes.
// The 16-block 4x4x1 FP32 MFMA forms, in block b (lanes 4b .. 4b+3), D[i][j] += a_i b_j with
// a_i, b_j supplied by lanes 4b + i and 4b + j and D[i][j] returned in lane 4b + j,
// register i. With lane 4b + i supplying u[i][p] and every lane its own x[p], the four
// K-steps p give every lane its own (u x)[i]: the per-thread matrix-vector product of the
// vector ALU at twice its FP32 rate, in the same data layout. All 64 lanes must execute it.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
struct Gate4 {
  float re[4], im[4], nim[4];  // row (lane % 4) of the gate, column p
};

// Row lane % 4 of gate src (row-major 4x4), in the local basis with indices 1 and 2
// exchanged when swapped.
template <typename P>
__device__ __forceinline__ Gate4 gate4_row(P src, bool swapped) {
  constexpr int pm[4] = {0, 2, 1, 3};
  const int r = threadIdx.x & 3;
  const int rr = swapped ? pm[r] : r;
  Gate4 G;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int pp = swapped ? pm[p] : p;
    const float re = (float)src[rr * 4 + pp].re, im = (float)src[rr * 4 + pp].im;
    G.re[p] = re;
    G.im[p] = im;
    G.nim[p] = -im;
  }
  return G;
}

__device__ __forceinline__ void gate4_apply(const Gate4 &G, const c64 (&x)[4], c64 (&y)[4]) {
  f32x4_t dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    dr = __builtin_amdgcn_mfma_f32_4x4x1f32(G.re[p], x[p].re, dr, 0, 0, 0);
    dr = __builtin_amdgcn_mfma_f32_4x4x1f32(G.nim[p], x[p].im, dr, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_4x4x1f32(G.re[p], x[p].im, di, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_4x4x1f32(G.im[p], x[p].re, di, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = cmake(dr[i], di[i]);
}

}  // namespace qfs
