// Grouped backward pass of QFactor-Sample (Sec. 3; Fig. env_calc_tensor; Fig. pre-comp).
//
// The right-to-left update visits the gates one at a time: gate k's environment
//   Gamma_k[q][p] = sum_j sum_r a_k,j(q, r) conj(B_k,j(p, r))
// pairs the backward state a_k (every later gate already updated) with the forward state
// B_k (the gates before k, as they were before the sweep), and u_k <- polar(Gamma_k) must be
// known before a_{k-1} = u_k^dag a_k exists. A pass per gate therefore reads and writes the
// whole backward state once per gate.
//
// Here consecutive gates whose qubits fit in four slots form a group k_lo .. k_hi and share
// one pass. The pass reduces the 16 x 16 second-moment matrix
//   G[z][y] = sum_j sum_r a_{k_hi},j(z, r) conj(B_{k_lo},j(y, r))
// (z, y: the values of the four slots; r: every other amplitude bit). Every environment of
// the group follows from G exactly: inside the group the backward state is
// a_k = V_k a_{k_hi} with V_k the daggers of the group's already-updated gates above k, and
// the forward state is B_k = W_k B_{k_lo} with W_k the group's pre-sweep gates below k, so
//   H_k = V_k G W_k^dag,   Gamma_k[q][p] = sum_s H_k[(q, s)][(p, s)],
//   H_{k-1} = u_k^dag H_k u_{k-1}   (u_k updated, u_{k-1} as before the sweep),
// the partial trace running over the two slots outside gate k. The state thus makes one
// round trip per group instead of one per gate, and the forward pass stores one B entry
// per group. G is a (16 x K)(K x 16)^H product with K = M 2^(n-4) per start: it runs on the
// matrix cores (16x16x4 MFMA; FP32 products for complex64 states, FP64 for complex128), over
// tiles of the state staged in LDS. The 16 x 16 algebra and the polar updates run in FP64 in
// one work-group per start.
//
// Tiles: a tile is a set of nT bits of the chunk-local element index (see the chunked layout
// in qfs_internal.h) that contains the packet bits, the qubits of the gates applied in the
// pass and the four slots, filled with the lowest remaining bits so that every tile read is
// a run of whole 128-byte lines. A work-group loads a tile of the state and the same tile of
// the B entry into LDS, applies the previous group's updated gates (u^dag, in order) in LDS,
// writes the state back, and feeds the MFMA from LDS.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

// complex64 forward products: 1 on the matrix cores (4x4x1 MFMA), 0 on the vector ALU (the
// two measured within 7 % of each other on MI355X, the matrix cores ahead)
#ifndef QFS_FWD_MFMA
#define QFS_FWD_MFMA 1
#endif

#include "polar2.h"
#include "polar4.h"
#include "qfs_internal.h"
#include "stream_common.h"

namespace qfs {

namespace {

constexpr int kGBlock = 512;
constexpr int kGWaves = kGBlock / 64;
constexpr int kMaxBits = 28;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core product per precision: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator entry v of lane l is D[row(l, v)][l % 16].
template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct Mfma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

template <typename R>
struct GroupArgs {
  const cx<R> *a_in;     // backward state (or U psi), nullptr: none
  int64_t a_in_stride;
  cx<R> *a_out;          // updated state, nullptr: not stored
  int64_t a_out_stride;
  const cx<R> *b;        // forward state B_{k_lo} (or psi in the distance mode)
  int64_t b_stride;
  const c128 *vop;       // [S][256]: the previous group's operator (16 x 16 over its four
                         // slots, the u^dag of its gates in order), nullptr: none
  c128 *partials;        // [S][pstride][256]: second-moment block partials
  double *dpartials;     // [S][pstride]: distance block partials
  const int32_t *slot_to_start;
  int32_t pstride;       // blocks per start in either partials (>= gridDim.x)
  int32_t n, logC;
  int32_t nT;            // tile bits of the chunk-local index (packet bits included)
  int32_t nX;            // chunk-local bits outside the tile
  int32_t nch;
  int32_t lowP;          // packet bits of the tile that sit at their own position
  int32_t tpos[kMaxBits];  // chunk-local position of tile bit i (ascending)
  int32_t xpos[kMaxBits];  // chunk-local positions outside the tile (ascending)
  int32_t apos[4];         // tile packet-bit positions of the operator's four slots
  int32_t cpos[kMaxBits];  // the other tile packet bits (ascending): the operator's columns
  int32_t env;             // reduce the second-moment matrix
  int32_t zpos[4];         // tile packet-bit positions of the four slots of the reduction
  int32_t nK;              // packet bits of the reduction index
  int32_t kpos[kMaxBits];  // their tile packet-bit positions (ascending)
};

__device__ __forceinline__ uint32_t spread_bits(uint32_t x, const int32_t *pos, int nb) {
  uint32_t r = 0;
  for (int i = 0; i < nb; ++i) r |= ((x >> i) & 1u) << pos[i];
  return r;
}

__device__ __forceinline__ int lds_slot16(uint32_t pk) { return (int)(pk + (pk >> 4)); }

template <typename R>
__device__ __forceinline__ Pk<R> lds_pk(const float4 *lds, uint32_t pk) {
  const float4 x = lds[lds_slot16(pk)];
  return *reinterpret_cast<const Pk<R> *>(&x);
}

// One complex element (sample e of packet pk) of a staged tile.
__device__ __forceinline__ c64 lds_elem(const float4 *lds, uint32_t pk, int e, float) {
  const float2 x = reinterpret_cast<const float2 *>(lds)[2 * lds_slot16(pk) + e];
  return cmake(x.x, x.y);
}
__device__ __forceinline__ c128 lds_elem(const float4 *lds, uint32_t pk, int, double) {
  const double2 x = reinterpret_cast<const double2 *>(lds)[lds_slot16(pk)];
  return cmake(x.x, x.y);
}
__device__ __forceinline__ void lds_elem_put(float4 *lds, uint32_t pk, int e, c64 v) {
  reinterpret_cast<float2 *>(lds)[2 * lds_slot16(pk) + e] = make_float2(v.re, v.im);
}
__device__ __forceinline__ void lds_elem_put(float4 *lds, uint32_t pk, int, c128 v) {
  reinterpret_cast<double2 *>(lds)[lds_slot16(pk)] = make_double2(v.re, v.im);
}

// Packets per thread and set of one tile (tiles of at most 2048 packets).
constexpr int kMaxPkt = 2048 / kGBlock;

// DIST selects the distance pass (the last group's operator applied to the state, then
// sum |a - b|^2) instead of the environment pass; each has its own kernel, so neither
// carries the other's registers.
template <typename R, bool DIST>
__global__ __launch_bounds__(kGBlock) void k_bwd_group(GroupArgs<R> A) {
  constexpr int V = Pk<R>::V, LOGV = Pk<R>::LOGV;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc_t;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int nP = A.nT - LOGV;
  const uint32_t npk = 1u << nP;
  const uint32_t nslot = npk + (npk >> 4);
  float4 *la = reinterpret_cast<float4 *>(lds_raw);
  float4 *lb = la + nslot;

  const int s = A.slot_to_start[blockIdx.y];
  const int P = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const cx<R> *a_in = A.a_in ? A.a_in + A.a_in_stride * s : nullptr;
  cx<R> *a_out = A.a_out ? A.a_out + A.a_out_stride * s : nullptr;
  const cx<R> *bsrc = A.b + A.b_stride * s;
  const int n = A.n, logC = A.logC, nX = A.nX;

  // chunk-local element offset of packet tid + 256 u of a tile: the bits are disjoint, so
  // the offset of the thread's bits and of u's bits are ORed
  const uint32_t lowmask = (1u << A.lowP) - 1u;
  const int nhi = nP - A.lowP;
  const int32_t *hipos = A.tpos + LOGV + A.lowP;
  auto elem_off = [&](uint32_t pk) __attribute__((always_inline)) -> uint32_t {
    return ((pk & lowmask) << LOGV) | spread_bits(pk >> A.lowP, hipos, nhi);
  };
  uint32_t eo[kMaxPkt];
  const uint32_t eo_t = elem_off((uint32_t)tid & (npk - 1u));
#pragma unroll
  for (int u = 0; u < kMaxPkt; ++u) eo[u] = eo_t | elem_off(((uint32_t)u * kGBlock) & (npk - 1u));

  // the previous group's operator as the A operand of the apply: V[l % 16][4 t + l / 16],
  // as Re V, Re V + Im V and Im V - Re V for the three-product complex multiply
  const bool apply = A.vop != nullptr;
  R vre[4], vsum[4], vdif[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) vre[t] = vsum[t] = vdif[t] = R(0);
  uint32_t rd_off[4], wr_off[4];
  const int ncb = nP - 4;
  const uint32_t ncols = (1u << ncb) << LOGV;
  const uint32_t nblk = ncols >= 16 ? ncols >> 4 : 1u;
  if (apply) {
    const c128 *vs = A.vop + (int64_t)s * 256;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const c128 x = vs[(lane & 15) * 16 + 4 * t + (lane >> 4)];
      vre[t] = (R)x.re;
      vsum[t] = (R)x.re + (R)x.im;
      vdif[t] = (R)x.im - (R)x.re;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = 4 * t + (lane >> 4), rw = MF::row(lane, t);
      rd_off[t] = wr_off[t] = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        rd_off[t] |= (uint32_t)((rr >> i) & 1) << A.apos[i];
        wr_off[t] |= (uint32_t)((rw >> i) & 1) << A.apos[i];
      }
    }
  }

  // reduction lanes: slot index z = lane % 16 (rows of A, columns of B), K quad lane kk
  const int zl = lane & 15, kk = lane >> 4;
  uint32_t zoff = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) zoff |= (uint32_t)((zl >> i) & 1) << A.zpos[i];
  const int nK = A.nK;
  uint32_t kkoff = 0;
  if (nK >= 1) kkoff |= (uint32_t)(kk & 1) << A.kpos[0];
  if (nK >= 2) kkoff |= (uint32_t)((kk >> 1) & 1) << A.kpos[1];
  const bool kk_ok = kk < (1 << min(nK, 2));
  const uint32_t nkq = nK >= 2 ? 1u << (nK - 2) : 1u;
  double gre[4] = {0.0, 0.0, 0.0, 0.0}, gim[4] = {0.0, 0.0, 0.0, 0.0};
  double dacc = 0.0;

  const uint32_t tiles = (uint32_t)A.nch << nX;
  auto tile_base = [&](uint32_t t) __attribute__((always_inline)) -> int64_t {
    const uint32_t q = t >> nX, e = t & ((1u << nX) - 1u);
    return ((int64_t)q << (n + logC)) + spread_bits(e, A.xpos, nX);
  };
  // the next tile's packets are loaded into registers while the current tile is worked on
  // (packets beyond a small tile re-read packet tid: every load is unconditional, so the
  // registers are never partly written)
  const int npt = npk >= kGBlock ? (int)(npk / kGBlock) : 1;
#pragma unroll
  for (int u = 0; u < kMaxPkt; ++u)
    if (u >= npt || (uint32_t)(tid + u * kGBlock) >= npk) eo[u] = eo_t;
  const cx<R> *a_rd = a_in ? a_in : bsrc;
  // (native vectors: HIP's float4 struct is copied through memcpy, which keeps an array
  // of it out of registers)
  f32x4 ra[kMaxPkt], rb[kMaxPkt];
  auto fetch = [&](uint32_t t) __attribute__((always_inline)) {
    const int64_t base = tile_base(t);
#pragma unroll
    for (int u = 0; u < kMaxPkt; ++u) {
      ra[u] = *reinterpret_cast<const f32x4 *>(a_rd + base + eo[u]);
      rb[u] = *reinterpret_cast<const f32x4 *>(bsrc + base + eo[u]);
    }
  };
  uint32_t tau = blockIdx.x;
  if (tau < tiles) fetch(tau);
  for (; tau < tiles; tau += P) {
    const int64_t base = tile_base(tau);
#pragma unroll
    for (int u = 0; u < kMaxPkt; ++u) {
      const uint32_t pk = tid + u * kGBlock;
      if (pk < npk) {
        if (a_in) reinterpret_cast<f32x4 *>(la)[lds_slot16(pk)] = ra[u];
        reinterpret_cast<f32x4 *>(lb)[lds_slot16(pk)] = rb[u];
      }
    }
    lds_barrier();
    if (tau + P < tiles) fetch(tau + P);
    if (apply) {
      // a <- V a on the operator's slots: (16 x 16) x (16 x 16-column block) products on the
      // matrix cores, each wave on its own column blocks, results written back in place.
      // Three real products per complex one: T1 = Re V (Re x + Im x), T2 = (Re V + Im V) Im x,
      // T3 = (Im V - Re V) Re x; Re(V x) = T1 - T2, Im(V x) = T1 + T3.
      for (uint32_t blk = wv; blk < nblk; blk += kGWaves) {
        const uint32_t j = blk * 16 + (lane & 15);
        const bool ok = j < ncols;
        const int e = (int)(j & (V - 1));
        const uint32_t cofs = spread_bits(j >> LOGV, A.cpos, ncb);
        acc_t t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          cx<R> x = cmake<R>(0, 0);
          if (ok) x = lds_elem(la, rd_off[t] | cofs, e, R(0));
          t1 = MF::mma(vre[t], x.re + x.im, t1);
          t2 = MF::mma(vsum[t], x.im, t2);
          t3 = MF::mma(vdif[t], x.re, t3);
        }
        if (ok) {
#pragma unroll
          for (int v = 0; v < 4; ++v) lds_elem_put(la, wr_off[v] | cofs, e, cmake<R>(t1[v] - t2[v], t1[v] + t3[v]));
        }
      }
      lds_barrier();
    }
    if (a_out) {
#pragma unroll
      for (int u = 0; u < kMaxPkt; ++u) {
        const uint32_t pk = tid + u * kGBlock;
        if (pk < npk) *reinterpret_cast<float4 *>(a_out + base + eo[u]) = la[lds_slot16(pk)];
      }
    }
    if (!DIST && A.env) {
      // G += a b^H by three real products: T1 = (Re a + Im a)(Re b + Im b)^T,
      // T2 = Re a Im b^T, T3 = Im a Re b^T; Re G = T1 - T2 - T3, Im G = T3 - T2
      acc_t t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
      for (uint32_t j = wv; j < nkq; j += kGWaves) {
        const uint32_t pk = zoff | kkoff | (nK > 2 ? spread_bits(j, A.kpos + 2, nK - 2) : 0u);
        Pk<R> av, bv;
        if (kk_ok) {
          av = lds_pk<R>(la, pk);
          bv = lds_pk<R>(lb, pk);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) av.v[v] = bv.v[v] = cmake<R>(0, 0);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
          t1 = MF::mma(av.v[v].re + av.v[v].im, bv.v[v].re + bv.v[v].im, t1);
          t2 = MF::mma(av.v[v].re, bv.v[v].im, t2);
          t3 = MF::mma(av.v[v].im, bv.v[v].re, t3);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        gre[v] += ((double)t1[v] - (double)t2[v]) - (double)t3[v];
        gim[v] += (double)t3[v] - (double)t2[v];
      }
    }
    if (DIST) {
#pragma unroll
      for (int u = 0; u < kMaxPkt; ++u) {
        const uint32_t pk = tid + u * kGBlock;
        if (pk < npk) {
          const Pk<R> x = lds_pk<R>(la, pk), y = lds_pk<R>(lb, pk);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const R dr = x.v[v].re - y.v[v].re, di = x.v[v].im - y.v[v].im;
            dacc += (double)dr * (double)dr + (double)di * (double)di;
          }
        }
      }
    }
    lds_barrier();
  }

  if (!DIST && A.env) {
    // wave matrices -> block partial, summed over the waves in order in FP64
    double2 *red = reinterpret_cast<double2 *>(lds_raw);
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv * 256 + MF::row(lane, v) * 16 + zl] = make_double2(gre[v], gim[v]);
    __syncthreads();
    if (tid < 256) {
      double2 acc = red[tid];
#pragma unroll
      for (int w = 1; w < kGWaves; ++w) {
        acc.x += red[w * 256 + tid].x;
        acc.y += red[w * 256 + tid].y;
      }
      A.partials[((int64_t)s * A.pstride + blockIdx.x) * 256 + tid] = cmake(acc.x, acc.y);
    }
  }
  if (DIST) {
    __shared__ double dred[kGWaves];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dacc += __shfl_xor(dacc, o);
    if (lane == 0) dred[wv] = dacc;
    __syncthreads();
    if (tid == 0) {
      double sum = dred[0];
      for (int w = 1; w < kGWaves; ++w) sum += dred[w];
      A.dpartials[(int64_t)s * A.pstride + blockIdx.x] = sum;
    }
  }
}

struct GroupFin {
  int32_t k_hi, k_lo, nvar;
  int32_t sa[kGroupMaxGates], sb[kGroupMaxGates];  // slots of gate k_lo + i's qubits
  int32_t kind[kGroupMaxGates];
};

// Per start: fixed-order FP64 sum of the block partials of G, then the group's gates from
// the top down: Gamma_k by partial trace of H_k, u_k <- polar((1 - beta) Gamma_k + beta u_k)
// (one wave; one-qubit slots by the closed-form 2x2 update), H_{k-1} = u_k^dag H_k u_{k-1}.
// Also the group's operator Vop = u_{k_lo}^dag ... u_{k_hi}^dag over its four slots (the
// updated gates), which the next pass applies to the backward state.
__global__ __launch_bounds__(256) void k_group_finalize(const c128 *partials, int P, int pstride,
                                                        const int32_t *slot_to_start, GroupFin F,
                                                        double beta, c128 *g64, c64 *g32,
                                                        int32_t gstride, c128 *vstore, c128 *vop) {
  __shared__ c128 H[256], Vm[256];
  __shared__ c128 ug[kGroupMaxGates][16];  // the group's gates (pre-sweep, then updated)
  __shared__ c128 vw[kGroupMaxGates][16];  // their Jacobi warm starts
  __shared__ c128 gam[16];
  __shared__ c128 pg[16], pv[16];
  __shared__ double psig[4];
  const int s = slot_to_start[blockIdx.x];
  const int t = threadIdx.x;
  const int z = t >> 4, y = t & 15;
  const int ngate = F.k_hi - F.k_lo + 1;
  c128 *gs = g64 + (int64_t)s * gstride;
  if (t < 16 * ngate) {
    ug[t >> 4][t & 15] = gs[(F.k_lo + (t >> 4)) * 16 + (t & 15)];
    if (vstore) vw[t >> 4][t & 15] = vstore[(int64_t)s * gstride + (F.k_lo + (t >> 4)) * 16 + (t & 15)];
  }
  if (F.nvar > 0) {
    // fixed-order sum of the block partials: eight interleaved accumulators, each batch of
    // eight loads in flight together
    const c128 *src = partials + (int64_t)s * pstride * 256 + t;
    c128 acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = cmake(0.0, 0.0);
    int p = 0;
    for (; p + 7 < P; p += 8) {
      c128 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(p + u) * 256];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = acc[u] + v[u];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u)
      if (p + u < P) acc[u] = acc[u] + src[(int64_t)(p + u) * 256];
    H[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  Vm[t] = cmake(z == y ? 1.0 : 0.0, 0.0);
  // X <- X op(u) with u on slots (a, b) of the column index; op(u) = u^dag or u
  auto right = [&](c128 *X, const c128 *u, int a, int b, bool dag) {
    const int ly = 2 * ((y >> a) & 1) + ((y >> b) & 1);
    const int yb = y & ~((1 << a) | (1 << b));
    c128 v = cmake(0.0, 0.0);
#pragma unroll
    for (int p2 = 0; p2 < 4; ++p2) {
      const int yy = yb | ((p2 >> 1) << a) | ((p2 & 1) << b);
      const c128 m = dag ? cconj(u[ly * 4 + p2]) : u[p2 * 4 + ly];
      cfma(v, X[z * 16 + yy], m);
    }
    __syncthreads();
    X[t] = v;
    __syncthreads();
  };
  // X <- u^dag X (and Y <- u^dag Y when given) with u on slots (a, b) of the row index
  auto left_dag = [&](c128 *X, c128 *Y, const c128 *u, int a, int b) {
    const int lz = 2 * ((z >> a) & 1) + ((z >> b) & 1);
    const int zb = z & ~((1 << a) | (1 << b));
    c128 v = cmake(0.0, 0.0), w = cmake(0.0, 0.0);
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) {
      const int zz = zb | ((q2 >> 1) << a) | ((q2 & 1) << b);
      const c128 m = cconj(u[q2 * 4 + lz]);
      cfma(v, m, X[zz * 16 + y]);
      if (Y) cfma(w, m, Y[zz * 16 + y]);
    }
    __syncthreads();
    X[t] = v;
    if (Y) Y[t] = w;
    __syncthreads();
  };
  __syncthreads();
  // H_{k_hi} = G W^dag, W = u_{k_hi - 1} ... u_{k_lo} (pre-sweep gates)
  if (F.nvar > 0)
    for (int k = F.k_lo; k < F.k_hi; ++k) right(H, ug[k - F.k_lo], F.sa[k - F.k_lo], F.sb[k - F.k_lo], true);
  // the variable gate lowest in the group: H is not needed below it
  int k_last = F.k_lo;
  while (k_last < F.k_hi && F.kind[k_last - F.k_lo] == QFS_GATE_FIXED) ++k_last;
  for (int k = F.k_hi; k >= F.k_lo; --k) {
    const int i = k - F.k_lo;
    const int a = F.sa[i], b = F.sb[i];
    if (F.kind[i] != QFS_GATE_FIXED) {
      if (t < 16) {
        // Gamma[q][p] = sum over the two other slots o0 < o1 of H[(q, o)][(p, o)]
        const int om = 15 & ~((1 << a) | (1 << b));
        const int o0 = __ffs(om) - 1, o1 = __ffs(om & (om - 1)) - 1;
        const int qq = t >> 2, pp = t & 3;
        const int zq = ((qq >> 1) << a) | ((qq & 1) << b), zp = ((pp >> 1) << a) | ((pp & 1) << b);
        c128 g = cmake(0.0, 0.0);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int zo = ((s2 >> 1) << o0) | ((s2 & 1) << o1);
          g = g + H[(zq | zo) * 16 + (zp | zo)];
        }
        gam[t] = g;
      }
      __syncthreads();
      if (t < 64) {
        if (F.kind[i] == QFS_GATE_1Q) {
          if (t == 0) polar2_update<float>(gam, beta, ug[i], nullptr);
        } else {
          polar4_wave(gam, beta, gs + k * 16, ug[i], nullptr, pg, pv, psig,
                      vstore ? vstore + (int64_t)s * gstride + k * 16 : nullptr, vw[i]);
        }
      }
      __syncthreads();
      if (t < 16) {
        gs[k * 16 + t] = ug[i][t];
        if (g32) g32[(int64_t)s * gstride + k * 16 + t] = cmake<float>((float)ug[i][t].re, (float)ug[i][t].im);
      }
    }
    const bool more = F.nvar > 0 && k > k_last;
    left_dag(Vm, more ? H : nullptr, ug[i], a, b);
    if (more) right(H, ug[i - 1], F.sa[i - 1], F.sb[i - 1], false);
  }
  vop[(int64_t)s * 256 + t] = Vm[t];
}

// ------------------------------------------------------------------ grouped forward pass
// The forward pass (Fig. pre-comp) with the same gate groups: a work-group holds one chunk
// of samples in LDS (see the chunked layout in qfs_internal.h) and applies the gates one
// group at a time, each thread taking a 16-element item (the values of the group's four slot
// bits, for fixed other bits and sample) into registers, applying every gate of the group
// there (complex64: the 4x4x1 matrix-core product on the lane's own four amplitudes per
// pair of slots; complex128: FMA), and writing it back: one LDS round trip per group instead
// of one per gate. The B list entry before a group, when the backward pass reads it, is
// stored from the registers on the way in.
template <typename R>
struct FwdGroupSeg {
  const cx<R> *src;     // initial states (shared by all starts), chunked
  cx<R> *blist;         // B list (B_{k+1} at list index k) or nullptr
  int64_t bstride;      // per start
  int64_t sN;           // per list entry
  const cx<R> *ref;     // states to compare against after the last gate, or nullptr
  double *partials;     // [S][nch] distance partials
  int32_t nch;
  int32_t kapply;       // gates applied: 0 .. kapply-1 (whole groups)
};

// Plan entry of a group (forward order): k_lo, k_hi, the chunk-local positions of its four
// slots (qubits first, then fillers), store flag (the entry B_{k_lo} is read); per gate k:
// the slots of its two qubits at gslot[kFwdGS k], gslot[kFwdGS k + 1], and how the gate is
// applied at gslot[kFwdGS k + 2] (kFwdDense, kFwd1Q, kFwdCnotA, kFwdCnotB).
constexpr int kFwdPlan = 8;

// Gate on item slots (SA, SB) applied to the four amplitudes whose other two slots take the
// value C; every index is a compile-time constant, so the item stays in registers.
template <int SA, int SB, int C, typename R, bool MF>
__device__ __forceinline__ void item_quad(cx<R> (&x)[16], const cx<R> (&u)[16], const Gate4 &G4) {
  constexpr int o0 = (0 != SA && 0 != SB) ? 0 : (1 != SA && 1 != SB) ? 1 : 2;
  constexpr int o1 = (3 != SA && 3 != SB) ? 3 : (2 != SA && 2 != SB && 2 != o0) ? 2 : 1;
  constexpr int cb = ((C >> 1) << o0) | ((C & 1) << o1);
  constexpr int i0 = cb, i1 = cb | (1 << SB), i2 = cb | (1 << SA), i3 = cb | (1 << SA) | (1 << SB);
  if constexpr (std::is_same<R, float>::value && MF) {
    const c64 xi[4] = {x[i0], x[i1], x[i2], x[i3]};
    c64 yo[4];
    gate4_apply(G4, xi, yo);
    x[i0] = yo[0];
    x[i1] = yo[1];
    x[i2] = yo[2];
    x[i3] = yo[3];
  } else {
    const cx<R> xi[4] = {x[i0], x[i1], x[i2], x[i3]};
    cx<R> yo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cx<R> acc = cmake<R>(0, 0);
#pragma unroll
      for (int p = 0; p < 4; ++p) cfma(acc, u[q * 4 + p], xi[p]);
      yo[q] = acc;
    }
    x[i0] = yo[0];
    x[i1] = yo[1];
    x[i2] = yo[2];
    x[i3] = yo[3];
  }
}

template <int SA, int SB, typename R, bool MF>
__device__ __forceinline__ void item_gate(cx<R> (&x)[16], const cx<R> (&u)[16], const Gate4 &G4) {
  // (a convergent no-op keeps the compiler from merging the twelve slot cases into one body
  // that selects between array elements, which would move the item out of registers)
  __builtin_amdgcn_wave_barrier();
  item_quad<SA, SB, 0, R, MF>(x, u, G4);
  item_quad<SA, SB, 1, R, MF>(x, u, G4);
  item_quad<SA, SB, 2, R, MF>(x, u, G4);
  item_quad<SA, SB, 3, R, MF>(x, u, G4);
}

template <typename R, bool MF>
__device__ __forceinline__ void item_gate_slots(int sa, int sb, cx<R> (&x)[16], const cx<R> (&u)[16],
                                                const Gate4 &G4) {
  switch (sa * 4 + sb) {
    case 1: item_gate<0, 1, R, MF>(x, u, G4); break;
    case 2: item_gate<0, 2, R, MF>(x, u, G4); break;
    case 3: item_gate<0, 3, R, MF>(x, u, G4); break;
    case 4: item_gate<1, 0, R, MF>(x, u, G4); break;
    case 6: item_gate<1, 2, R, MF>(x, u, G4); break;
    case 7: item_gate<1, 3, R, MF>(x, u, G4); break;
    case 8: item_gate<2, 0, R, MF>(x, u, G4); break;
    case 9: item_gate<2, 1, R, MF>(x, u, G4); break;
    case 11: item_gate<2, 3, R, MF>(x, u, G4); break;
    case 12: item_gate<3, 0, R, MF>(x, u, G4); break;
    case 13: item_gate<3, 1, R, MF>(x, u, G4); break;
    default: item_gate<3, 2, R, MF>(x, u, G4); break;
  }
}

// A one-qubit gate v (x) I_2 on item slot SA (the pair's first qubit), as 2x2 products on
// the vector ALU: v00 = u[0][0], v01 = u[0][2], v10 = u[2][0], v11 = u[2][2] of the 4x4 form.
template <int SA, typename R>
__device__ __forceinline__ void item_1q(cx<R> (&x)[16], cx<R> v00, cx<R> v01, cx<R> v10, cx<R> v11) {
  // (the convergent no-op keeps the slot cases apart, as in item_gate)
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i & (1 << SA)) continue;
    const cx<R> x0 = x[i], x1 = x[i | (1 << SA)];
    cx<R> y0 = cmake<R>(0, 0), y1 = cmake<R>(0, 0);
    cfma(y0, v00, x0);
    cfma(y0, v01, x1);
    cfma(y1, v10, x0);
    cfma(y1, v11, x1);
    x[i] = y0;
    x[i | (1 << SA)] = y1;
  }
  __builtin_amdgcn_wave_barrier();
}

template <typename R>
__device__ __forceinline__ void item_1q_slot(int sa, cx<R> (&x)[16], cx<R> v00, cx<R> v01, cx<R> v10,
                                             cx<R> v11) {
  switch (sa) {
    case 0: item_1q<0, R>(x, v00, v01, v10, v11); break;
    case 1: item_1q<1, R>(x, v00, v01, v10, v11); break;
    case 2: item_1q<2, R>(x, v00, v01, v10, v11); break;
    default: item_1q<3, R>(x, v00, v01, v10, v11); break;
  }
}

// A CNOT (control item slot SC, target slot ST) exchanges the amplitudes it maps onto each
// other: no arithmetic.
template <int SC, int ST, typename R>
__device__ __forceinline__ void item_cnot(cx<R> (&x)[16]) {
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (!(i & (1 << SC)) || (i & (1 << ST))) continue;
    const cx<R> t = x[i];
    x[i] = x[i | (1 << ST)];
    x[i | (1 << ST)] = t;
  }
  __builtin_amdgcn_wave_barrier();
}

template <typename R>
__device__ __forceinline__ void item_cnot_slots(int sc, int st, cx<R> (&x)[16]) {
  switch (sc * 4 + st) {
    case 1: item_cnot<0, 1, R>(x); break;
    case 2: item_cnot<0, 2, R>(x); break;
    case 3: item_cnot<0, 3, R>(x); break;
    case 4: item_cnot<1, 0, R>(x); break;
    case 6: item_cnot<1, 2, R>(x); break;
    case 7: item_cnot<1, 3, R>(x); break;
    case 8: item_cnot<2, 0, R>(x); break;
    case 9: item_cnot<2, 1, R>(x); break;
    case 11: item_cnot<2, 3, R>(x); break;
    case 12: item_cnot<3, 0, R>(x); break;
    case 13: item_cnot<3, 1, R>(x); break;
    default: item_cnot<3, 2, R>(x); break;
  }
}

// FORMS: the plan holds one-qubit or CNOT gate forms (a separate instantiation, so that the
// dense-only kernel keeps its code as small as before).
template <typename R, int FB, bool FORMS>
__global__ __launch_bounds__(FB) void k_forward_groups(FwdGroupSeg<R> seg0, FwdGroupSeg<R> seg1, int nseg,
                                                       int n, int logC, const int32_t *plan_in, int ngroups,
                                                       const int32_t *gslot_in, const cx<R> *gates_in,
                                                       int32_t gstride, const int32_t *slot_to_start, int L,
                                                       int gates_in_lds) {
  constexpr int V = Pk<R>::V;
  const cptr<int32_t> plan = as_const(plan_in);
  const cptr<int32_t> gslot = as_const(gslot_in);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cx<R> *lds = reinterpret_cast<cx<R> *>(lds_raw);
  __shared__ double red[FB / 64];
  const bool second = nseg == 2 && (blockIdx.x & 1);
  const FwdGroupSeg<R> sg = second ? seg1 : seg0;
  const int q = nseg == 2 ? (int)(blockIdx.x >> 1) : (int)blockIdx.x;
  if (q >= sg.nch) return;
  const int s = slot_to_start[blockIdx.y];
  const cx<R> *gates = gates_in + (int64_t)s * gstride;
  const cptr<cx<R>> gates_c = as_const(gates);
  const uint32_t chunk = 1u << (n + logC);  // elements per chunk
  const int64_t cbase = (int64_t)q << (n + logC);
  const cx<R> *src = sg.src + cbase;
  for (uint32_t e = threadIdx.x * V; e < chunk; e += FB * V) st_pk(lds + e, ld_pk(src + e));
  // the start's gates behind the chunk, so reading a gate row never waits on memory
  cx<R> *lgates = lds + chunk;
  if (gates_in_lds)
    for (int e = threadIdx.x; e < 16 * L; e += FB) lgates[e] = gates[e];
  lds_barrier();
  cx<R> *bl = sg.blist ? sg.blist + sg.bstride * s + cbase : nullptr;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nitems = chunk >> 4;
  // complex64: the products on the matrix cores (splitting the waves between the matrix
  // cores and the vector ALU measured slower)
  const bool mf = std::is_same<R, float>::value && QFS_FWD_MFMA;
  for (int gi = 0; gi < ngroups; ++gi) {
    const cptr<int32_t> pg = plan + gi * kFwdPlan;
    const int k_lo = pg[0], k_hi = pg[1];
    const bool store = bl && pg[6] && k_lo - 1 < sg.kapply;
    const bool apply = k_hi < sg.kapply;
    if (!store && !apply) break;  // (groups come in forward order)
    int sp[4], srt[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) srt[i] = sp[i] = pg[2 + i];
    // ascending slot positions for the item index
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (srt[j] > srt[j + 1]) {
          const int t = srt[j];
          srt[j] = srt[j + 1];
          srt[j + 1] = t;
        }
    uint32_t ro[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
      ro[r] = ((uint32_t)(r & 1) << sp[0]) | ((uint32_t)((r >> 1) & 1) << sp[1]) |
              ((uint32_t)((r >> 2) & 1) << sp[2]) | ((uint32_t)((r >> 3) & 1) << sp[3]);
    cx<R> *dst = store ? bl + sg.sN * (k_lo - 1) : nullptr;
    // (wave-uniform trip count: every lane of a wave runs the matrix-core products)
    for (uint32_t ib = threadIdx.x - lane; ib < nitems; ib += FB) {
      const uint32_t it = ib + lane;
      const bool ok = it < nitems;
      const uint32_t base = deposit(it, srt, 4);
      cx<R> x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = ok ? lds[base + ro[r]] : cmake<R>(0, 0);
      if (store && ok) {
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[base + ro[r]] = x[r];
      }
      if (!apply) continue;
      for (int k = k_lo; k <= k_hi; ++k) {
        const int sa = gslot[kFwdGS * k], sb = gslot[kFwdGS * k + 1];
        const int mode = FORMS ? gslot[kFwdGS * k + 2] : kFwdDense;
        if (FORMS && (mode == kFwdCnotA || mode == kFwdCnotB)) {
          const bool ca = mode == kFwdCnotA;
          item_cnot_slots<R>(ca ? sa : sb, ca ? sb : sa, x);
        } else if (FORMS && mode == kFwd1Q) {
          // v = the 2x2 block u[2a][2a'] of the gate's v (x) I_2 form
          const int b0 = k * 16;
          const cx<R> v00 = gates_in_lds ? lgates[b0] : cmake<R>(gates_c[b0].re, gates_c[b0].im);
          const cx<R> v01 = gates_in_lds ? lgates[b0 + 2] : cmake<R>(gates_c[b0 + 2].re, gates_c[b0 + 2].im);
          const cx<R> v10 = gates_in_lds ? lgates[b0 + 8] : cmake<R>(gates_c[b0 + 8].re, gates_c[b0 + 8].im);
          const cx<R> v11 = gates_in_lds ? lgates[b0 + 10] : cmake<R>(gates_c[b0 + 10].re, gates_c[b0 + 10].im);
          item_1q_slot<R>(sa, x, v00, v01, v10, v11);
        } else {
        Gate4 G4;
        cx<R> u[16];
        if (mf) {
          G4 = gates_in_lds ? gate4_row(lgates + k * 16, false) : gate4_row(gates_c + k * 16, false);
          item_gate_slots<R, true>(sa, sb, x, u, G4);
        } else {
          if (gates_in_lds) {
#pragma unroll
            for (int e = 0; e < 16; ++e) u[e] = lgates[k * 16 + e];
          } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) u[e] = cmake<R>(gates_c[k * 16 + e].re, gates_c[k * 16 + e].im);
          }
          item_gate_slots<R, false>(sa, sb, x, u, G4);
        }
        }
      }
      if (ok) {
#pragma unroll
        for (int r = 0; r < 16; ++r) lds[base + ro[r]] = x[r];
      }
    }
    lds_barrier();
  }
  if (sg.ref) {
    const cx<R> *ref = sg.ref + cbase;
    double acc = 0.0;
    for (uint32_t e = threadIdx.x * V; e < chunk; e += FB * V) {
      const Pk<R> a = ld_pk(lds + e), b = ld_pk(ref + e);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const R dr = a.v[v].re - b.v[v].re, di = a.v[v].im - b.v[v].im;
        acc += (double)dr * (double)dr + (double)di * (double)di;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int w = 0; w < FB / 64; ++w) tot += red[w];
      sg.partials[(int64_t)s * sg.nch + q] = tot;
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ host side
std::vector<GateGroup> plan_gate_groups(int L, const int32_t *pairs, const int32_t *kinds) {
  std::vector<GateGroup> out;
  int k = L - 1;
  while (k >= 0) {
    GateGroup gg{};
    gg.k_hi = k;
    gg.nq = 0;
    gg.nvar = 0;
    auto slot_of = [&](int q) {
      for (int i = 0; i < gg.nq; ++i)
        if (gg.q[i] == q) return i;
      return -1;
    };
    while (k >= 0 && gg.k_hi - k < kGroupMaxGates) {
      const int a = pairs[2 * k], b = pairs[2 * k + 1];
      const int need = (slot_of(a) < 0) + (slot_of(b) < 0);
      if (gg.nq + need > 4) break;
      if (slot_of(a) < 0) gg.q[gg.nq++] = a;
      if (slot_of(b) < 0) gg.q[gg.nq++] = b;
      if (!(kinds && kinds[k] == QFS_GATE_FIXED)) ++gg.nvar;
      --k;
    }
    gg.k_lo = k + 1;
    out.push_back(gg);
  }
  return out;
}

bool group_path_supported(const Geometry &g, size_t rbytes) {
  const int logV = rbytes == 4 ? 1 : 0;
  return g.n >= 3 && g.n + g.logC - logV >= 4 && g.n + g.logC <= 24;
}

static int tile_bits_for(size_t rbytes) {
  static const int tb = [] {
    // tuning aid (complex64 value), at most 12: a tile holds at most 2048 packets
    const char *e = std::getenv("QFS_GROUP_TILE_BITS");
    return e ? std::min(12, std::max(5, std::atoi(e))) : 12;
  }();
  return rbytes == 4 ? tb : tb - 1;
}

static int target_blocks() {
  static const int tb = [] {
    const char *e = std::getenv("QFS_GROUP_BLOCKS");  // tuning aid: work-groups per pass
    return e ? std::max(1, std::atoi(e)) : 512;
  }();
  return tb;
}

int group_blocks_per_start(int running_starts) {
  // a power of two of starts, so that the split of the sums changes only when the number
  // of running starts crosses one
  int r = 1;
  while (r < running_starts) r *= 2;
  return std::max(1, target_blocks() / r);
}

int group_partials_stride(const Geometry &g, size_t rbytes) {
  const int logV = rbytes == 4 ? 1 : 0;
  const int nC = g.n + g.logC;
  // every pass's tile has at least min(nC, tile bits) bits, so at most this many tiles
  const int nT = std::max(std::min(nC, tile_bits_for(rbytes)), logV + 4);
  const int64_t tiles = (int64_t)g.nch << std::max(0, nC - nT);
  return (int)std::max<int64_t>(1, std::min<int64_t>({tiles, (int64_t)kGPcap, (int64_t)target_blocks()}));
}

template <typename R>
int launch_group_pass(const Geometry &g, const int32_t *pairs, const GateGroup *prev,
                      const GateGroup *cur, bool dist, const c128 *vop, SBuf<R> a_in, SBuf<R> a_out,
                      SBuf<R> b, const int32_t *slot_to_start, int nslots, int blocks_per_start,
                      c128 *gpartials, int pstride, double *dpartials, int *P_out, hipStream_t s,
                      LaunchEvents ev) {
  if (nslots <= 0) return QFS_OK;
  constexpr int LOGV = Pk<R>::LOGV;
  const int nC = g.n + g.logC;
  GroupArgs<R> A;
  std::memset(&A, 0, sizeof(A));
  A.a_in = a_in.base;
  A.a_in_stride = a_in.stride;
  A.a_out = a_out.base;
  A.a_out_stride = a_out.stride;
  A.b = b.base;
  A.b_stride = b.stride;
  A.vop = prev ? vop : nullptr;
  A.partials = gpartials;
  A.dpartials = dpartials;
  A.slot_to_start = slot_to_start;
  A.pstride = pstride;
  A.n = g.n;
  A.logC = g.logC;
  A.nch = g.nch;
  auto qpos = [&](int qubit) { return g.logC + (g.n - 1 - qubit); };
  // tile: packet bits, the previous group's qubits, the slots' qubits, then the lowest others
  bool in_t[kMaxBits] = {};
  for (int i = 0; i < LOGV; ++i) in_t[i] = true;
  if (prev)
    for (int i = 0; i < prev->nq; ++i) in_t[qpos(prev->q[i])] = true;
  if (cur && !dist)
    for (int i = 0; i < cur->nq; ++i) in_t[qpos(cur->q[i])] = true;
  int nT = 0;
  for (int p = 0; p < nC; ++p) nT += in_t[p];
  const int want = std::max(std::min(nC, tile_bits_for(sizeof(R))), LOGV + 4);
  for (int p = 0; p < nC && nT < want; ++p)
    if (!in_t[p]) {
      in_t[p] = true;
      ++nT;
    }
  if (nT - LOGV < 4 || nT - LOGV > 11) {
    set_error_detail("grouped backward pass: tile geometry out of range");
    return QFS_EUNSUPPORTED;
  }
  int tix[kMaxBits];  // tile bit index of a chunk-local position (-1: outside)
  A.nT = 0;
  A.nX = 0;
  for (int p = 0; p < nC; ++p) {
    if (in_t[p]) {
      tix[p] = A.nT;
      A.tpos[A.nT++] = p;
    } else {
      tix[p] = -1;
      A.xpos[A.nX++] = p;
    }
  }
  A.lowP = 0;
  while (A.lowP < A.nT - LOGV && A.tpos[LOGV + A.lowP] == LOGV + A.lowP) ++A.lowP;
  auto ppos = [&](int qubit) { return tix[qpos(qubit)] - LOGV; };  // tile packet-bit position
  const int nP = A.nT - LOGV;
  // four slots over the given qubits, completed with the lowest other packet bits
  auto slots4 = [&](const GateGroup &gg, int32_t (&pos)[4], bool (&used)[kMaxBits]) {
    for (int i = 0; i < gg.nq; ++i) {
      pos[i] = ppos(gg.q[i]);
      used[pos[i]] = true;
    }
    for (int i = gg.nq, p = 0; i < 4; ++i) {
      while (used[p]) ++p;
      pos[i] = p;
      used[p] = true;
    }
  };
  if (prev) {
    bool used[kMaxBits] = {};
    slots4(*prev, A.apos, used);
    for (int p = 0, c = 0; p < nP; ++p)
      if (!used[p]) A.cpos[c++] = p;
  }
  A.env = (!dist && cur && cur->nvar > 0) ? 1 : 0;
  if (A.env) {
    bool used[kMaxBits] = {};
    slots4(*cur, A.zpos, used);
    A.nK = 0;
    for (int p = 0; p < nP; ++p)
      if (!used[p]) A.kpos[A.nK++] = p;
  }
  const uint32_t npk = 1u << (A.nT - LOGV);
  const size_t lds = std::max<size_t>(2 * (size_t)(npk + (npk >> 4)) * 16, (size_t)kGWaves * 256 * 16);
  static size_t attr[2][2] = {{0, 0}, {0, 0}};
  size_t &ab = attr[sizeof(R) == 4 ? 0 : 1][dist ? 1 : 0];
  const void *fn = dist ? reinterpret_cast<const void *>(k_bwd_group<R, true>)
                        : reinterpret_cast<const void *>(k_bwd_group<R, false>);
  QFS_TRY(ensure_dynamic_lds(fn, lds, &ab));
  const int64_t tiles = (int64_t)g.nch << A.nX;
  const int P = (int)std::min<int64_t>({tiles, (int64_t)std::max(1, pstride),
                                         (int64_t)std::max(1, blocks_per_start)});
  *P_out = P;
  if (dist)
    hipExtLaunchKernelGGL((k_bwd_group<R, true>), dim3(P, nslots), dim3(kGBlock), lds, s, ev.start, ev.stop, 0,
                          A);
  else
    hipExtLaunchKernelGGL((k_bwd_group<R, false>), dim3(P, nslots), dim3(kGBlock), lds, s, ev.start, ev.stop,
                          0, A);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_group_finalize(int P, const c128 *gpartials, int pstride, const int32_t *slot_to_start,
                          int nslots,
                          const GateGroup &cur, const int32_t *pairs, const int32_t *kinds,
                          double beta, c128 *g64, c64 *g32, int32_t gstride, c128 *vstore,
                          c128 *vop, hipStream_t s, LaunchEvents ev) {
  if (nslots <= 0) return QFS_OK;
  GroupFin F;
  std::memset(&F, 0, sizeof(F));
  F.k_hi = cur.k_hi;
  F.k_lo = cur.k_lo;
  F.nvar = cur.nvar;
  auto slot = [&](int q) {
    for (int i = 0; i < cur.nq; ++i)
      if (cur.q[i] == q) return i;
    return -1;
  };
  for (int k = cur.k_lo; k <= cur.k_hi; ++k) {
    F.sa[k - cur.k_lo] = slot(pairs[2 * k]);
    F.sb[k - cur.k_lo] = slot(pairs[2 * k + 1]);
    F.kind[k - cur.k_lo] = kinds ? kinds[k] : QFS_GATE_2Q;
  }
  hipExtLaunchKernelGGL(k_group_finalize, dim3(nslots), dim3(256), 0, s, ev.start, ev.stop, 0, gpartials, P,
                        pstride, slot_to_start, F, beta, g64, g32, gstride, vstore, vop);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}


// ------------------------------------------------------------------ grouped forward, host
std::vector<int32_t> forward_gate_modes(int L, const int32_t *kinds, const c128 *gates_host, int copies) {
  std::vector<int32_t> mode(L, kFwdDense);
  if (!kinds) return mode;
  // exactly a CNOT, control on the pair's first (A) or second (B) qubit: the 4x4 entries
  // (row-major) that are 1, every other entry 0
  static const int onesA[4] = {0, 5, 11, 14}, onesB[4] = {0, 7, 10, 13};
  auto is_perm = [](const c128 *u, const int (&ones)[4]) {
    for (int e = 0; e < 16; ++e) {
      const bool one = e == ones[0] || e == ones[1] || e == ones[2] || e == ones[3];
      if (u[e].re != (one ? 1.0 : 0.0) || u[e].im != 0.0) return false;
    }
    return true;
  };
  for (int k = 0; k < L; ++k) {
    if (kinds[k] == QFS_GATE_1Q) {
      mode[k] = kFwd1Q;
    } else if (kinds[k] == QFS_GATE_FIXED && gates_host && copies > 0) {
      bool a = true, b = true;
      for (int c = 0; c < copies; ++c) {
        const c128 *u = gates_host + ((size_t)c * L + k) * 16;
        a = a && is_perm(u, onesA);
        b = b && is_perm(u, onesB);
      }
      mode[k] = a ? kFwdCnotA : b ? kFwdCnotB : kFwdDense;
    }
  }
  return mode;
}

int build_forward_plan(const Geometry &g, int L, const int32_t *pairs, const std::vector<GateGroup> &groups,
                       const int32_t *bneed_host, const int32_t *mode_host, std::vector<int32_t> &plan,
                       std::vector<int32_t> &gslot) {
  const int nC = g.n + g.logC;
  if (nC < 4) return QFS_EUNSUPPORTED;
  plan.assign(groups.size() * kFwdPlan, 0);
  gslot.assign(kFwdGS * (size_t)L, 0);
  const int ng = (int)groups.size();
  for (int fi = 0; fi < ng; ++fi) {
    const GateGroup &gg = groups[ng - 1 - fi];  // forward order
    int32_t *pe = &plan[fi * kFwdPlan];
    pe[0] = gg.k_lo;
    pe[1] = gg.k_hi;
    bool used[32] = {};
    for (int i = 0; i < gg.nq; ++i) {
      pe[2 + i] = g.logC + (g.n - 1 - gg.q[i]);
      used[pe[2 + i]] = true;
    }
    // fillers: the highest free positions, so the lanes of an item run over the low bits
    for (int i = gg.nq, p = nC - 1; i < 4; ++i) {
      while (used[p]) --p;
      pe[2 + i] = p;
      used[p] = true;
    }
    pe[6] = (gg.k_lo >= 1 && bneed_host && bneed_host[gg.k_lo]) ? 1 : 0;
    auto slot = [&](int q) {
      for (int i = 0; i < gg.nq; ++i)
        if (gg.q[i] == q) return i;
      return -1;
    };
    for (int k = gg.k_lo; k <= gg.k_hi; ++k) {
      gslot[kFwdGS * k] = slot(pairs[2 * k]);
      gslot[kFwdGS * k + 1] = slot(pairs[2 * k + 1]);
      gslot[kFwdGS * k + 2] = mode_host ? mode_host[k] : kFwdDense;
    }
  }
  return QFS_OK;
}

template <typename R>
int launch_forward_groups(const Geometry &g, const Geometry *gv, int L, GateRef gates, const cx<R> *psi,
                          cx<R> *blist, int64_t bstride, const cx<R> *phi_ref, double *c0_partials,
                          const cx<R> *psiv, const cx<R> *phiv, double *val_partials,
                          const int32_t *slot_to_start, int nslots, const int32_t *plan_dev, int ngroups,
                          const int32_t *gslot_dev, bool forms, hipStream_t s) {
  if (nslots <= 0) return QFS_OK;
  FwdGroupSeg<R> a{}, b{};
  a.src = psi;
  a.blist = blist;
  a.bstride = bstride;
  a.sN = (int64_t)g.nch * ((int64_t)g.N << g.logC);
  a.ref = phi_ref;
  a.partials = c0_partials;
  a.nch = g.nch;
  a.kapply = phi_ref ? L : L - 1;
  int nz = 1;
  if (gv) {
    if (gv->logC != g.logC) {
      set_error_detail("grouped forward: training and validation chunk widths differ");
      return QFS_EINVAL;
    }
    b.src = psiv;
    b.ref = phiv;
    b.partials = val_partials;
    b.nch = gv->nch;
    b.kapply = L;
    nz = 2;
  }
  const int gx = std::max(a.nch, gv ? b.nch : 0);
  const size_t chunk_bytes = (size_t(1) << (g.n + g.logC)) * sizeof(cx<R>);
  const size_t gate_bytes = (size_t)16 * L * sizeof(cx<R>);
  const int gates_in_lds = chunk_bytes + gate_bytes <= 160 * 1024 ? 1 : 0;
  const size_t lds = chunk_bytes + (gates_in_lds ? gate_bytes : 0);
  const int64_t items = int64_t(1) << (g.n + g.logC - 4);
  const int threads = items >= 1024 ? 1024 : 512;
  auto go = [&](auto kernel) -> int {
    static size_t attr = 0;
    QFS_TRY(ensure_dynamic_lds(reinterpret_cast<const void *>(kernel), lds, &attr));
    hipLaunchKernelGGL(kernel, dim3(gx * nz, nslots, 1), dim3(threads), lds, s, a, b, nz, g.n, g.logC, plan_dev,
                       ngroups, gslot_dev, static_cast<const cx<R> *>(gates.gR), gates.gstride, slot_to_start, L,
                       gates_in_lds);
    QFS_HIP(hipGetLastError());
    return QFS_OK;
  };
  if (forms) {
    if (threads == 1024) return go(k_forward_groups<R, 1024, true>);
    return go(k_forward_groups<R, 512, true>);
  }
  if (threads == 1024) return go(k_forward_groups<R, 1024, false>);
  return go(k_forward_groups<R, 512, false>);
}

#define QFS_FINST(R)                                                                              \
  template int launch_forward_groups<R>(const Geometry &, const Geometry *, int, GateRef, const cx<R> *, \
                                        cx<R> *, int64_t, const cx<R> *, double *, const cx<R> *,  \
                                        const cx<R> *, double *, const int32_t *, int,            \
                                        const int32_t *, int, const int32_t *, bool, hipStream_t);
QFS_FINST(float)
#undef QFS_FINST

#define QFS_GINST(R)                                                                          \
  template int launch_group_pass<R>(const Geometry &, const int32_t *, const GateGroup *,      \
                                    const GateGroup *, bool, const c128 *, SBuf<R>, SBuf<R>,   \
                                    SBuf<R>, const int32_t *, int, int, c128 *, int, double *, \
                                    int *, hipStream_t, LaunchEvents);
QFS_GINST(float)
QFS_GINST(double)
#undef QFS_GINST

}  // namespace qfs
