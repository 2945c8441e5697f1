// QFactor-Sample on qudits (Sec. 5: the method carries over unchanged to d-level gates,
// where a sweep costs O(M d^n) against QFactor's O(d^{2n})).
//
// n qudits of dimension d, N = d^n amplitudes, qudit 0 the most significant base-d
// digit; a two-qudit gate on (a, b) is a D x D unitary, D = d^2, row-major u[q][p], local
// index d digit(a) + digit(b). State sets are amplitude-major: element (i, j) (amplitude
// i of sample j) at i * M + j, so the D amplitudes of a gate group are D rows of M
// consecutive samples, read and written as runs whatever qudits the gate acts on.
// Kernels are templated on the state precision R and on d; the environment partials,
// the polar update and the costs are FP64.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "philox.h"
#include "polar4.h"
#include "qfs_internal.h"

namespace qfs {
namespace {

constexpr int kQdBlock = 256;
constexpr int kQdMaxP = 64;  // environment partial blocks per (start, row group)
constexpr int kQdMaxDD = 256;  // entries of the largest gate (d = 4: 16 x 16)
// Jacobi stops when every column pair has |g_p^dagger g_q| <= tol |g_p| |g_q|. The Gram
// entry of D-long columns carries a rounding error of about D eps |g_p| |g_q| (1e-15 for
// D = 9), so the threshold sits above it; the polar factor is then accurate to ~1e-14.
constexpr double kQdJacobiTol = 1e-14;

// Position of a gate group: items are (group r, sample j), j fastest.
struct QdGeom {
  int32_t M;        // samples in the set (row length)
  int64_t groups;   // N / D
  int64_t s_lo;     // d^(lower digit position of the two gate qudits)
  int64_t mid;      // d^(digits strictly between the two positions)
  int64_t sa, sb;   // strides of the gate's first and second qudit
};

template <int d>
__device__ __forceinline__ int64_t qd_base(const QdGeom &g, int64_t r) {
  const int64_t r_lo = r % g.s_lo;
  const int64_t t = r / g.s_lo;
  const int64_t r_mid = t % g.mid, r_hi = t / g.mid;
  // digits: r_hi | 0 (upper gate qudit) | r_mid | 0 (lower gate qudit) | r_lo
  return r_hi * d * g.mid * d * g.s_lo + r_mid * d * g.s_lo + r_lo;
}

QdGeom qd_geom(int d, int n, int M, int qa, int qb) {
  auto pw = [&](int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= d;
    return r;
  };
  const int pa = n - 1 - qa, pb = n - 1 - qb;
  const int lo = std::min(pa, pb), hi = std::max(pa, pb);
  QdGeom g;
  g.M = M;
  g.groups = pw(n) / (d * d);
  g.s_lo = pw(lo);
  g.mid = pw(hi - lo - 1);
  g.sa = pw(pa);
  g.sb = pw(pb);
  return g;
}

// dst = u_k src (dagger: u_k^dagger src) for every active start; the gate (FP64 master)
// goes through LDS in the state precision.
template <typename R, int d>
__global__ __launch_bounds__(kQdBlock) void k_qd_apply(const cx<R> *src, int64_t src_stride, cx<R> *dst,
                                                       int64_t dst_stride, const c128 *gates,
                                                       int32_t gstride, int32_t k, int32_t dagger,
                                                       QdGeom g, const int32_t *slots) {
  constexpr int D = d * d;
  __shared__ cx<R> u[D * D];
  const int s = slots[blockIdx.y];
  const c128 *gk = gates + (int64_t)s * gstride + (int64_t)k * D * D;
  for (int e = threadIdx.x; e < D * D; e += kQdBlock) {
    const int q = e / D, p = e % D;
    const c128 v = dagger ? cconj(gk[p * D + q]) : gk[e];
    u[e] = cmake<R>((R)v.re, (R)v.im);
  }
  __syncthreads();
  const cx<R> *x = src + (int64_t)s * src_stride;
  cx<R> *y = dst + (int64_t)s * dst_stride;
  const int64_t items = g.groups * g.M;
  for (int64_t it = blockIdx.x * (int64_t)kQdBlock + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * kQdBlock) {
    const int64_t j = it % g.M, r = it / g.M;
    const int64_t base = qd_base<d>(g, r);
    int64_t off[D];
    cx<R> in[D];
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
      for (int b = 0; b < d; ++b) {
        off[a * d + b] = (base + a * g.sa + b * g.sb) * g.M + j;
        in[a * d + b] = x[off[a * d + b]];
      }
    // (d > 2: output rows d at a time, so the compiler does not hold the whole gate in
    // registers across the item loop)
    constexpr int UQ = d == 2 ? D : d;
#pragma unroll UQ
    for (int q = 0; q < D; ++q) {
      cx<R> acc = cmake<R>(0, 0);
#pragma unroll
      for (int p = 0; p < D; ++p) cfma(acc, u[q * D + p], in[p]);
      y[off[q]] = acc;
    }
  }
}

// Wave sums of NV values (NV = 16, 32 or 64; FP64) by recursive halving: at the exchange
// with lane ^ MASK each lane keeps C of its 2C values (the upper ones when that lane bit is
// set) and adds its partner's copy; the lane bits left over are summed plainly. Lane l
// returns the wave sum of value l >> (6 - log2 NV).
template <int C, int MASK, int NV>
__device__ __forceinline__ void qhalve(double (&v)[NV], int lane) {
  const bool hi = (lane & MASK) != 0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const double give = hi ? v[i] : v[C + i];
    const double keep = hi ? v[C + i] : v[i];
    v[i] = keep + __shfl_xor(give, MASK);
  }
}
template <int NV>
__device__ __forceinline__ double qwave_sum(double (&v)[NV]) {
  static_assert(NV == 16 || NV == 32 || NV == 64, "16, 32 or 64 values");
  const int lane = threadIdx.x & 63;
  qhalve<NV / 2, 32>(v, lane);
  qhalve<NV / 4, 16>(v, lane);
  qhalve<NV / 8, 8>(v, lane);
  qhalve<NV / 16, 4>(v, lane);
  if constexpr (NV >= 32) qhalve<NV / 32, 2>(v, lane);
  else v[0] += __shfl_xor(v[0], 2);
  if constexpr (NV >= 64) qhalve<1, 1>(v, lane);
  else v[0] += __shfl_xor(v[0], 1);
  return v[0];
}

// Rows of the environment one block accumulates: d (one value of the first gate qudit's
// digit) for d <= 3, two for d = 4, where d rows would hold 128 FP64 accumulators a thread.
template <int d>
constexpr int qd_env_rows() {
  return d <= 3 ? d : 2;
}

// Environment partials: block (row set xg, partial blk, start) accumulates rows
// q = RY xg + y (y < RY) of Gamma[q][p] = sum a(q) conj(b(p)) over its items in FP64 and
// writes them to partials[s][blk][q][p].
template <typename R, int d>
__global__ __launch_bounds__(kQdBlock) void k_qd_env(const cx<R> *a, int64_t a_stride, const cx<R> *b,
                                                     int64_t b_stride, QdGeom g, int32_t P,
                                                     c128 *partials, const int32_t *slots) {
  constexpr int D = d * d;
  constexpr int RY = qd_env_rows<d>();
  constexpr int NX = D / RY;  // row sets
  constexpr int W = kQdBlock / 64;
  __shared__ c128 red[W][RY * D];
  const int s = slots[blockIdx.y];
  const int xg = blockIdx.x % NX, blk = blockIdx.x / NX;
  const cx<R> *as = a + (int64_t)s * a_stride;
  const cx<R> *bs = b + (int64_t)s * b_stride;
  c128 acc[RY][D];
#pragma unroll
  for (int y = 0; y < RY; ++y)
#pragma unroll
    for (int p = 0; p < D; ++p) acc[y][p] = cmake(0.0, 0.0);
  const int64_t items = g.groups * g.M;
  for (int64_t it = blk * (int64_t)kQdBlock + threadIdx.x; it < items; it += (int64_t)P * kQdBlock) {
    const int64_t j = it % g.M, r = it / g.M;
    const int64_t base = qd_base<d>(g, r);
    c128 bv[D], av[RY];
#pragma unroll
    for (int x = 0; x < d; ++x)
#pragma unroll
      for (int y = 0; y < d; ++y) {
        const cx<R> v = bs[(base + x * g.sa + y * g.sb) * g.M + j];
        bv[x * d + y] = cmake((double)v.re, (double)v.im);
      }
#pragma unroll
    for (int y = 0; y < RY; ++y) {
      const int q = xg * RY + y;  // local row: digits q / d (first qudit), q % d (second)
      const cx<R> v = as[(base + (q / d) * g.sa + (q % d) * g.sb) * g.M + j];
      av[y] = cmake((double)v.re, (double)v.im);
    }
#pragma unroll
    for (int y = 0; y < RY; ++y)
#pragma unroll
      for (int p = 0; p < D; ++p) cfma_conj(acc[y][p], av[y], bv[p]);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  {
    // the 2 RY D reals (value 2 (y D + p) + part), padded with zeros to a power of two
    constexpr int NR = 2 * RY * D;
    constexpr int NV = NR <= 16 ? 16 : (NR <= 32 ? 32 : 64);
    static_assert(NR <= 64, "at most 64 reals a lane");
    double v[NV];
#pragma unroll
    for (int y = 0; y < RY; ++y)
#pragma unroll
      for (int p = 0; p < D; ++p) {
        v[2 * (y * D + p)] = acc[y][p].re;
        v[2 * (y * D + p) + 1] = acc[y][p].im;
      }
#pragma unroll
    for (int i = NR; i < NV; ++i) v[i] = 0.0;
    const double ws = qwave_sum<NV>(v);
    constexpr int SH = NV == 16 ? 2 : (NV == 32 ? 1 : 0);
    const int idx = lane >> SH;
    if ((lane & ((1 << SH) - 1)) == 0 && idx < NR) reinterpret_cast<double *>(&red[w][0])[idx] = ws;
  }
  __syncthreads();
  if (threadIdx.x < RY * D) {
    c128 t = red[0][threadIdx.x];
    for (int ww = 1; ww < W; ++ww) t = t + red[ww][threadIdx.x];
    const int y = threadIdx.x / D, p = threadIdx.x % D;
    const int q = xg * RY + y;
    partials[(((int64_t)s * P + blk) * D + q) * D + p] = t;
  }
}

// Per start: the environment Gamma_k as the fixed-order sum of its work-group partials
// (partial i in running sum i mod 8), then u_k <- W V^dagger for the mixed
// environment (1 - beta) Gamma_k + beta u_k = W S V^dagger by one-sided (Hestenes) Jacobi. The working
// matrix G and V are kept by columns in LDS (rows padded to 16 with zeros; a zero ghost
// column when D is odd). Pairs are rotated in round-robin rounds (circle method on the PL
// columns): the pairs of a round are disjoint, and pair i of the round is worked by the
// 16 lanes of row i of the block's waves (lane r holds row r of both columns of G and V),
// which sum the pair's three Gram entries by DPP moves within their row, so each lane
// computes the same rotation and applies it to its own row. Zero rows and ghost columns
// contribute nothing and never rotate. Warm start: Jacobi begins from G V_prev with
// V_prev, the right singular vectors this gate had after its previous update (vst, made
// unitary to rounding by one Newton-Schulz step V (3I - V^dagger V) / 2), so a sweep of
// small changes converges in a few Jacobi sweeps; the new V is stored back.
// u for a (near) singular environment: left vectors in decreasing-sigma order,
// orthonormalised in place in LDS (W column kk in Tm[. * D + kk]) and completed with unit
// vectors (any such completion attains the maximum); one thread.
template <int D, int PL>
__device__ __noinline__ void qd_polar_singular(const c128 (*Gc)[16], const c128 (*Vc)[16], c128 *Tm,
                                               const double *sig, double smax, c128 *u) {
  int ord[D];
#pragma unroll 1
  for (int c = 0; c < D; ++c) ord[c] = c;
#pragma unroll 1
  for (int a = 0; a < D; ++a)
#pragma unroll 1
    for (int b2 = a + 1; b2 < D; ++b2)
      if (sig[ord[b2]] > sig[ord[a]]) {
        const int tmp = ord[a];
        ord[a] = ord[b2];
        ord[b2] = tmp;
      }
#pragma unroll 1
  for (int kk = 0; kk < D; ++kk) {
    const int cc = ord[kk];
    bool ok = sig[cc] > 0.0 && sig[cc] > 1e-13 * smax;
#pragma unroll 1
    for (int rr = 0; rr < D; ++rr) Tm[rr * D + kk] = ok ? cscale(Gc[cc][rr], 1.0 / sig[cc]) : cmake(0.0, 0.0);
#pragma unroll 1
    for (int attempt = 0; attempt <= D; ++attempt) {
      if (attempt > 0) {  // complete with unit vector e = attempt - 1
        if (ok) break;
#pragma unroll 1
        for (int rr = 0; rr < D; ++rr) Tm[rr * D + kk] = cmake(rr == attempt - 1 ? 1.0 : 0.0, 0.0);
      }
#pragma unroll 1
      for (int rep = 0; rep < 2; ++rep)
#pragma unroll 1
        for (int o = 0; o < kk; ++o) {
          c128 dd = cmake(0.0, 0.0);
#pragma unroll 1
          for (int rr = 0; rr < D; ++rr) cfma(dd, cconj(Tm[rr * D + o]), Tm[rr * D + kk]);
#pragma unroll 1
          for (int rr = 0; rr < D; ++rr) Tm[rr * D + kk] = Tm[rr * D + kk] - dd * Tm[rr * D + o];
        }
      double nn = 0.0;
#pragma unroll 1
      for (int rr = 0; rr < D; ++rr) nn += cabs2(Tm[rr * D + kk]);
      nn = sqrt(nn);
      if (nn > 0.5) {
#pragma unroll 1
        for (int rr = 0; rr < D; ++rr) Tm[rr * D + kk] = cscale(Tm[rr * D + kk], 1.0 / nn);
        ok = true;
        break;
      }
      ok = false;
    }
  }
#pragma unroll 1
  for (int q = 0; q < D; ++q)
#pragma unroll 1
    for (int p2 = 0; p2 < D; ++p2) {
      c128 acc = cmake(0.0, 0.0);
#pragma unroll 1
      for (int kk = 0; kk < D; ++kk) cfma_conj(acc, Tm[q * D + kk], Vc[ord[kk]][p2]);
      u[q * D + p2] = acc;
    }
}

constexpr int kQdFinBlock = 128;  // eight 16-lane rows: one column pair each (DM <= 16)

// LDS workspace of one DM x DM polar update.
template <int DM>
struct QdPolarLds {
  static constexpr int PL = (DM + 1) / 2 * 2;  // players of the round-robin schedule
  c128 Gc[PL][16];   // G by columns: Gc[c][r] = G[r][c]
  c128 Vc[PL][16];   // V by columns
  c128 Tm[DM * DM];  // the mixed environment (row-major), then W in the singular case
  c128 Vs[DM * DM];  // V_prev (row-major) in, the new V out
  c128 Nm[DM * DM];  // V_prev^dagger V_prev
  c128 Pu[DM * DM];  // the polar factor (row-major) out
  double sig[DM];
};

// The whole block: Pu <- the unitary polar factor of Tm, started from V_prev in Vs, and the
// new right singular vectors into Vs (Tm and Vs filled and a barrier passed by the caller).
template <int DM>
__device__ void qd_polar_block(QdPolarLds<DM> &W) {
  constexpr int PL = QdPolarLds<DM>::PL;
  constexpr int NP = PL / 2;  // pairs per round
  static_assert(DM <= 16 && NP * 16 <= kQdFinBlock, "one 16-lane row per pair");
  const int t = threadIdx.x;
  for (int e = t; e < PL * 16; e += kQdFinBlock) {
    W.Gc[e >> 4][e & 15] = cmake(0.0, 0.0);
    W.Vc[e >> 4][e & 15] = cmake(0.0, 0.0);
  }
  // Newton-Schulz on V_prev: N = V^dagger V, then V <- V (3I - N) / 2 (into Vc by columns)
  for (int e = t; e < DM * DM; e += kQdFinBlock) {
    const int i = e / DM, j = e % DM;
    c128 acc = cmake(0.0, 0.0);
    for (int kk = 0; kk < DM; ++kk) cfma(acc, cconj(W.Vs[kk * DM + i]), W.Vs[kk * DM + j]);
    W.Nm[e] = acc;
  }
  __syncthreads();
  for (int e = t; e < DM * DM; e += kQdFinBlock) {
    const int i = e / DM, j = e % DM;
    c128 acc = cmake(0.0, 0.0);
    for (int kk = 0; kk < DM; ++kk) {
      const c128 x = W.Nm[kk * DM + j];
      cfma(acc, W.Vs[i * DM + kk], cmake((kk == j ? 3.0 : 0.0) - x.re, -x.im));
    }
    W.Vc[j][i] = cscale(acc, 0.5);
  }
  __syncthreads();
  // G <- Gamma V
  for (int e = t; e < DM * DM; e += kQdFinBlock) {
    const int i = e / DM, j = e % DM;
    c128 acc = cmake(0.0, 0.0);
    for (int kk = 0; kk < DM; ++kk) cfma(acc, W.Tm[i * DM + kk], W.Vc[j][kk]);
    W.Gc[j][i] = acc;
  }
  __syncthreads();
  const int pi = t >> 4, r = t & 15;  // pair (row of 16 lanes) and matrix row of this lane
  const bool worker = pi < NP;
  // rotate when |Gram_pq| > tol sqrt(al be), compared squared
  constexpr double kTol2 = kQdJacobiTol * kQdJacobiTol;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
#pragma unroll 1
    for (int rd = 0; rd < PL - 1; ++rd) {
      if (worker) {
        const int p = pi == 0 ? 0 : (rd + pi) % (PL - 1) + 1;
        const int q = pi == 0 ? rd % (PL - 1) + 1 : (rd - pi + PL - 1) % (PL - 1) + 1;
        const c128 gp = W.Gc[p][r], gq = W.Gc[q][r], vp = W.Vc[p][r], vq = W.Vc[q][r];
        double al = cabs2(gp), be = cabs2(gq);
        double gr = gp.re * gq.re + gp.im * gq.im;  // conj(gp) gq
        double gi = gp.re * gq.im - gp.im * gq.re;
        al += xor_lane<1>(al);
        be += xor_lane<1>(be);
        gr += xor_lane<1>(gr);
        gi += xor_lane<1>(gi);
        al += xor_lane<2>(al);
        be += xor_lane<2>(be);
        gr += xor_lane<2>(gr);
        gi += xor_lane<2>(gi);
        al += xor_lane<4>(al);
        be += xor_lane<4>(be);
        gr += xor_lane<4>(gr);
        gi += xor_lane<4>(gi);
        al += xor_lane<8>(al);
        be += xor_lane<8>(be);
        gr += xor_lane<8>(gr);
        gi += xor_lane<8>(gi);
        const double x2 = gr * gr + gi * gi, ab = al * be;
        if (x2 > 0.0 && x2 > kTol2 * ab) {
          rotated = 1;
          const double rag = rsq_nr(x2);               // 1 / |Gram_pq|
          const c128 ec = cmake(gr * rag, -gi * rag);  // conj(Gram_pq) / |Gram_pq|
          const double tau = (be - al) * (0.5 * rag);
          const double t1 = fma(tau, tau, 1.0);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(tau) + t1 * rsq_nr(t1));
          const double cs = rsq_nr(fma(tt, tt, 1.0)), sn = cs * tt;
          const c128 egq = ec * gq, evq = ec * vq;
          W.Gc[p][r] = cmake(cs * gp.re - sn * egq.re, cs * gp.im - sn * egq.im);
          W.Gc[q][r] = cmake(sn * gp.re + cs * egq.re, sn * gp.im + cs * egq.im);
          W.Vc[p][r] = cmake(cs * vp.re - sn * evq.re, cs * vp.im - sn * evq.im);
          W.Vc[q][r] = cmake(sn * vp.re + cs * evq.re, sn * vp.im + cs * evq.im);
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  // singular values (column norms of G); the new V by rows
  if (t < DM) {
    double a = 0.0;
    for (int rr = 0; rr < DM; ++rr) a += cabs2(W.Gc[t][rr]);
    W.sig[t] = sqrt(a);
  }
  for (int e = t; e < DM * DM; e += kQdFinBlock) W.Vs[e] = W.Vc[e % DM][e / DM];
  __syncthreads();
  double smax = 0.0, smin = INFINITY;
  for (int c = 0; c < DM; ++c) {
    smax = fmax(smax, W.sig[c]);
    smin = fmin(smin, W.sig[c]);
  }
  if (smin > 1e-200 && smin > 1e-13 * smax) {
    // u = W V^dagger with W = G diag(1 / sigma)
    for (int e = t; e < DM * DM; e += kQdFinBlock) {
      const int i = e / DM, c = e % DM;
      c128 acc = cmake(0.0, 0.0);
      for (int kk = 0; kk < DM; ++kk) cfma_conj(acc, cscale(W.Gc[kk][i], 1.0 / W.sig[kk]), W.Vc[kk][c]);
      W.Pu[e] = acc;
    }
  } else if (t == 0) {
    // a (near) singular environment: thread 0 alone
    qd_polar_singular<DM, PL>(W.Gc, W.Vc, W.Tm, W.sig, smax, W.Pu);
  }
  __syncthreads();
}

// Fixed-order sum of the work-group partials of entry e of a start's environment (partial
// i in running sum i mod 8, each batch of eight loads in flight together).
template <int D>
__device__ __forceinline__ c128 qd_partial_sum(const c128 *partials, int32_t P, int s, int e) {
  const c128 *src = partials + (int64_t)s * P * D * D + e;
  c128 acc[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) acc[v] = cmake(0.0, 0.0);
  int blk = 0;
  for (; blk + 7 < P; blk += 8) {
    c128 x[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) x[v] = src[(int64_t)(blk + v) * D * D];
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[v] = acc[v] + x[v];
  }
#pragma unroll
  for (int v = 0; v < 7; ++v)
    if (blk + v < P) acc[v] = acc[v] + src[(int64_t)(blk + v) * D * D];
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__device__ __forceinline__ c128 qd_mix(c128 g, c128 u, double beta) {
  return beta != 0.0 ? cmake((1.0 - beta) * g.re + beta * u.re, (1.0 - beta) * g.im + beta * u.im) : g;
}

template <int d>
__global__ __launch_bounds__(kQdFinBlock) void k_qd_finalize(const c128 *partials, int32_t P, double beta,
                                                             const int32_t *slots, c128 *gates, c128 *vstore,
                                                             int32_t gstride, int32_t k) {
  constexpr int D = d * d;
  __shared__ QdPolarLds<D> W;
  const int s = slots[blockIdx.x];
  c128 *u = gates + (int64_t)s * gstride + (int64_t)k * D * D;
  c128 *vst = vstore + (int64_t)s * gstride + (int64_t)k * D * D;
  const int t = threadIdx.x;
  for (int e = t; e < D * D; e += kQdFinBlock) {
    W.Tm[e] = qd_mix(qd_partial_sum<D>(partials, P, s, e), u[e], beta);
    W.Vs[e] = vst[e];
  }
  __syncthreads();
  qd_polar_block<D>(W);
  for (int e = t; e < D * D; e += kQdFinBlock) {
    u[e] = W.Pu[e];
    vst[e] = W.Vs[e];
  }
}

// A one-qudit gate v on the slot's first qudit, held as v (x) I_d: its d x d environment is
// the trace of the slot's D x D environment over the spectator digit,
// G1[x][y] = sum_z G[d x + z][d y + z]; v <- polar((1 - beta) G1 + beta v), written back as
// v (x) I_d. Its warm-start V (d x d) sits at the slot positions (d x, d y) of the stored V.
template <int d>
__global__ __launch_bounds__(kQdFinBlock) void k_qd_finalize1(const c128 *partials, int32_t P, double beta,
                                                              const int32_t *slots, c128 *gates, c128 *vstore,
                                                              int32_t gstride, int32_t k) {
  constexpr int D = d * d;
  __shared__ QdPolarLds<d> W;
  __shared__ c128 Gf[D * D];
  const int s = slots[blockIdx.x];
  c128 *u = gates + (int64_t)s * gstride + (int64_t)k * D * D;
  c128 *vst = vstore + (int64_t)s * gstride + (int64_t)k * D * D;
  const int t = threadIdx.x;
  for (int e = t; e < D * D; e += kQdFinBlock) Gf[e] = qd_partial_sum<D>(partials, P, s, e);
  __syncthreads();
  for (int e = t; e < d * d; e += kQdFinBlock) {
    const int x = e / d, y = e % d;
    c128 g1 = cmake(0.0, 0.0);
    for (int z = 0; z < d; ++z) g1 = g1 + Gf[(d * x + z) * D + d * y + z];
    W.Tm[e] = qd_mix(g1, u[(d * x) * D + d * y], beta);
    W.Vs[e] = vst[(d * x) * D + d * y];
  }
  __syncthreads();
  qd_polar_block<d>(W);
  for (int e = t; e < D * D; e += kQdFinBlock) {
    const int r = e / D, c = e % D;
    u[e] = (r % d == c % d) ? W.Pu[(r / d) * d + c / d] : cmake(0.0, 0.0);
  }
  for (int e = t; e < d * d; e += kQdFinBlock) vst[(d * (e / d)) * D + d * (e % d)] = W.Vs[e];
}

// count D x D identity matrices (the initial warm-start V).
__global__ void k_qd_identity(int64_t count, int D, c128 *v) {
  const int64_t tot = count * D * D;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % ((int64_t)D * D);
    v[e] = cmake((w / D == w % D) ? 1.0 : 0.0, 0.0);
  }
}

// sum |x - ref|^2 over a set, per block, FP64 (partials[s][blk]).
template <typename R>
__global__ __launch_bounds__(kQdBlock) void k_qd_dist(const cx<R> *x, int64_t x_stride, const cx<R> *ref,
                                                      int64_t ref_stride, int64_t count, double *partials,
                                                      const int32_t *slots) {
  __shared__ double red[kQdBlock / 64];
  const int s = slots[blockIdx.y];
  const cx<R> *xs = x + (int64_t)s * x_stride;
  const cx<R> *rs = ref + (int64_t)s * ref_stride;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)kQdBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kQdBlock) {
    const double dr = (double)xs[e].re - (double)rs[e].re, di = (double)xs[e].im - (double)rs[e].im;
    acc += dr * dr + di * di;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kQdBlock / 64; ++w) t += red[w];
    partials[(int64_t)s * gridDim.x + blockIdx.x] = t;
  }
}

// Sample-major [rows][N] complex128 (rows row0 .. row0 + M - 1 of src) to amplitude-major
// [N][M] in precision R.
template <typename R>
__global__ void k_qd_pack(const c128 *src, int64_t N, int64_t row0, int32_t M, cx<R> *dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * M; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / M, j = e % M;
    const c128 v = src[(row0 + j) * N + i];
    dst[e] = cmake<R>((R)v.re, (R)v.im);
  }
}

// Haar D x D initial gates: Ginibre block at indices 256 gate + D col + row of the start's
// initial-gate stream, orthonormalised column by column (positive diag(R)).
template <int d>
__global__ void k_qd_haar(uint64_t seed, int32_t start0, int32_t starts, int32_t L, c128 *out) {
  constexpr int D = d * d;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)starts * L) return;
  const int s = (int)(t / L), k = (int)(t % L);
  c128 q[D][D];  // [col][row]
  for (int c = 0; c < D; ++c)
    for (int r = 0; r < D; ++r)
      q[c][r] = complex_normal(seed, kRoleInit, (uint32_t)(start0 + s), (uint64_t)k * 256u + (uint64_t)(c * D + r));
  for (int c = 0; c < D; ++c) {
    for (int rep = 0; rep < 2; ++rep)
      for (int o = 0; o < c; ++o) {
        c128 dd = cmake(0.0, 0.0);
        for (int r = 0; r < D; ++r) cfma(dd, cconj(q[o][r]), q[c][r]);
        for (int r = 0; r < D; ++r) q[c][r] = q[c][r] - dd * q[o][r];
      }
    double nn = 0.0;
    for (int r = 0; r < D; ++r) nn += cabs2(q[c][r]);
    const double inv = 1.0 / sqrt(nn);
    for (int r = 0; r < D; ++r) q[c][r] = cscale(q[c][r], inv);
  }
  c128 *u = out + t * D * D;
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) u[r * D + c] = q[c][r];
}

// Gate kinds of the initial slots: a constant gate's slot takes the template's gate (every
// start); with drawn gates, a one-qudit gate's slot becomes v (x) I_d with v Haar on U(d)
// from the d x d Ginibre block at indices 256 gate + d col + row of the start's stream.
template <int d>
__global__ void k_qd_kinds(uint64_t seed, int32_t start0, int32_t starts, int32_t L, const int32_t *kinds,
                           const c128 *fixed, int32_t drawn, c128 *out) {
  constexpr int D = d * d;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)starts * L) return;
  const int s = (int)(t / L), k = (int)(t % L);
  c128 *u = out + t * D * D;
  if (kinds[k] == QFS_GATE_FIXED) {
    for (int e = 0; e < D * D; ++e) u[e] = fixed[(int64_t)k * D * D + e];
    return;
  }
  if (kinds[k] != QFS_GATE_1Q || !drawn) return;
  c128 q[d][d];  // [col][row]
  for (int c = 0; c < d; ++c)
    for (int r = 0; r < d; ++r)
      q[c][r] = complex_normal(seed, kRoleInit, (uint32_t)(start0 + s), (uint64_t)k * 256u + (uint64_t)(c * d + r));
  for (int c = 0; c < d; ++c) {
    for (int rep = 0; rep < 2; ++rep)
      for (int o = 0; o < c; ++o) {
        c128 dd = cmake(0.0, 0.0);
        for (int r = 0; r < d; ++r) cfma(dd, cconj(q[o][r]), q[c][r]);
        for (int r = 0; r < d; ++r) q[c][r] = q[c][r] - dd * q[o][r];
      }
    double nn = 0.0;
    for (int r = 0; r < d; ++r) nn += cabs2(q[c][r]);
    const double inv = 1.0 / sqrt(nn);
    for (int r = 0; r < d; ++r) q[c][r] = cscale(q[c][r], inv);
  }
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) u[r * D + c] = (r % d == c % d) ? q[c / d][r / d] : cmake(0.0, 0.0);
}

double qd_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t qd_pow(int d, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= d;
  return r;
}

int qd_grid(int64_t items) { return (int)std::min<int64_t>((items + kQdBlock - 1) / kQdBlock, 4096); }

// One problem's device state: the sweep machinery over `S` starts for state precision R.
template <typename R>
struct QdSweeper {
  int d = 0, n = 0, L = 0, S = 0;
  int64_t N = 0;
  const int32_t *pairs = nullptr;  // host [L][2]
  const int32_t *kinds = nullptr;  // host [L] or nullptr (every gate QFS_GATE_2Q)
  hipStream_t st = nullptr;
  int M = 0, Mv = 0;
  DevBuf psi, phi, psiv, phiv;  // working sets [N][M] in R (shared by the starts)
  DevBuf blist, astate, vstate, partials, dpart, costs, slots;
  c128 *g64 = nullptr;  // [S][L][D][D]
  c128 *vst = nullptr;  // [S][L][D][D] Jacobi warm start
  double beta = 0.0;
  int nslots = 0;
  // second stream of the backward pass (default priority) and its fork/join events: the
  // two halves of the running starts go on two streams, so one half's environment
  // reduction and polar update overlap the other half's propagation and reduction
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool one_stream = false;  // keep the whole sweep on `st` (problems run side by side)

  QdSweeper() = default;
  QdSweeper(const QdSweeper &) = delete;
  QdSweeper &operator=(const QdSweeper &) = delete;
  ~QdSweeper() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
  }

  int D() const { return d * d; }
  int64_t set() const { return N * M; }

  // (sl, ns, s: the starts a launch covers and its stream; the partial-sum block count
  // P depends on the geometry only, and the partials are indexed by start, so
  // launches over disjoint start sets never share them)
  template <int dd>
  int apply_t(const cx<R> *src, int64_t ss, cx<R> *dst, int64_t ds, int k, bool dagger, int Mrows,
              const int32_t *sl, int ns, hipStream_t s) {
    const int qa = pairs[2 * k], qb = pairs[2 * k + 1];
    const QdGeom g = qd_geom(dd, n, Mrows, qa, qb);
    hipLaunchKernelGGL((k_qd_apply<R, dd>), dim3(qd_grid(g.groups * Mrows), ns), dim3(kQdBlock), 0, s, src, ss,
                       dst, ds, g64, L * dd * dd * dd * dd, k, dagger ? 1 : 0, g, sl);
    QFS_HIP(hipGetLastError());
    return QFS_OK;
  }
  int apply_on(const cx<R> *src, int64_t ss, cx<R> *dst, int64_t ds, int k, bool dagger, int Mrows,
               const int32_t *sl, int ns, hipStream_t s) {
    return d == 2   ? apply_t<2>(src, ss, dst, ds, k, dagger, Mrows, sl, ns, s)
           : d == 3 ? apply_t<3>(src, ss, dst, ds, k, dagger, Mrows, sl, ns, s)
                    : apply_t<4>(src, ss, dst, ds, k, dagger, Mrows, sl, ns, s);
  }
  int apply(const cx<R> *src, int64_t ss, cx<R> *dst, int64_t ds, int k, bool dagger, int Mrows) {
    return apply_on(src, ss, dst, ds, k, dagger, Mrows, slots.as<int32_t>(), nslots, st);
  }
  template <int dd>
  int env_t(const cx<R> *a, int64_t as, const cx<R> *b, int64_t bs, int k, const int32_t *sl, int ns,
            hipStream_t s) {
    const QdGeom g = qd_geom(dd, n, M, pairs[2 * k], pairs[2 * k + 1]);
    const int P = (int)std::max<int64_t>(1, std::min<int64_t>(kQdMaxP, (g.groups * M + kQdBlock - 1) / kQdBlock));
    hipLaunchKernelGGL((k_qd_env<R, dd>), dim3(dd * dd / qd_env_rows<dd>() * P, ns), dim3(kQdBlock), 0, s, a, as,
                       b, bs, g, P, partials.as<c128>(), sl);
    QFS_HIP(hipGetLastError());
    if (kinds && kinds[k] == QFS_GATE_1Q)
      hipLaunchKernelGGL((k_qd_finalize1<dd>), dim3(ns), dim3(kQdFinBlock), 0, s, partials.as<c128>(), P, beta, sl,
                         g64, vst, L * dd * dd * dd * dd, k);
    else
      hipLaunchKernelGGL((k_qd_finalize<dd>), dim3(ns), dim3(kQdFinBlock), 0, s, partials.as<c128>(), P, beta, sl,
                         g64, vst, L * dd * dd * dd * dd, k);
    QFS_HIP(hipGetLastError());
    return QFS_OK;
  }
  int env_on(const cx<R> *a, int64_t as, const cx<R> *b, int64_t bs, int k, const int32_t *sl, int ns,
             hipStream_t s) {
    return d == 2   ? env_t<2>(a, as, b, bs, k, sl, ns, s)
           : d == 3 ? env_t<3>(a, as, b, bs, k, sl, ns, s)
                    : env_t<4>(a, as, b, bs, k, sl, ns, s);
  }
  int dist(const cx<R> *x, int64_t xs, const cx<R> *ref, int64_t rs, int64_t count, int Mrows, double *out) {
    const int P = (int)std::min<int64_t>(kQdMaxP * 4, (count + kQdBlock - 1) / kQdBlock);
    hipLaunchKernelGGL((k_qd_dist<R>), dim3(P, nslots), dim3(kQdBlock), 0, st, x, xs, ref, rs, count,
                       dpart.as<double>(), slots.as<int32_t>());
    QFS_HIP(hipGetLastError());
    return launch_dist_finalize(P, dpart.as<double>(), slots.as<int32_t>(), nslots, Mrows, out, st);
  }

  size_t budget = 0;  // device bytes the sweeper may hold (0: as much as allocates)

  int alloc(int Mnew, int Mvnew) {
    M = Mnew;
    Mv = Mvnew;
    const size_t cb = sizeof(cx<R>);
    if (budget) {
      const size_t need = cb * set() * (2 + (size_t)std::max(L - 1, 1) * S + S) +
                          (Mv > 0 ? cb * N * Mv * (2 + (size_t)S) : 0) +
                          sizeof(c128) * (size_t)S * kQdMaxP * kQdMaxDD;
      if (need > budget) {
        set_error_detail("qudits: the sets and B lists of " + std::to_string(S) + " starts need " +
                         std::to_string(need) + " bytes, above the device budget");
        return QFS_ENOMEM;
      }
    }
    QFS_TRY(psi.alloc(cb * set()));
    QFS_TRY(phi.alloc(cb * set()));
    QFS_TRY(blist.alloc(cb * set() * (size_t)std::max(L - 1, 1) * S));
    QFS_TRY(astate.alloc(cb * set() * S));
    if (Mv > 0) {
      QFS_TRY(psiv.alloc(cb * N * Mv));
      QFS_TRY(phiv.alloc(cb * N * Mv));
      QFS_TRY(vstate.alloc(cb * N * Mv * S));
    }
    QFS_TRY(partials.alloc(sizeof(c128) * (size_t)S * kQdMaxP * kQdMaxDD));
    QFS_TRY(dpart.alloc(sizeof(double) * (size_t)S * kQdMaxP * 4));
    if (!costs.ptr) QFS_TRY(costs.alloc(sizeof(double) * 3 * S));
    if (!slots.ptr) QFS_TRY(slots.alloc(sizeof(int32_t) * S));
    return QFS_OK;
  }

  // forward: B list from the current gates; with_c0: cost of the current gates
  // (costs[2S + s]); validation cost (costs[S + s]) when Mv > 0
  int forward(bool with_c0) {
    cx<R> *P0 = psi.as<cx<R>>(), *B = blist.as<cx<R>>();
    const int64_t sN = set(), bstride = sN * std::max(L - 1, 1);
    for (int k = 0; k < L - 1; ++k)
      QFS_TRY(apply(k == 0 ? P0 : B + (k - 1) * sN, k == 0 ? 0 : bstride, B + k * sN, bstride, k, false, M));
    if (with_c0) {
      cx<R> *A = astate.as<cx<R>>();
      QFS_TRY(apply(L == 1 ? P0 : B + (L - 2) * sN, L == 1 ? 0 : bstride, A, sN, L - 1, false, M));
      QFS_TRY(dist(A, sN, phi.as<cx<R>>(), 0, sN, M, costs.as<double>() + 2 * S));
    }
    if (Mv > 0) {
      cx<R> *V = vstate.as<cx<R>>();
      const int64_t vN = N * Mv;
      for (int k = 0; k < L; ++k)
        QFS_TRY(apply(k == 0 ? psiv.as<cx<R>>() : V, k == 0 ? 0 : vN, V, vN, k, false, Mv));
      QFS_TRY(dist(V, vN, phiv.as<cx<R>>(), 0, vN, Mv, costs.as<double>() + S));
    }
    return QFS_OK;
  }

  // right to left: a <- u_{k+1}^dagger a, Gamma_k against B_k, u_k <- polar; then the
  // Eq. 9 cost of the updated gates (costs[s])
  int backward() {
    cx<R> *P0 = psi.as<cx<R>>(), *F = phi.as<cx<R>>(), *B = blist.as<cx<R>>(), *A = astate.as<cx<R>>();
    const int64_t sN = set(), bstride = sN * std::max(L - 1, 1);
    static const bool split_ok = [] {
      const char *e = std::getenv("QFS_BWD_SPLIT");  // 0: one stream for the backward pass
      return !(e && std::atoi(e) == 0);
    }();
    const bool split = split_ok && !one_stream && nslots >= 2;
    if (split && !side) {
      QFS_TRY(pool_stream(2, &side));
      QFS_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
      QFS_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    }
    const int halves = split ? 2 : 1, h0 = split ? nslots / 2 : nslots;
    const int32_t *hsl[2] = {slots.as<int32_t>(), slots.as<int32_t>() + h0};
    const int hn[2] = {h0, nslots - h0};
    hipStream_t hst[2] = {st, side};
    if (split) {
      QFS_HIP(hipEventRecord(fork, st));
      QFS_HIP(hipStreamWaitEvent(side, fork, 0));
    }
    for (int k = L - 1; k >= 0; --k) {
      const cx<R> *a = k == L - 1 ? F : A;
      const int64_t as = k == L - 1 ? 0 : sN;
      for (int h = 0; h < halves; ++h) {
        if (k < L - 1)
          QFS_TRY(apply_on(k == L - 2 ? F : A, k == L - 2 ? 0 : sN, A, sN, k + 1, true, M, hsl[h], hn[h], hst[h]));
        if (!(kinds && kinds[k] == QFS_GATE_FIXED))  // a constant gate has no environment
          QFS_TRY(env_on(a, as, k == 0 ? P0 : B + (k - 1) * sN, k == 0 ? 0 : bstride, k, hsl[h], hn[h], hst[h]));
      }
    }
    if (split) {
      QFS_HIP(hipEventRecord(join, side));
      QFS_HIP(hipStreamWaitEvent(st, join, 0));
    }
    QFS_TRY(apply(L == 1 ? F : A, L == 1 ? 0 : sN, A, sN, 0, true, M));
    QFS_TRY(dist(A, sN, P0, 0, sN, M, costs.as<double>()));
    return QFS_OK;
  }

  int set_slots(const std::vector<int> &active) {
    nslots = (int)active.size();
    if (nslots == 0) return QFS_OK;
    QFS_HIP(hipMemcpyAsync(slots.ptr, active.data(), sizeof(int32_t) * nslots, hipMemcpyHostToDevice, st));
    return QFS_OK;
  }
};

// Host check that count D x D gates (device) are unitary to 1e-10.
int check_gates_unitary_n(const qfs_c128 *gates_dev, size_t count, int D, const char *what, hipStream_t s) {
  std::vector<qfs_c128> h(count * D * D);
  QFS_HIP(hipMemcpyAsync(h.data(), gates_dev, sizeof(qfs_c128) * h.size(), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  for (size_t gi = 0; gi < count; ++gi) {
    const qfs_c128 *u = h.data() + gi * D * D;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double re = (i == j) ? -1.0 : 0.0, im = 0.0;
        for (int k = 0; k < D; ++k) {
          const qfs_c128 a = u[k * D + i], b = u[k * D + j];  // conj(u[k][i]) u[k][j]
          re += a.re * b.re + a.im * b.im;
          im += a.re * b.im - a.im * b.re;
        }
        if (!std::isfinite(re) || !std::isfinite(im) || std::fabs(re) > 1e-10 || std::fabs(im) > 1e-10) {
          set_error_detail(std::string(what) + ": gate " + std::to_string(gi) + " is not unitary to 1e-10");
          return QFS_EINVAL;
        }
      }
  }
  return QFS_OK;
}

int qd_validate(int d, const qfs_template *t) {
  if (d < 2 || d > 4) {
    set_error_detail("qudits: d must be 2, 3 or 4");
    return QFS_EUNSUPPORTED;
  }
  if (!t || t->n_qubits < 2 || t->n_gates < 1 || !t->pairs || qd_pow(d, t->n_qubits) > (int64_t(1) << 24)) {
    set_error_detail("qudits: need n >= 2, d^n <= 2^24, n_gates >= 1, pairs");
    return QFS_EINVAL;
  }
  for (int k = 0; k < t->n_gates; ++k) {
    const int a = t->pairs[2 * k], b = t->pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= t->n_qubits || b >= t->n_qubits || a == b) {
      set_error_detail("qudits: gate " + std::to_string(k) + " has an invalid qudit pair");
      return QFS_EINVAL;
    }
    if (t->kinds && (t->kinds[k] < QFS_GATE_2Q || t->kinds[k] > QFS_GATE_FIXED)) {
      set_error_detail("qudits: gate " + std::to_string(k) + " has an unknown kind");
      return QFS_EINVAL;
    }
  }
  return QFS_OK;
}

// Load rows [row0, row0 + M) of a sample-major complex128 set into an amplitude-major R set.
template <typename R>
int qd_pack(const qfs_c128 *src, int64_t N, int row0, int M, DevBuf &dst, hipStream_t st) {
  if (M <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_qd_pack<R>, dim3(qd_grid(N * M)), dim3(kQdBlock), 0, st, reinterpret_cast<const c128 *>(src),
                     N, (int64_t)row0, M, dst.as<cx<R>>());
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

template <typename R>
int qd_load_sets(QdSweeper<R> &w, const qfs_c128 *psi, const qfs_c128 *phi, int n_train, int n_val) {
  QFS_TRY(qd_pack<R>(psi, w.N, 0, w.M, w.psi, w.st));
  QFS_TRY(qd_pack<R>(phi, w.N, 0, w.M, w.phi, w.st));
  if (w.Mv > 0) {
    QFS_TRY(qd_pack<R>(psi, w.N, n_train, n_val, w.psiv, w.st));
    QFS_TRY(qd_pack<R>(phi, w.N, n_train, n_val, w.phiv, w.st));
  }
  return QFS_OK;
}

// FP64 amplitude-major master [N][M] into a working set in precision R.
template <typename R>
int qd_from_master(const DevBuf &src, int64_t count, DevBuf &dst, hipStream_t st) {
  if (count <= 0) return QFS_OK;
  if constexpr (sizeof(R) == 8) {
    QFS_HIP(hipMemcpyAsync(dst.ptr, src.ptr, sizeof(c128) * (size_t)count, hipMemcpyDeviceToDevice, st));
    return QFS_OK;
  } else {
    return launch_narrow(count, src.as<c128>(), dst.as<c64>(), st);
  }
}

// x <- u_k x for k = 0 .. Lt-1 (gates [Lt][D][D], FP64) on an amplitude-major FP64 set of
// `cols` samples: the target circuit's output states.
template <int dd>
int qd_apply_circuit(int n, int cols, c128 *x, const qfs_template *ct, const c128 *gates, const int32_t *slot0,
                     hipStream_t st) {
  for (int k = 0; k < ct->n_gates; ++k) {
    const QdGeom g = qd_geom(dd, n, cols, ct->pairs[2 * k], ct->pairs[2 * k + 1]);
    hipLaunchKernelGGL((k_qd_apply<double, dd>), dim3(qd_grid(g.groups * cols), 1), dim3(kQdBlock), 0, st, x,
                       (int64_t)0, x, (int64_t)0, gates, 0, k, 0, g, slot0);
    QFS_HIP(hipGetLastError());
  }
  return QFS_OK;
}

// Where the sample pairs come from: the caller's fixed set (sample-major rows; the last
// n_val rows validate), or states drawn here (Sec. 3, App. A: columns of a Haar unitary;
// Philox roles, streams and indices as for qubits with N = d^n amplitudes) with their
// target outputs formed here, kept as FP64 amplitude-major masters [N][M]. A doubling
// extends the drawn training set by the next columns of its stream, orthonormalised
// against the earlier ones, and draws a new validation set (the next generation).
struct QdData {
  int d = 0, n = 0;
  int64_t N = 0;
  hipStream_t st = nullptr;
  const qfs_c128 *psi = nullptr, *phi = nullptr;  // fixed sets
  int n_train = 0, n_val = 0;
  const qfs_target *tgt = nullptr;  // drawn sets: DENSE or CIRCUIT target
  uint64_t seed = 0;
  int m_val = 0;
  int M = 0, Mv = 0, generation = 0;
  bool one_stream = false;  // the sweeps keep to the call's stream
  DevBuf tpsi, tphi, vpsi, vphi, work, slot0;

  bool drawn() const { return tgt != nullptr; }
  int val_rows() const { return drawn() ? Mv : n_val; }

  // dst = target applied to the `cols` states of src (both [N][cols])
  int targets(const DevBuf &src, DevBuf &dst, int cols) {
    if (tgt->kind == QFS_TARGET_DENSE) {
      return launch_zgemm(false, (int)N, cols, (int)N, cmake(1.0, 0.0), reinterpret_cast<const c128 *>(tgt->U),
                          (int)N, src.as<c128>(), cols, cmake(0.0, 0.0), dst.as<c128>(), cols, st);
    }
    QFS_HIP(hipMemcpyAsync(dst.ptr, src.ptr, sizeof(c128) * (size_t)N * cols, hipMemcpyDeviceToDevice, st));
    if (!slot0.ptr) {
      const int32_t zero = 0;
      QFS_TRY(slot0.alloc(sizeof(int32_t)));
      QFS_HIP(hipMemcpyAsync(slot0.ptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice, st));
      QFS_HIP(hipStreamSynchronize(st));
    }
    const c128 *tg = reinterpret_cast<const c128 *>(tgt->circuit_gates);
    c128 *x = dst.as<c128>();
    const int32_t *s0 = slot0.as<int32_t>();
    return d == 2   ? qd_apply_circuit<2>(n, cols, x, tgt->circuit, tg, s0, st)
           : d == 3 ? qd_apply_circuit<3>(n, cols, x, tgt->circuit, tg, s0, st)
                    : qd_apply_circuit<4>(n, cols, x, tgt->circuit, tg, s0, st);
  }
  // columns [c0, c1) of the [N][c1] set A: Ginibre draw, orthonormalised against columns
  // [0, c0) and among themselves
  int draw(DevBuf &A, int c0, int c1, uint32_t role, uint32_t stream) {
    QFS_TRY(launch_ginibre(N, c0, c1, c1, seed, role, stream, A.as<c128>(), st));
    QFS_TRY(work.alloc(work_bytes_orth(N, c1)));
    QFS_TRY(orthonormalize_columns(N, c1, c0, c1, A.as<c128>(), work.ptr, st));
    work.release();
    return QFS_OK;
  }
  int draw_validation(int Mtrain) {
    Mv = (int)std::min<int64_t>(m_val > 0 ? m_val : Mtrain, N);
    QFS_TRY(vpsi.alloc(sizeof(c128) * (size_t)N * Mv));
    QFS_TRY(vphi.alloc(sizeof(c128) * (size_t)N * Mv));
    QFS_TRY(draw(vpsi, 0, Mv, kRoleVal, (uint32_t)generation));
    return targets(vpsi, vphi, Mv);
  }
  int init(int M0) {
    if (!drawn()) return QFS_OK;
    M = M0;
    QFS_TRY(tpsi.alloc(sizeof(c128) * (size_t)N * M));
    QFS_TRY(tphi.alloc(sizeof(c128) * (size_t)N * M));
    QFS_TRY(draw(tpsi, 0, M, kRoleTrain, 0));
    QFS_TRY(targets(tpsi, tphi, M));
    return draw_validation(M);
  }
  int grow(int Mnew) {
    if (!drawn() || Mnew == M) return QFS_OK;
    DevBuf np, nf;
    QFS_TRY(np.alloc(sizeof(c128) * (size_t)N * Mnew));
    QFS_TRY(nf.alloc(sizeof(c128) * (size_t)N * Mnew));
    QFS_HIP(hipMemcpy2DAsync(np.ptr, sizeof(c128) * Mnew, tpsi.ptr, sizeof(c128) * M, sizeof(c128) * M, N,
                             hipMemcpyDeviceToDevice, st));
    QFS_TRY(draw(np, M, Mnew, kRoleTrain, 0));
    QFS_TRY(targets(np, nf, Mnew));  // each column's output depends on that column alone
    QFS_HIP(hipStreamSynchronize(st));
    std::swap(tpsi.ptr, np.ptr);
    std::swap(tpsi.bytes, np.bytes);
    std::swap(tphi.ptr, nf.ptr);
    std::swap(tphi.bytes, nf.bytes);
    M = Mnew;
    ++generation;
    return draw_validation(M);
  }
  template <typename R>
  int load(QdSweeper<R> &w) {
    if (!drawn()) return qd_load_sets<R>(w, psi, phi, n_train, n_val);
    QFS_TRY(qd_from_master<R>(tpsi, N * w.M, w.psi, st));
    QFS_TRY(qd_from_master<R>(tphi, N * w.M, w.phi, st));
    QFS_TRY(qd_from_master<R>(vpsi, N * w.Mv, w.psiv, st));
    QFS_TRY(qd_from_master<R>(vphi, N * w.Mv, w.phiv, st));
    return QFS_OK;
  }
};

// The App. A control loop on a fixed sample set, for one precision; returns when every
// start has stopped, a start succeeded, or the precision switch is due (refine = true).
struct QdState {
  std::vector<int> status, reason, iter, z;
  std::vector<int64_t> total;
  std::vector<double> c_prev, ct, cv;
  int M = 0, m_cap = 0, restarts = 0, m_total = 0, chosen = -1;
  bool need_c0 = true;
  int64_t start_sweeps = 0;
  double amp_updates = 0.0, sweep_seconds = 0.0;
};

template <typename R>
int qd_run(int d, const qfs_template *t, QdData &data, const qfs_params &p, c128 *g64, c128 *vst, int S,
           QdState &cs, double t0, bool &refine) {
  int n_val = data.val_rows();
  QdSweeper<R> w;
  w.d = d;
  w.n = t->n_qubits;
  w.L = t->n_gates;
  w.S = S;
  w.N = qd_pow(d, w.n);
  w.pairs = t->pairs;
  w.kinds = t->kinds;
  w.st = static_cast<hipStream_t>(p.hip_stream);
  w.g64 = g64;
  w.vst = vst;
  w.beta = effective_beta(p.beta, p.beta_normalized != 0, cs.M);
  w.budget = p.device_mem_budget;
  w.one_stream = data.one_stream;
  QFS_TRY(w.alloc(cs.M, n_val));
  QFS_TRY(data.load<R>(w));
  std::vector<int> active;
  for (int s = 0; s < S; ++s)
    if (cs.status[s] != ST_STOP) active.push_back(s);
  QFS_TRY(w.set_slots(active));
  std::vector<double> h(3 * S);
  auto read = [&]() -> int {
    QFS_HIP(hipMemcpyAsync(h.data(), w.costs.ptr, sizeof(double) * 3 * S, hipMemcpyDeviceToHost, w.st));
    QFS_HIP(hipStreamSynchronize(w.st));
    return QFS_OK;
  };
  hipEvent_t e0, e1;
  QFS_HIP(hipEventCreate(&e0));
  QFS_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  QFS_TRY(w.forward(cs.need_c0));
  QFS_TRY(read());
  if (cs.need_c0) {
    for (int s : active) cs.c_prev[s] = h[2 * S + s];
    cs.need_c0 = false;
  }
  const int64_t N = w.N;
  for (;;) {
    QFS_HIP(hipEventRecord(e0, w.st));
    QFS_TRY(w.backward());
    QFS_TRY(w.forward(false));
    QFS_HIP(hipEventRecord(e1, w.st));
    QFS_TRY(read());
    float ms = 0.f;
    QFS_HIP(hipEventElapsedTime(&ms, e0, e1));
    cs.sweep_seconds += 1e-3 * ms;
    cs.start_sweeps += (int64_t)active.size();
    cs.amp_updates += (double)active.size() * (double)(cs.M + n_val) * (double)N * (double)w.L;
    const bool full = (int64_t)cs.M == N;
    const bool timed_out = p.time_budget_s > 0 && qd_now() - t0 > p.time_budget_s;
    bool any_success = false, any_over = false;
    for (int s : active) {
      cs.ct[s] = h[s];
      cs.cv[s] = n_val > 0 ? h[S + s] : h[s];
      cs.status[s] = control_step(p, cs.ct[s], cs.cv[s], full || n_val == 0, cs.M < cs.m_cap, timed_out, cs.iter[s],
                                  cs.z[s], cs.total[s], cs.c_prev[s], cs.reason[s]);
      any_success |= cs.status[s] == ST_STOP && cs.reason[s] == QFS_SUCCESS;
      any_over |= cs.status[s] == ST_OVER;
    }
    if (any_success) {
      double best = INFINITY;
      for (int s : active)
        if (cs.status[s] == ST_STOP && cs.reason[s] == QFS_SUCCESS && cs.ct[s] < best) {
          best = cs.ct[s];
          cs.chosen = s;
        }
      return QFS_OK;
    }
    if (any_over) {
      // double-and-restart: more rows of the sample set, every gate kept (App. A)
      cs.M = std::min(2 * cs.M, cs.m_cap);
      cs.m_total += cs.M;
      ++cs.restarts;
      active.clear();
      for (int s = 0; s < S; ++s)
        if (cs.status[s] != ST_STOP) {
          cs.status[s] = ST_RUN;
          cs.iter[s] = 0;
          cs.z[s] = 0;
          active.push_back(s);
        }
      QFS_HIP(hipStreamSynchronize(w.st));
      QFS_TRY(data.grow(cs.M));
      n_val = data.val_rows();
      QFS_TRY(w.alloc(cs.M, n_val));
      w.beta = effective_beta(p.beta, p.beta_normalized != 0, cs.M);
      QFS_TRY(data.load<R>(w));
      QFS_TRY(w.set_slots(active));
      QFS_TRY(w.forward(true));
      QFS_TRY(read());
      for (int s : active) cs.c_prev[s] = h[2 * S + s];
      continue;
    }
    std::vector<int> next;
    for (int s : active)
      if (cs.status[s] == ST_RUN) next.push_back(s);
    if (next.empty()) return QFS_OK;
    if (sizeof(R) == 4) {
      double best = INFINITY;
      for (int s : next) best = std::min(best, cs.ct[s]);
      if (best < p.refine_below) {
        refine = true;  // complex128 sweeps from here, same gates and counters
        return QFS_OK;
      }
    }
    if (next.size() != active.size()) {
      // the forward pass of this sweep already holds the survivors' B lists (per start)
      active = next;
      QFS_TRY(w.set_slots(active));
    }
  }
}

// Multistart instantiation from initial gates (given or Haar-drawn) on the samples of
// `data`, FP64 or MIXED with refinement.
// One group of starts [start0, start0 + S) with its own control loop (all starts when
// the device memory holds them): the returned start's gates (host) and counters.
struct QdGroupResult {
  int reason = QFS_MAX_ITER, m_final = 0, sweeps = 0, restarts = 0, best = 0, m_total = 0, refined = 0;
  double c_train = INFINITY, c_val = INFINITY, sweep_seconds = 0.0, amp_updates = 0.0;
  int64_t start_sweeps = 0;
  std::vector<qfs_c128> gates;
};

int qd_group(int d, const qfs_template *tmpl, const QdData &cfg, const qfs_params &p, const qfs_c128 *gates_in,
             int start0, int S, double t0, QdGroupResult &r) {
  const int n = tmpl->n_qubits, L = tmpl->n_gates, D = d * d;
  const int64_t N = qd_pow(d, n);
  hipStream_t st = static_cast<hipStream_t>(p.hip_stream);
  QdData data;  // the group's own sets (drawn sets are drawn again from the same streams)
  data.psi = cfg.psi;
  data.phi = cfg.phi;
  data.n_train = cfg.n_train;
  data.n_val = cfg.n_val;
  data.tgt = cfg.tgt;
  data.seed = cfg.seed;
  data.m_val = cfg.m_val;
  data.one_stream = cfg.one_stream;
  data.d = d;
  data.n = n;
  data.N = N;
  data.st = st;
  DevBuf gates;
  QFS_TRY(gates.alloc(sizeof(c128) * (size_t)S * L * D * D));
  if (gates_in) {
    QFS_HIP(hipMemcpyAsync(gates.ptr, gates_in + (size_t)start0 * L * D * D, sizeof(c128) * (size_t)S * L * D * D,
                           hipMemcpyDeviceToDevice, st));
  } else {
    const int64_t tot = (int64_t)S * L;
    const dim3 grid((unsigned)((tot + 63) / 64));
    if (d == 2)
      hipLaunchKernelGGL(k_qd_haar<2>, grid, dim3(64), 0, st, p.seed, start0, S, L, gates.as<c128>());
    else if (d == 3)
      hipLaunchKernelGGL(k_qd_haar<3>, grid, dim3(64), 0, st, p.seed, start0, S, L, gates.as<c128>());
    else
      hipLaunchKernelGGL(k_qd_haar<4>, grid, dim3(64), 0, st, p.seed, start0, S, L, gates.as<c128>());
    QFS_HIP(hipGetLastError());
  }
  DevBuf dkinds;
  if (tmpl->kinds) {
    QFS_TRY(dkinds.alloc(sizeof(int32_t) * L));
    QFS_HIP(hipMemcpyAsync(dkinds.ptr, tmpl->kinds, sizeof(int32_t) * L, hipMemcpyHostToDevice, st));
    const int64_t tot = (int64_t)S * L;
    const dim3 grid((unsigned)((tot + 63) / 64));
    const c128 *fx = reinterpret_cast<const c128 *>(tmpl->fixed_gates);
    const int drawn = gates_in ? 0 : 1;
    if (d == 2)
      hipLaunchKernelGGL(k_qd_kinds<2>, grid, dim3(64), 0, st, p.seed, start0, S, L, dkinds.as<int32_t>(), fx,
                         drawn, gates.as<c128>());
    else if (d == 3)
      hipLaunchKernelGGL(k_qd_kinds<3>, grid, dim3(64), 0, st, p.seed, start0, S, L, dkinds.as<int32_t>(), fx,
                         drawn, gates.as<c128>());
    else
      hipLaunchKernelGGL(k_qd_kinds<4>, grid, dim3(64), 0, st, p.seed, start0, S, L, dkinds.as<int32_t>(), fx,
                         drawn, gates.as<c128>());
    QFS_HIP(hipGetLastError());
  }
  DevBuf vstore;
  QFS_TRY(vstore.alloc(sizeof(c128) * (size_t)S * L * D * D));
  hipLaunchKernelGGL(k_qd_identity, dim3(qd_grid((int64_t)S * L * D * D)), dim3(kQdBlock), 0, st, (int64_t)S * L, D,
                     vstore.as<c128>());
  QFS_HIP(hipGetLastError());
  QdState cs;
  cs.status.assign(S, ST_RUN);
  cs.reason.assign(S, QFS_MAX_ITER);
  cs.iter.assign(S, 0);
  cs.z.assign(S, 0);
  cs.total.assign(S, 0);
  cs.c_prev.assign(S, 0.0);
  cs.ct.assign(S, INFINITY);
  cs.cv.assign(S, INFINITY);
  cs.m_cap = (p.m_max > 0 && p.m_max < N) ? p.m_max : (int)N;
  if (!data.drawn()) cs.m_cap = std::min(cs.m_cap, data.n_train);
  cs.M = std::max(1, std::min(p.m_init, cs.m_cap));
  if (p.fixed_m) cs.m_cap = cs.M;
  cs.m_total = cs.M;
  QFS_TRY(data.init(cs.M));
  bool refine = false;
  if (p.precision == QFS_PREC_MIXED) {
    QFS_TRY(qd_run<float>(d, tmpl, data, p, gates.as<c128>(), vstore.as<c128>(), S, cs, t0, refine));
    if (refine) {
      r.refined = 1;
      QFS_TRY(qd_run<double>(d, tmpl, data, p, gates.as<c128>(), vstore.as<c128>(), S, cs, t0, refine));
    }
  } else {
    QFS_TRY(qd_run<double>(d, tmpl, data, p, gates.as<c128>(), vstore.as<c128>(), S, cs, t0, refine));
  }
  if (cs.chosen < 0) {
    double best = INFINITY;
    for (int s = 0; s < S; ++s)
      if (cs.ct[s] < best || cs.chosen < 0) {
        best = cs.ct[s];
        cs.chosen = s;
      }
  }
  const int c = cs.chosen;
  r.gates.resize((size_t)L * D * D);
  QFS_HIP(hipMemcpyAsync(r.gates.data(), gates.as<c128>() + (size_t)c * L * D * D, sizeof(c128) * r.gates.size(),
                         hipMemcpyDeviceToHost, st));
  QFS_HIP(hipStreamSynchronize(st));
  r.reason = cs.reason[c];
  r.m_final = cs.M;
  r.sweeps = (int32_t)cs.total[c];
  r.restarts = cs.restarts;
  r.best = start0 + c;
  r.m_total = cs.m_total;
  r.c_train = cs.ct[c];
  r.c_val = cs.cv[c];
  r.start_sweeps = cs.start_sweeps;
  r.sweep_seconds = cs.sweep_seconds;
  r.amp_updates = cs.amp_updates;
  return QFS_OK;
}

// App. A: when the starts' sets and B lists do not fit the device (out of memory, or
// params->device_mem_budget), the starts run as two halves, recursively, one after the
// other, each with its own control loop.
int qd_split(int d, const qfs_template *tmpl, const QdData &cfg, const qfs_params &p, const qfs_c128 *gates_in,
             int start0, int S, double t0, std::vector<QdGroupResult> &results) {
  QdGroupResult r;
  const int rc = qd_group(d, tmpl, cfg, p, gates_in, start0, S, t0, r);
  if (rc == QFS_ENOMEM && S > 1) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(p.hip_stream));
    (void)hipGetLastError();
    const int h = S / 2;
    QFS_TRY(qd_split(d, tmpl, cfg, p, gates_in, start0, h, t0, results));
    return qd_split(d, tmpl, cfg, p, gates_in, start0 + h, S - h, t0, results);
  }
  if (rc != QFS_OK) return rc;
  results.push_back(std::move(r));
  return QFS_OK;
}

// Multistart instantiation from initial gates (given or Haar-drawn) on the samples of
// `cfg`, FP64 or MIXED with refinement; the returned start is the best of the groups
// (a success first, then the lower training cost).
int qd_instantiate_impl(int d, const qfs_template *tmpl, const QdData &cfg, const qfs_params &p,
                        const qfs_c128 *gates_in, qfs_c128 *gates_out, qfs_result *res, double t0) {
  const int L = tmpl->n_gates, D = d * d;
  if (p.multistarts < 1 || p.m_init < 1 || p.max_iter < 1 || p.plateau_window < 1 || !(p.beta >= 0 && p.beta <= 1) ||
      (p.precision != QFS_PREC_FP64 && p.precision != QFS_PREC_MIXED) || p.full_unitary) {
    set_error_detail("qudits: bad params");
    return QFS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(p.hip_stream);
  const int S = p.multistarts;
  if (gates_in)
    QFS_TRY(check_gates_unitary_n(gates_in, (size_t)S * L, D, "gates_in", st));
  if (tmpl->kinds) {
    bool any_fixed = false;
    for (int k = 0; k < L; ++k) any_fixed |= tmpl->kinds[k] == QFS_GATE_FIXED;
    if (any_fixed && !tmpl->fixed_gates) {
      set_error_detail("qudits: constant gates need tmpl->fixed_gates");
      return QFS_EINVAL;
    }
  }
  std::vector<QdGroupResult> results;
  QFS_TRY(qd_split(d, tmpl, cfg, p, gates_in, 0, S, t0, results));
  size_t bi = 0;
  for (size_t i = 1; i < results.size(); ++i) {
    const bool si = results[i].reason == QFS_SUCCESS, sb = results[bi].reason == QFS_SUCCESS;
    if ((si && !sb) || (si == sb && results[i].c_train < results[bi].c_train)) bi = i;
  }
  const QdGroupResult &r = results[bi];
  QFS_HIP(hipMemcpyAsync(gates_out, r.gates.data(), sizeof(c128) * r.gates.size(), hipMemcpyHostToDevice, st));
  QFS_HIP(hipStreamSynchronize(st));
  std::memset(res, 0, sizeof(*res));
  res->reason = r.reason;
  res->m_final = r.m_final;
  res->sweeps = r.sweeps;
  res->restarts = r.restarts;
  res->best_start = r.best;
  res->m_total = r.m_total;
  res->start_groups = (int32_t)results.size();
  res->refined = r.refined;
  res->c_train = r.c_train;
  res->c_val = r.c_val;
  for (const auto &x : results) {
    res->start_sweeps += x.start_sweeps;
    res->sweep_seconds += x.sweep_seconds;
    res->amp_updates += x.amp_updates;
  }
  res->seconds = qd_now() - t0;
  return QFS_OK;
}

constexpr int kQdBatchStreams = 8;  // problems run side by side by the batched entry

// One problem: argument checks, then the multistart run on the samples or drawn states of
// its target. one_stream keeps every sweep on the call's stream (no second stream for half
// the starts), so problems on several streams do not share one.
int qd_entry(int d, const qfs_template *tmpl, const qfs_target *target, const qfs_params *params,
             const qfs_c128 *gates_in, qfs_c128 *gates_out, qfs_result *res, bool one_stream) {
  const double t0 = qd_now();
  if (!target) {
    set_error_detail("qudits: null target");
    return QFS_EINVAL;
  }
  QFS_TRY(qd_validate(d, tmpl));
  if (!params || !gates_out || !res) {
    set_error_detail("qudits: null argument");
    return QFS_EINVAL;
  }
  const int n = tmpl->n_qubits;
  const int64_t N = qd_pow(d, n);
  QdData data;
  data.one_stream = one_stream;
  if (target->kind == QFS_TARGET_SAMPLES) {
    const int n_train = target->n_samples - target->n_val;
    if (!target->psi || !target->phi || target->n_val < 0 || n_train < 1 || n_train > N) {
      set_error_detail(!target->psi || !target->phi ? "qudits: null argument" : "qudits: bad sample counts");
      return QFS_EINVAL;
    }
    data.psi = target->psi;
    data.phi = target->phi;
    data.n_train = n_train;
    data.n_val = target->n_val;
    return qd_instantiate_impl(d, tmpl, data, *params, gates_in, gates_out, res, t0);
  }
  if (target->kind == QFS_TARGET_DENSE) {
    if (!target->U || N > (int64_t(1) << 16)) {
      set_error_detail("qudits: a dense target needs U and d^n <= 2^16");
      return QFS_EINVAL;
    }
  } else if (target->kind == QFS_TARGET_CIRCUIT) {
    const qfs_template *ct = target->circuit;
    if (!ct || ct->n_qubits != n || ct->n_gates < 0 || (ct->n_gates > 0 && (!ct->pairs || !target->circuit_gates))) {
      set_error_detail("qudits: a circuit target needs a template on the same qudits and its gates");
      return QFS_EINVAL;
    }
    for (int k = 0; k < ct->n_gates; ++k) {
      const int a = ct->pairs[2 * k], b = ct->pairs[2 * k + 1];
      if (a < 0 || b < 0 || a >= n || b >= n || a == b) {
        set_error_detail("qudits: target gate " + std::to_string(k) + " has an invalid qudit pair");
        return QFS_EINVAL;
      }
    }
  } else {
    set_error_detail("qudits: unknown target kind");
    return QFS_EINVAL;
  }
  data.tgt = target;
  data.seed = params->seed;
  data.m_val = params->m_val;
  return qd_instantiate_impl(d, tmpl, data, *params, gates_in, gates_out, res, t0);
}

}  // namespace
}  // namespace qfs

using namespace qfs;

extern "C" {

int qfs_qudit_instantiate(int32_t d, const qfs_template *tmpl, const qfs_c128 *psi, const qfs_c128 *phi,
                          int32_t n_samples, int32_t n_val, const qfs_params *params,
                          const qfs_c128 *gates_in, qfs_c128 *gates_out, qfs_result *res) {
  qfs_target t{};
  t.kind = QFS_TARGET_SAMPLES;
  t.psi = psi;
  t.phi = phi;
  t.n_samples = n_samples;
  t.n_val = n_val;
  return qd_entry(d, tmpl, &t, params, gates_in, gates_out, res, false);
}

int qfs_qudit_instantiate_target(int32_t d, const qfs_template *tmpl, const qfs_target *target,
                                 const qfs_params *params, const qfs_c128 *gates_in, qfs_c128 *gates_out,
                                 qfs_result *res) {
  return qd_entry(d, tmpl, target, params, gates_in, gates_out, res, false);
}

int qfs_qudit_instantiate_batch(int32_t d, int32_t P, const qfs_template *tmpls, const qfs_target *targets,
                                const qfs_params *params, qfs_c128 *const *gates_out, qfs_result *res) {
  if (P < 1 || !tmpls || !targets || !params || !gates_out || !res) {
    set_error_detail("qudits batch: need P >= 1 and every array");
    return QFS_EINVAL;
  }
  int dev = 0;
  QFS_HIP(hipGetDevice(&dev));
  // the caller's stream first: work it holds for the inputs comes before the problems
  QFS_HIP(hipStreamSynchronize(static_cast<hipStream_t>(params->hip_stream)));
  const int W = std::min<int>(P, kQdBatchStreams);
  std::atomic<int> next{0};
  std::vector<int> rc(W, QFS_OK);
  std::vector<std::string> detail(W);
  auto worker = [&](int w) {
    hipStream_t st = nullptr;
    if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      rc[w] = QFS_EDEVICE;
      detail[w] = "qudits batch: no stream for a worker";
      return;
    }
    qfs_params q = *params;
    q.hip_stream = st;
    for (int i = next.fetch_add(1); i < P; i = next.fetch_add(1)) {
      const int r = qd_entry(d, &tmpls[i], &targets[i], &q, nullptr, gates_out[i], &res[i], true);
      if (r != QFS_OK) {
        rc[w] = r;
        detail[w] = "problem " + std::to_string(i) + ": " + qfs_last_error_detail();
        next.store(P);  // no new problems once one has failed
        break;
      }
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < W; ++w) pool.emplace_back(worker, w);
  for (auto &t : pool) t.join();
  for (int w = 0; w < W; ++w)
    if (rc[w] != QFS_OK) {
      set_error_detail(detail[w]);
      return rc[w];
    }
  return QFS_OK;
}

int qfs_qudit_sweep(int32_t d, int32_t n, int32_t L, const int32_t *pairs, const int32_t *kinds, int32_t M,
                    const qfs_c128 *psi, const qfs_c128 *phi, int32_t starts, qfs_c128 *gates, int32_t precision,
                    double beta, double *c_train, void *hip_stream) {
  qfs_template t{n, L, pairs, kinds, nullptr};
  QFS_TRY(qd_validate(d, &t));
  const int64_t N = qd_pow(d, n);
  if (M < 1 || M > N || starts < 1 || !psi || !phi || !gates || !c_train ||
      (precision != QFS_PREC_FP64 && precision != QFS_PREC_MIXED) || !(beta >= 0 && beta <= 1)) {
    set_error_detail("qudits: bad sweep arguments");
    return QFS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::vector<int> all(starts);
  for (int s = 0; s < starts; ++s) all[s] = s;
  const int D = d * d;
  DevBuf vst;
  QFS_TRY(vst.alloc(sizeof(c128) * (size_t)starts * L * D * D));
  hipLaunchKernelGGL(k_qd_identity, dim3(qd_grid((int64_t)starts * L * D * D)), dim3(kQdBlock), 0, st,
                     (int64_t)starts * L, D, vst.as<c128>());
  QFS_HIP(hipGetLastError());
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    QdSweeper<R> w;
    w.d = d;
    w.n = n;
    w.L = L;
    w.S = starts;
    w.N = N;
    w.pairs = pairs;
    w.kinds = kinds;
    w.st = st;
    w.g64 = reinterpret_cast<c128 *>(gates);
    w.vst = vst.as<c128>();
    w.beta = beta;
    QFS_TRY(w.alloc(M, 0));
    QFS_TRY(qd_load_sets<R>(w, psi, phi, M, 0));
    QFS_TRY(w.set_slots(all));
    QFS_TRY(w.forward(false));
    QFS_TRY(w.backward());
    QFS_HIP(hipMemcpyAsync(c_train, w.costs.ptr, sizeof(double) * starts, hipMemcpyDeviceToHost, st));
    QFS_HIP(hipStreamSynchronize(st));
    return QFS_OK;
  };
  return precision == QFS_PREC_MIXED ? run(float{}) : run(double{});
}

}  // extern "C"
