// FP64 4x4 unitary polar factor on one wave, shared by the per-gate and the grouped
// backward passes (sweep.hip, group.hip).
#pragma once

#include "qfs_internal.h"

namespace qfs {

// ------------------------------------------------------------------ FP64 4x4 polar
// One-sided (Hestenes) Jacobi on one wave: lane l = 4c + r (of each 16-lane group)
// holds column c, row r of the working matrix G and of V. Each round rotates the two
// disjoint column pairs c <-> c ^ (m >> 2), m in {4, 8, 12}; the pair's Gram entries
// are summed over the four rows of a quad, so both columns' lanes compute bitwise
// equal rotations. Then W = normalised columns of G (re-orthonormalised and completed
// when a singular value is negligible) and u = W V^dagger.
//
// Warm start (vstore != nullptr): Jacobi starts from G V_prev and V_prev, the right
// singular vectors this gate had after its previous update (the environment changes
// little between sweeps), so it converges in one or two sweeps instead of ~6. V_prev is
// first made unitary to rounding by one Newton-Schulz step V (3I - V^dag V) / 2, so no
// error accumulates across sweeps; the new V is stored back. vstart, when given, holds a
// copy of the stored V_prev (in LDS) to read instead.
__device__ __forceinline__ c128 shfl_c(c128 x, int src) {
  return cmake(__shfl(x.re, src), __shfl(x.im, src));
}

// Exchange between the lanes of a 16-lane row by DPP moves (no trip through the LDS
// crossbar): lane i receives lane i ^ M's value, M in {1, 2, 4, 8, 12}. xor 1 and 2 are quad
// permutations, xor 8 the rotation of the row by 8, xor 4 the reversal of each half row
// followed by the reversal of each quad.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int M>
__device__ __forceinline__ double xor_lane(double x) {
  if constexpr (M == 1) {
    return dpp_move<0xB1>(x);  // quad_perm [1, 0, 3, 2]
  } else if constexpr (M == 2) {
    return dpp_move<0x4E>(x);  // quad_perm [2, 3, 0, 1]
  } else if constexpr (M == 8) {
    return dpp_move<0x128>(x);  // row_ror:8
  } else if constexpr (M == 4) {
    return dpp_move<0x1B>(dpp_move<0x141>(x));  // row_half_mirror, then quad_perm [3, 2, 1, 0]
  } else {
    static_assert(M == 12, "lane exchange within a row");
    return xor_lane<8>(xor_lane<4>(x));
  }
}

__device__ __forceinline__ c128 quad_sum(c128 x) {
  x.re += xor_lane<1>(x.re);
  x.im += xor_lane<1>(x.im);
  x.re += xor_lane<2>(x.re);
  x.im += xor_lane<2>(x.im);
  return x;
}

// 1/sqrt(x) and 1/x from the hardware estimates, each refined by two Newton steps (about
// one ulp; the rotations below need cs^2 + sn^2 = 1 and |e| = 1 to rounding, not the
// correctly rounded values, and the estimates shorten their dependent chain).
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// One round of the one-sided Jacobi below: the column pairs c <-> c ^ (M >> 2).
template <int M>
__device__ __forceinline__ void jacobi_round(int l, c128 &g, c128 &v, int &large) {
  const c128 go = cmake(xor_lane<M>(g.re), xor_lane<M>(g.im));
  const c128 vo = cmake(xor_lane<M>(v.re), xor_lane<M>(v.im));
  const bool is_p = (l ^ M) > l;
  const c128 gp = is_p ? g : go, gq = is_p ? go : g;
  const c128 vp = is_p ? v : vo, vq = is_p ? vo : v;
  double al = cabs2(gp), be = cabs2(gq);
  double gr = gp.re * gq.re + gp.im * gq.im;  // conj(gp) * gq
  double gi = gp.re * gq.im - gp.im * gq.re;
  al += xor_lane<1>(al);
  be += xor_lane<1>(be);
  gr += xor_lane<1>(gr);
  gi += xor_lane<1>(gi);
  al += xor_lane<2>(al);
  be += xor_lane<2>(be);
  gr += xor_lane<2>(gr);
  gi += xor_lane<2>(gi);
  // |Gram_pq|^2 against the product of the column norms squared: rotate when |Gram_pq| >
  // 1e-15 sqrt(al be), and count the round as large above 1e-7 sqrt(al be)
  const double x2 = gr * gr + gi * gi, ab = al * be;
  if (x2 > 1e-30 * ab) {
    large |= x2 > 1e-14 * ab;
    const double rag = rsq_nr(x2);  // 1 / |Gram_pq|
    const c128 ec = cmake(gr * rag, -gi * rag);  // conj(e^{i phi})
    const double tau = (be - al) * (0.5 * rag);
    const double t1 = fma(tau, tau, 1.0);
    const double tt = (tau >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(tau) + t1 * rsq_nr(t1));
    const double cs = rsq_nr(fma(tt, tt, 1.0)), sn = cs * tt;
    const c128 egq = ec * gq, evq = ec * vq;
    if (is_p) {
      g = cmake(cs * gp.re - sn * egq.re, cs * gp.im - sn * egq.im);
      v = cmake(cs * vp.re - sn * evq.re, cs * vp.im - sn * evq.im);
    } else {
      g = cmake(sn * gp.re + cs * egq.re, sn * gp.im + cs * egq.im);
      v = cmake(sn * vp.re + cs * evq.re, sn * vp.im + cs * evq.im);
    }
  }
}

__device__ __forceinline__ void polar4_wave(const c128 *G, double beta, const c128 *u_prev, c128 *out64,
                            c64 *out32, c128 *lds_g, c128 *lds_v, double *lds_s,
                            c128 *vstore = nullptr, const c128 *vstart = nullptr) {
  const int lane = threadIdx.x & 63;
  const int l = lane & 15, c = l >> 2, r = l & 3, base = lane & ~15;
  auto gm = [&](int row, int col) {
    c128 x = G[row * 4 + col];
    if (beta != 0.0) {
      const c128 up = u_prev[row * 4 + col];
      x = cmake((1.0 - beta) * x.re + beta * up.re, (1.0 - beta) * x.im + beta * up.im);
    }
    return x;
  };
  c128 g, v;
  if (vstore) {
    // lane 4c + r holds X[r][c]; Y[a][c] = sum_k conj(X[k][a]) X[k][c] (quad c);
    // Z[r][c] = (3 X[r][c] - sum_a X[r][a] Y[a][c]) / 2
    const c128 x = (vstart ? vstart : vstore)[r * 4 + c];
    c128 acc = cmake(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const c128 xca = shfl_c(x, base + 4 * a + r);  // X[r][a]
      const c128 yac = quad_sum(cconj(xca) * x);     // Y[a][c]
      cfma(acc, xca, yac);
    }
    v = cmake(0.5 * (3.0 * x.re - acc.re), 0.5 * (3.0 * x.im - acc.im));
    g = cmake(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) cfma(g, gm(r, k), shfl_c(v, base + 4 * c + k));  // (G V)[r][c]
  } else {
    g = gm(r, c);
    v = cmake(r == c ? 1.0 : 0.0, 0.0);
  }
  // Cyclic Jacobi converges quadratically: a sweep whose rotations all started from a
  // relative off-diagonal Gram entry below 1e-7 leaves them at the 1e-14 level, so the
  // iteration stops after it instead of running a further sweep that rotates nothing.
  bool converged = false;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int large = 0;
    jacobi_round<4>(l, g, v, large);
    jacobi_round<8>(l, g, v, large);
    jacobi_round<12>(l, g, v, large);
    if (!__any(large)) {
      converged = true;
      break;
    }
  }
  double s2 = cabs2(g);
  s2 += xor_lane<1>(s2);
  s2 += xor_lane<2>(s2);
  const double sig = sqrt(s2);
  double smin = sig, smax = sig;
  smin = fmin(smin, xor_lane<4>(smin));
  smin = fmin(smin, xor_lane<8>(smin));
  smax = fmax(smax, xor_lane<4>(smax));
  smax = fmax(smax, xor_lane<8>(smax));
  if (converged && smin > 1e-200 && smin > 1e-15 * smax) {
    // W = G diag(1/sigma) is unitary to the Jacobi tolerance; u = W V^dagger with
    // lane 4q + p computing u[q][p] = sum_k W[q][k] conj(V[p][k]); W[q][k] and V[p][k]
    // live on lanes 4k + q and 4k + p.
    const c128 w = cscale(g, 1.0 / sig);
    const int q = l >> 2, p = l & 3, base = lane & ~15;
    c128 acc = cmake(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int lw = base + 4 * k + q, lv = base + 4 * k + p;
      const c128 wk = cmake(__shfl(w.re, lw), __shfl(w.im, lw));
      const c128 vk = cmake(__shfl(v.re, lv), __shfl(v.im, lv));
      cfma_conj(acc, wk, vk);
    }
    if (lane < 16) {
      out64[l] = acc;
      if (out32) out32[l] = cmake<float>((float)acc.re, (float)acc.im);
      if (vstore) vstore[r * 4 + c] = v;
    }
    return;
  }
  // Rank-deficient (or unconverged) case: lane 0 orders the columns by singular value,
  // re-orthonormalises them and completes W with unit vectors where sigma vanishes.
  if (lane < 16) {
    lds_g[c * 4 + r] = g;
    lds_v[c * 4 + r] = v;
    if (r == 0) lds_s[c] = sig;
    if (vstore) vstore[r * 4 + c] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
    int ord[4] = {0, 1, 2, 3};
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (lds_s[ord[b]] > lds_s[ord[a]]) {
          const int tmp = ord[a];
          ord[a] = ord[b];
          ord[b] = tmp;
        }
    const double sm = lds_s[ord[0]];
    c128 w[4][4];  // [k][row]
    for (int k = 0; k < 4; ++k) {
      const int cc = ord[k];
      const double sk = lds_s[cc];
      c128 x[4];
      bool ok = sk > 0.0 && sk > 1e-13 * sm;
      if (ok) {
        for (int rr = 0; rr < 4; ++rr) x[rr] = cscale(lds_g[cc * 4 + rr], 1.0 / sk);
        for (int rep = 0; rep < 2; ++rep)
          for (int o = 0; o < k; ++o) {
            c128 d = cmake(0.0, 0.0);
            for (int rr = 0; rr < 4; ++rr) cfma(d, cconj(w[o][rr]), x[rr]);
            for (int rr = 0; rr < 4; ++rr) x[rr] = x[rr] - d * w[o][rr];
          }
        double nn = 0.0;
        for (int rr = 0; rr < 4; ++rr) nn += cabs2(x[rr]);
        nn = sqrt(nn);
        if (nn > 0.5)
          for (int rr = 0; rr < 4; ++rr) x[rr] = cscale(x[rr], 1.0 / nn);
        else
          ok = false;
      }
      if (!ok) {  // complete with the unit vector of largest orthogonal remainder
        double best = -1.0;
        c128 bx[4];
        for (int e = 0; e < 4; ++e) {
          c128 y[4];
          for (int rr = 0; rr < 4; ++rr) y[rr] = cmake(rr == e ? 1.0 : 0.0, 0.0);
          for (int rep = 0; rep < 2; ++rep)
            for (int o = 0; o < k; ++o) {
              c128 d = cmake(0.0, 0.0);
              for (int rr = 0; rr < 4; ++rr) cfma(d, cconj(w[o][rr]), y[rr]);
              for (int rr = 0; rr < 4; ++rr) y[rr] = y[rr] - d * w[o][rr];
            }
          double nn = 0.0;
          for (int rr = 0; rr < 4; ++rr) nn += cabs2(y[rr]);
          if (nn > best) {
            best = nn;
            for (int rr = 0; rr < 4; ++rr) bx[rr] = y[rr];
          }
        }
        const double inv = 1.0 / sqrt(best);
        for (int rr = 0; rr < 4; ++rr) x[rr] = cscale(bx[rr], inv);
      }
      for (int rr = 0; rr < 4; ++rr) w[k][rr] = x[rr];
    }
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < 4; ++p) {
        c128 acc = cmake(0.0, 0.0);
        for (int k = 0; k < 4; ++k) cfma_conj(acc, w[k][q], lds_v[ord[k] * 4 + p]);
        out64[q * 4 + p] = acc;
        if (out32) out32[q * 4 + p] = cmake<float>((float)acc.re, (float)acc.im);
      }
  }
}


}  // namespace qfs
