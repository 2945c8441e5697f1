// Batched QFactor-Sample: thousands of small instantiation problems x multistarts in
// persistent launches (one work-group per (problem, start) job, jobs pulled from a
// device work queue, longest first).
//
// Per job the two working state sets live in LDS when they fit (else in a per-work-group
// global scratch slot): the forward pass runs Psi through the gates in place, and the
// backward pass recovers each intermediate state B_k = u_k^dag B_{k+1} with the gate as
// it was before the sweep (gate k is updated only after its environment is reduced),
// so no B list is stored. The paper's per-sweep steps are unchanged (Sec. 3, Fig.
// pre-comp, Fig. env_calc_tensor); the control decisions of App. A run on the device
// after every sweep; doublings and the complex128 refinement switch are applied by the
// host between launches.
#include <algorithm>

#include "batch.h"
#include "philox.h"
#include "polar2.h"

namespace qfs {

namespace {

template <typename R>
__device__ __forceinline__ R bwave_sum(R x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ uint32_t deposit2(uint32_t r, int lo, int hi) {
  r = ((r >> lo) << (lo + 1)) | (r & ((1u << lo) - 1u));
  r = ((r >> hi) << (hi + 1)) | (r & ((1u << hi) - 1u));
  return r;
}

// Wave sums of the 16 complex entries of a 4x4 environment (32 reals, FP64) by recursive
// halving: at the exchange with lane ^ 2C each lane keeps half of its values (the upper
// half when that lane bit is set) and adds its partner's copy of that half; a last
// exchange with lane ^ 1 completes the sums. Lane l returns the wave sum of real value
// l >> 1 (value 2e is entry e's real part, 2e + 1 its imaginary part).
template <int C>
__device__ __forceinline__ void bhalve(double (&v)[32], int lane) {
  const bool hi = (lane & (2 * C)) != 0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const double give = hi ? v[i] : v[C + i];
    const double keep = hi ? v[C + i] : v[i];
    v[i] = keep + __shfl_xor(give, 2 * C);
  }
}
template <typename R>
__device__ __forceinline__ double bwave_sum_env(const cx<R> (&acc)[16]) {
  const int lane = threadIdx.x & 63;
  double v[32];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    v[2 * e] = (double)acc[e].re;
    v[2 * e + 1] = (double)acc[e].im;
  }
  bhalve<16>(v, lane);
  bhalve<8>(v, lane);
  bhalve<4>(v, lane);
  bhalve<2>(v, lane);
  bhalve<1>(v, lane);
  return v[0] + __shfl_xor(v[0], 1);
}

// Sum over the work-group; result valid in every thread. `red` holds NT/64 values.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double *red) {
  x = bwave_sum<double>(x);
  if (NT == 64) return x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

// Apply u (or u^dagger) of qubit bit positions (pa, pb) to `rows` states of N amplitudes
// stored contiguously ([rows][N]) in `st`.
template <typename R, int NT>
__device__ __forceinline__ void apply_states(cx<R> *st, int rows, int n, int pa, int pb,
                                             const cx<R> *u, bool dagger) {
  cx<R> m[16];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) m[q * 4 + p] = dagger ? cconj(u[p * 4 + q]) : u[q * 4 + p];
  const int lo = min(pa, pb), hi = max(pa, pb);
  const uint32_t ma = 1u << pa, mb = 1u << pb;
  const uint32_t gper = 1u << (n - 2);
  const uint32_t total = gper * rows;
  // two groups per iteration: both groups' loads are issued before any store, which
  // doubles the memory accesses in flight when the states live in global scratch
  for (uint32_t g0 = threadIdx.x; g0 < total; g0 += 2 * NT) {
    cx<R> x[2][4];
    cx<R> *sp[2];
    uint32_t o[2][4];
    const bool two = g0 + NT < total;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t g = h ? (two ? g0 + NT : g0) : g0;
      const uint32_t j = g >> (n - 2), r = g & (gper - 1u);
      sp[h] = st + ((size_t)j << n);
      const uint32_t i0 = deposit2(r, lo, hi);
      o[h][0] = i0;
      o[h][1] = i0 + mb;
      o[h][2] = i0 + ma;
      o[h][3] = i0 + ma + mb;
#pragma unroll
      for (int p = 0; p < 4; ++p) x[h][p] = sp[h][o[h][p]];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !two) break;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cx<R> y = cmake<R>(0, 0);
#pragma unroll
        for (int p = 0; p < 4; ++p) cfma(y, m[q * 4 + p], x[h][p]);
        sp[h][o[h][q]] = y;
      }
    }
  }
}

// Load `rows` FP64 states [rows][N] from global into R precision.
template <typename R, int NT>
__device__ __forceinline__ void load_states(cx<R> *dst, const c128 *src, int rows, int n) {
  const uint32_t total = (uint32_t)rows << n;
  for (uint32_t e = threadIdx.x; e < total; e += NT) {
    const c128 v = src[e];
    dst[e] = cmake<R>((R)v.re, (R)v.im);
  }
}

// (1/rows) sum |x - ref|^2 with ref FP64 in global; every thread gets the result.
template <typename R, int NT>
__device__ __forceinline__ double dist_states(const cx<R> *x, const c128 *ref, int rows, int n,
                                              double *red) {
  const uint32_t total = (uint32_t)rows << n;
  double acc = 0.0;
  for (uint32_t e = threadIdx.x; e < total; e += NT) {
    const c128 r = ref[e];
    const double dr = (double)x[e].re - r.re, di = (double)x[e].im - r.im;
    acc += dr * dr + di * di;
  }
  return block_sum<NT>(acc, red) / (double)rows;
}

// ------------------------------------------------------------------ polar (one wave)
// Same one-sided Jacobi as the plain path: lane 4c + r holds column c, row r.
__device__ __forceinline__ c128 bshfl_c(c128 x, int src) {
  return cmake(__shfl(x.re, src), __shfl(x.im, src));
}
__device__ __forceinline__ c128 bquad_sum(c128 x) {
  x.re += __shfl_xor(x.re, 1);
  x.im += __shfl_xor(x.im, 1);
  x.re += __shfl_xor(x.re, 2);
  x.im += __shfl_xor(x.im, 2);
  return x;
}

// u <- polar((1 - beta) G + beta u), warm-started from vst (updated). Writes u64 (global)
// and u_r (R copy, LDS). Falls back to a serial completion on lane 0 when a singular
// value vanishes. Called by the 64 lanes of one wave.
template <typename R>
__device__ __forceinline__ void batch_polar(const c128 *G, double beta, c128 *u64, cx<R> *u_r, c128 *vst,
                            c128 *lds_g, c128 *lds_v, double *lds_s) {
  const int lane = threadIdx.x & 63;
  const int l = lane & 15, c = l >> 2, r = l & 3, base = lane & ~15;
  auto gm = [&](int row, int col) {
    c128 x = G[row * 4 + col];
    if (beta != 0.0) {
      const c128 up = u64[row * 4 + col];
      x = cmake((1.0 - beta) * x.re + beta * up.re, (1.0 - beta) * x.im + beta * up.im);
    }
    return x;
  };
  // warm start: V_prev made unitary by one Newton-Schulz step, G <- G V_prev
  const c128 x = vst[r * 4 + c];
  c128 acc = cmake(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const c128 xra = bshfl_c(x, base + 4 * a + r);
    cfma(acc, xra, bquad_sum(cconj(xra) * x));
  }
  c128 v = cmake(0.5 * (3.0 * x.re - acc.re), 0.5 * (3.0 * x.im - acc.im));
  c128 g = cmake(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) cfma(g, gm(r, k), bshfl_c(v, base + 4 * c + k));
  bool converged = false;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rotated = 0;
#pragma unroll
    for (int m = 4; m <= 12; m += 4) {
      const c128 go = cmake(__shfl_xor(g.re, m), __shfl_xor(g.im, m));
      const c128 vo = cmake(__shfl_xor(v.re, m), __shfl_xor(v.im, m));
      const bool is_p = (l ^ m) > l;
      const c128 gp = is_p ? g : go, gq = is_p ? go : g;
      const c128 vp = is_p ? v : vo, vq = is_p ? vo : v;
      double al = cabs2(gp), be = cabs2(gq);
      double gr = gp.re * gq.re + gp.im * gq.im;
      double gi = gp.re * gq.im - gp.im * gq.re;
#pragma unroll
      for (int o = 1; o <= 2; o <<= 1) {
        al += __shfl_xor(al, o);
        be += __shfl_xor(be, o);
        gr += __shfl_xor(gr, o);
        gi += __shfl_xor(gi, o);
      }
      const double ag = sqrt(gr * gr + gi * gi);
      if (ag > 0.0 && ag > 1e-15 * sqrt(al * be)) {
        rotated = 1;
        const c128 ec = cmake(gr / ag, -gi / ag);
        const double tau = (be - al) / (2.0 * ag);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
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
    if (!__any(rotated)) {
      converged = true;
      break;
    }
  }
  double s2 = cabs2(g);
  s2 += __shfl_xor(s2, 1);
  s2 += __shfl_xor(s2, 2);
  const double sig = sqrt(s2);
  double smin = fmin(sig, __shfl_xor(sig, 4)), smax = fmax(sig, __shfl_xor(sig, 4));
  smin = fmin(smin, __shfl_xor(smin, 8));
  smax = fmax(smax, __shfl_xor(smax, 8));
  if (converged && smin > 1e-200 && smin > 1e-15 * smax) {
    const c128 w = cscale(g, 1.0 / sig);
    const int q = l >> 2, p = l & 3;
    c128 u = cmake(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) cfma_conj(u, bshfl_c(w, base + 4 * k + q), bshfl_c(v, base + 4 * k + p));
    if (lane < 16) {
      u64[l] = u;
      u_r[l] = cmake<R>((R)u.re, (R)u.im);
      vst[r * 4 + c] = v;
    }
    return;
  }
  if (lane < 16) {
    lds_g[c * 4 + r] = g;
    lds_v[c * 4 + r] = v;
    if (r == 0) lds_s[c] = sig;
    vst[r * 4 + c] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
    int ord[4] = {0, 1, 2, 3};
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (lds_s[ord[b]] > lds_s[ord[a]]) {
          const int t = ord[a];
          ord[a] = ord[b];
          ord[b] = t;
        }
    const double sm = lds_s[ord[0]];
    c128 w[4][4];
    for (int k = 0; k < 4; ++k) {
      const int cc = ord[k];
      const double sk = lds_s[cc];
      c128 xx[4];
      bool ok = sk > 0.0 && sk > 1e-13 * sm;
      if (ok) {
        for (int rr = 0; rr < 4; ++rr) xx[rr] = cscale(lds_g[cc * 4 + rr], 1.0 / sk);
        for (int rep = 0; rep < 2; ++rep)
          for (int o = 0; o < k; ++o) {
            c128 d = cmake(0.0, 0.0);
            for (int rr = 0; rr < 4; ++rr) cfma(d, cconj(w[o][rr]), xx[rr]);
            for (int rr = 0; rr < 4; ++rr) xx[rr] = xx[rr] - d * w[o][rr];
          }
        double nn = 0.0;
        for (int rr = 0; rr < 4; ++rr) nn += cabs2(xx[rr]);
        nn = sqrt(nn);
        if (nn > 0.5)
          for (int rr = 0; rr < 4; ++rr) xx[rr] = cscale(xx[rr], 1.0 / nn);
        else
          ok = false;
      }
      if (!ok) {
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
        for (int rr = 0; rr < 4; ++rr) xx[rr] = cscale(bx[rr], inv);
      }
      for (int rr = 0; rr < 4; ++rr) w[k][rr] = xx[rr];
    }
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < 4; ++p) {
        c128 u = cmake(0.0, 0.0);
        for (int k = 0; k < 4; ++k) cfma_conj(u, w[k][q], lds_v[ord[k] * 4 + p]);
        u64[q * 4 + p] = u;
        u_r[q * 4 + p] = cmake<R>((R)u.re, (R)u.im);
      }
  }
}

// ------------------------------------------------------------------ job sweeps
template <int NW>
struct SweepShared {
  c128 wred[NW][16];
  c128 gam[16];
  c128 pg[16], pv[16];
  double ps[4];
  double red[NW];
  int flag;   // control decision after a sweep
  int pause;  // pause at the top of a sweep (a separate word: waves may still be reading
              // flag from the previous sweep's decision when thread 0 writes this one)
};

// Jobs with at most kGatesInLds gates keep all their gates (state precision) in LDS for
// the whole launch; longer templates stage one gate at a time from the FP64 masters.
constexpr int kGatesInLds = 24;

template <typename R, int NT>
__device__ void run_job(const BatchArgs &A, int jid, cx<R> *bufA, cx<R> *bufB,
                        SweepShared<NT / 64> &sh, cx<R> *gl, cx<R> *gates_l) {
  BJob &J = A.jobs[jid];
  BProb &P = A.probs[J.prob];
  const int n = P.n, L = P.L, M = P.M, Mv = P.Mv;
  const int32_t *pairs = P.pairs;
  c128 *g64 = P.g64 + (size_t)J.start * L * 16;
  c128 *vst = P.vst + (size_t)J.start * L * 16;
  const BParams &hp = A.hp;
  const double beta = effective_beta(hp.beta, hp.beta_normalized != 0, M);

  // gate k of this job in R precision: resident in LDS (short templates), or staged
  // from the FP64 master into the slot gl
  const bool resident = L <= kGatesInLds;
  if (resident) {
    for (int e = threadIdx.x; e < L * 16; e += NT) {
      const c128 u = g64[e];
      gates_l[e] = cmake<R>((R)u.re, (R)u.im);
    }
    __syncthreads();
  }
  auto gate = [&](int k) -> const cx<R> * {
    if (resident) return gates_l + k * 16;
    if (threadIdx.x < 16) {
      const c128 u = g64[k * 16 + threadIdx.x];
      gl[threadIdx.x] = cmake<R>((R)u.re, (R)u.im);
    }
    __syncthreads();
    return gl;
  };
  // forward: bufB <- C Psi (training), bufA <- C Psi_val; returns c_val; c0 optional
  auto forward = [&](double *c0) {
    load_states<R, NT>(bufB, P.psi, M, n);
    if (Mv > 0) load_states<R, NT>(bufA, P.psiv, Mv, n);
    // the loads fill one element per thread while a gate reads groups of four written by
    // other waves (and gate(k) returns without a barrier when the gates are resident)
    __syncthreads();
    for (int k = 0; k < L; ++k) {
      const cx<R> *u = gate(k);
      const int pa = n - 1 - pairs[2 * k], pb = n - 1 - pairs[2 * k + 1];
      apply_states<R, NT>(bufB, M, n, pa, pb, u, false);
      if (Mv > 0) apply_states<R, NT>(bufA, Mv, n, pa, pb, u, false);
      __syncthreads();
    }
    if (c0) *c0 = dist_states<R, NT>(bufB, P.phi, M, n, sh.red);
    return Mv > 0 ? dist_states<R, NT>(bufA, P.phiv, Mv, n, sh.red) : -1.0;
  };

  const int Kmax = A.sweeps_per_launch;
  double c0 = 0.0;
  // read once: thread 0 clears the flag below, and every wave must take the same branch
  // to the barrier inside it
  const bool need_c0 = J.need_c0 != 0;
  double cval = forward(need_c0 ? &c0 : nullptr);
  if (need_c0) {
    if (threadIdx.x == 0) {
      J.c_prev = c0;
      J.c_train = c0;
      J.c_val = Mv > 0 ? cval : c0;
      J.need_c0 = 0;
    }
    __syncthreads();
  }
  for (int sw = 0; sw < Kmax; ++sw) {
    // stop at a sweep boundary the problem already decided on
    if (threadIdx.x == 0) {
      const int ds = __hip_atomic_load(&P.done_sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int os = __hip_atomic_load(&P.over_sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh.pause = (!hp.independent && (J.total >= ds || J.total >= os)) ? 1 : 0;
    }
    __syncthreads();
    if (sh.pause) {
      if (threadIdx.x == 0) J.status = BJ_PAUSED;
      return;
    }
    // ---- backward (right to left), bufB holds C Psi on entry
    load_states<R, NT>(bufA, P.phi, M, n);
    __syncthreads();
    for (int k = L - 1; k >= 0; --k) {
      const int pa = n - 1 - pairs[2 * k], pb = n - 1 - pairs[2 * k + 1];
      const int kind = P.kinds ? P.kinds[k] : QFS_GATE_2Q;
      if (k < L - 1) {
        const cx<R> *u1 = gate(k + 1);  // already updated
        const int qa = n - 1 - pairs[2 * (k + 1)], qb = n - 1 - pairs[2 * (k + 1) + 1];
        apply_states<R, NT>(bufA, M, n, qa, qb, u1, true);
        __syncthreads();
      }
      const cx<R> *u0 = gate(k);  // not yet updated
      apply_states<R, NT>(bufB, M, n, pa, pb, u0, true);  // B_k
      __syncthreads();
      if (kind == QFS_GATE_FIXED) continue;  // applied only, no environment
      // environment of gate k
      cx<R> acc[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = cmake<R>(0, 0);
      const int lo = min(pa, pb), hi = max(pa, pb);
      const uint32_t ma = 1u << pa, mb = 1u << pb, gper = 1u << (n - 2);
      for (uint32_t gi = threadIdx.x; gi < gper * M; gi += NT) {
        const uint32_t j = gi >> (n - 2), rr = gi & (gper - 1u);
        const uint32_t i0 = deposit2(rr, lo, hi);
        const uint32_t o[4] = {i0, i0 + mb, i0 + ma, i0 + ma + mb};
        const cx<R> *sa = bufA + ((size_t)j << n), *sb = bufB + ((size_t)j << n);
        cx<R> av[4], bv[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          av[p] = sa[o[p]];
          bv[p] = sb[o[p]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int p = 0; p < 4; ++p) cfma_conj(acc[q * 4 + p], av[q], bv[p]);
      }
      const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
      {
        const double ws = bwave_sum_env<R>(acc);
        // (value 2e + part lands on the real or imaginary half of entry e)
        if ((lane & 1) == 0) reinterpret_cast<double *>(&sh.wred[w][0])[lane >> 1] = ws;
      }
      __syncthreads();
      if (threadIdx.x < 16) {
        c128 t = sh.wred[0][threadIdx.x];
        for (int ww = 1; ww < NT / 64; ++ww) t = t + sh.wred[ww][threadIdx.x];
        sh.gam[threadIdx.x] = t;
      }
      __syncthreads();
      // the new gate k goes to the FP64 master and (state precision) to its LDS slot;
      // the old one has served its last use (B_k above)
      cx<R> *unew = resident ? gates_l + k * 16 : gl;
      if (kind == QFS_GATE_1Q) {
        if (threadIdx.x == 0) polar2_update<R>(sh.gam, beta, g64 + k * 16, unew);
      } else if (threadIdx.x < 64) {
        batch_polar<R>(sh.gam, beta, g64 + k * 16, unew, vst + k * 16, sh.pg, sh.pv, sh.ps);
      }
      __syncthreads();
    }
    // cost of the updated gates: a_0 = u_0^dag a
    {
      const int pa = n - 1 - pairs[0], pb = n - 1 - pairs[1];
      apply_states<R, NT>(bufA, M, n, pa, pb, resident ? gates_l : gl, true);  // the new u_0
      __syncthreads();
    }
    const double ct = dist_states<R, NT>(bufA, P.psi, M, n, sh.red);
    __syncthreads();
    cval = forward(nullptr);
    // ---- control (App. A), one thread
    if (threadIdx.x == 0) {
      const double cv = Mv > 0 ? cval : ct;
      J.iter += 1;
      J.total += 1;
      J.work += (double)(M + Mv) * (double)(1u << n) * (double)L;
      const bool improved = fabs(J.c_prev) - fabs(ct) > hp.diff_tol_r * fabs(ct);
      J.z = improved ? 0 : J.z + 1;
      J.c_prev = ct;
      J.c_train = ct;
      J.c_val = cv;
      const bool gen_ok = P.full || Mv == 0 || cv <= (1.0 + hp.overtrain_ratio) * ct;
      int st = BJ_RUN;
      if (ct < hp.dist_tol && gen_ok) {
        st = BJ_SUCCESS;
        __hip_atomic_fetch_min(&P.done_sweep, J.total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (J.iter >= hp.min_iter && !gen_ok && M < P.mcap) {
        st = BJ_OVER;
        __hip_atomic_fetch_min(&P.over_sweep, J.total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (J.iter >= hp.min_iter && !gen_ok && ct < hp.dist_tol) {
        st = BJ_NOT_GEN;
      } else if (J.iter >= hp.min_iter && J.z >= hp.plateau_window) {
        st = BJ_PLATEAU;
      } else if (J.total >= hp.max_iter) {
        st = BJ_MAX_ITER;
      } else if (sizeof(R) == 4 && hp.mixed && ct < hp.refine_below) {
        st = BJ_REFINE;
      }
      J.status = st;
      sh.flag = st;
    }
    __syncthreads();
    if (sh.flag != BJ_RUN) return;
  }
}

template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_batch_sweep(BatchArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ SweepShared<NT / 64> sh;
  __shared__ int qi_s;
  __shared__ __align__(16) cx<R> gl[16];
  __shared__ __align__(16) cx<R> gates_l[kGatesInLds * 16];
  cx<R> *lds = reinterpret_cast<cx<R> *>(lds_raw);
  for (;;) {
    if (threadIdx.x == 0) qi_s = atomicAdd(A.queue_head, 1);
    __syncthreads();
    const int qi = qi_s;
    __syncthreads();
    if (qi >= A.njobs) break;
    const int jid = A.queue[qi];
    const BProb &P = A.probs[A.jobs[jid].prob];
    const size_t rowsA = (size_t)max(P.M, P.Mv) << P.n, rowsB = (size_t)P.M << P.n;
    cx<R> *bufA, *bufB;
    if (A.scratch) {  // states in this work-group's global slot
      cx<R> *slot = reinterpret_cast<cx<R> *>(A.scratch + (size_t)blockIdx.x * A.scratch_slot_bytes);
      bufA = slot;
      bufB = slot + rowsA;
    } else {
      bufA = lds;
      bufB = lds + rowsA;
    }
    (void)rowsB;
    run_job<R, NT>(A, jid, bufA, bufB, sh, gl, gates_l);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ per-problem setup
// One work-group per problem: training columns [m0, m1) of the Ginibre stream
// (role 1, stream 0, index j N + i) orthonormalised against all previous columns by
// classical Gram-Schmidt with one re-orthogonalisation pass (the unique QR with positive
// diag R), U psi for them; and, when val_gen >= 0, a fresh validation set (role 2,
// stream val_gen) with its U psi. All FP64, states [M][N] in global memory.

__device__ void orth_columns(c128 *Q, int n, int c0, int c1, double *red, c128 *coef) {
  const int N = 1 << n;
  for (int j = c0; j < c1; ++j) {
    c128 *v = Q + ((size_t)j << n);
    for (int pass = 0; pass < 2; ++pass) {
      // coef[k] = <q_k, v>, k < j (one thread per k)
      for (int k = threadIdx.x; k < j; k += blockDim.x) {
        const c128 *q = Q + ((size_t)k << n);
        c128 d = cmake(0.0, 0.0);
        for (int i = 0; i < N; ++i) cfma(d, cconj(q[i]), v[i]);
        coef[k] = d;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        c128 x = v[i];
        for (int k = 0; k < j; ++k) x = x - coef[k] * Q[((size_t)k << n) + i];
        v[i] = x;
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) s += cabs2(v[i]);
    s = bwave_sum<double>(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
    const double inv = 1.0 / sqrt(tot);
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) v[i] = cscale(v[i], inv);
    __syncthreads();
  }
}

__device__ void target_columns(const BProb &P, const c128 *psi, c128 *phi, int c0, int c1) {
  const int n = P.n, N = 1 << n;
  if (P.kind == QFS_TARGET_DENSE) {
    for (uint32_t e = threadIdx.x; e < (uint32_t)(c1 - c0) * N; e += blockDim.x) {
      const int j = c0 + (int)(e >> n), row = (int)(e & (N - 1));
      c128 acc = cmake(0.0, 0.0);
      for (int col = 0; col < N; ++col) cfma(acc, P.U[(size_t)row * N + col], psi[((size_t)j << n) + col]);
      phi[((size_t)j << n) + row] = acc;
    }
    __syncthreads();
    return;
  }
  for (uint32_t e = threadIdx.x; e < (uint32_t)(c1 - c0) * N; e += blockDim.x)
    phi[((size_t)c0 << n) + e] = psi[((size_t)c0 << n) + e];
  __syncthreads();
  for (int k = 0; k < P.Lt; ++k) {
    const int pa = n - 1 - P.tpairs[2 * k], pb = n - 1 - P.tpairs[2 * k + 1];
    const c128 *u = P.tgates + (size_t)k * 16;
    const int lo = min(pa, pb), hi = max(pa, pb);
    const uint32_t ma = 1u << pa, mb = 1u << pb, gper = 1u << (n - 2);
    for (uint32_t g = threadIdx.x; g < gper * (uint32_t)(c1 - c0); g += blockDim.x) {
      const uint32_t j = c0 + (g >> (n - 2)), r = g & (gper - 1u);
      c128 *s = phi + ((size_t)j << n);
      const uint32_t i0 = deposit2(r, lo, hi);
      const uint32_t o[4] = {i0, i0 + mb, i0 + ma, i0 + ma + mb};
      c128 x[4];
      for (int p = 0; p < 4; ++p) x[p] = s[o[p]];
      for (int q = 0; q < 4; ++q) {
        c128 y = cmake(0.0, 0.0);
        for (int p = 0; p < 4; ++p) cfma(y, u[q * 4 + p], x[p]);
        s[o[q]] = y;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_batch_setup(BProb *probs, const int32_t *todo, int ntodo,
                                                     const int32_t *m0s, uint64_t seed_base) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  if (t >= ntodo) return;
  BProb &P = probs[todo[t]];
  const int n = P.n, N = 1 << n;
  const int m0 = m0s[t], m1 = P.M;
  c128 *coef = P.coef;
  if (P.kind == QFS_TARGET_SAMPLES) {
    for (uint32_t e = threadIdx.x; e < (uint32_t)(m1 - m0) * N; e += blockDim.x) {
      const size_t o = ((size_t)m0 << n) + e;
      P.psi[o] = P.s_psi[o];
      P.phi[o] = P.s_phi[o];
    }
    if (m0 == 0)
      for (uint32_t e = threadIdx.x; e < (uint32_t)P.Mv * N; e += blockDim.x) {
        P.psiv[e] = P.s_psi[((size_t)P.n_train << n) + e];
        P.phiv[e] = P.s_phi[((size_t)P.n_train << n) + e];
      }
    __syncthreads();
    return;
  }
  for (uint32_t e = threadIdx.x; e < (uint32_t)(m1 - m0) * N; e += blockDim.x) {
    const int j = m0 + (int)(e >> n), i = (int)(e & (N - 1));
    P.psi[((size_t)j << n) + i] = complex_normal(P.seed, 1u, 0u, (uint64_t)j * N + i);
  }
  __syncthreads();
  orth_columns(P.psi, n, m0, m1, red, coef);
  target_columns(P, P.psi, P.phi, m0, m1);
  if (P.Mv > 0) {
    for (uint32_t e = threadIdx.x; e < (uint32_t)P.Mv * N; e += blockDim.x) {
      const int j = (int)(e >> n), i = (int)(e & (N - 1));
      P.psiv[((size_t)j << n) + i] = complex_normal(P.seed, 2u, (uint32_t)P.generation, (uint64_t)j * N + i);
    }
    __syncthreads();
    orth_columns(P.psiv, n, 0, P.Mv, red, coef);
    target_columns(P, P.psiv, P.phiv, 0, P.Mv);
  }
  (void)seed_base;
}

// Haar 4x4 per (problem, start, gate), role 3, stream = start, index 16 gate + 4 col + row.
__global__ void k_batch_gates(BProb *probs, const int32_t *prob_of, const int32_t *first_gate,
                              int total) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int pidx = prob_of[t];
  const BProb &P = probs[pidx];
  const int local = t - first_gate[pidx];
  const int s = local / P.L, k = local % P.L;
  const int kind = P.kinds ? P.kinds[k] : QFS_GATE_2Q;
  c128 *u = P.g64 + ((size_t)s * P.L + k) * 16;
  c128 *v = P.vst + ((size_t)s * P.L + k) * 16;
  for (int e = 0; e < 16; ++e) v[e] = cmake((e % 5 == 0) ? 1.0 : 0.0, 0.0);
  if (kind == QFS_GATE_FIXED) {
    for (int e = 0; e < 16; ++e) u[e] = P.fixed[(size_t)k * 16 + e];
    return;
  }
  if (kind == QFS_GATE_1Q) {
    // v (x) I_2 with v Haar on U(2) from indices 16 k + 2 col + row of the same stream
    c128 h[2][2];
    for (int c = 0; c < 2; ++c)
      for (int r = 0; r < 2; ++r) h[c][r] = complex_normal(P.seed, 3u, (uint32_t)s, (uint64_t)k * 16u + 2u * c + r);
    for (int c = 0; c < 2; ++c) {
      for (int rep = 0; rep < 2; ++rep)
        for (int o = 0; o < c; ++o) {
          const c128 d = cconj(h[o][0]) * h[c][0] + cconj(h[o][1]) * h[c][1];
          for (int r = 0; r < 2; ++r) h[c][r] = h[c][r] - d * h[o][r];
        }
      const double inv = 1.0 / sqrt(cabs2(h[c][0]) + cabs2(h[c][1]));
      for (int r = 0; r < 2; ++r) h[c][r] = cscale(h[c][r], inv);
    }
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) u[r * 4 + c] = ((r & 1) == (c & 1)) ? h[c >> 1][r >> 1] : cmake(0.0, 0.0);
    return;
  }
  c128 q[4][4];
  for (int c = 0; c < 4; ++c)
    for (int r = 0; r < 4; ++r) q[c][r] = complex_normal(P.seed, 3u, (uint32_t)s, (uint64_t)k * 16u + 4u * c + r);
  for (int c = 0; c < 4; ++c) {
    for (int rep = 0; rep < 2; ++rep)
      for (int o = 0; o < c; ++o) {
        c128 d = cmake(0.0, 0.0);
        for (int r = 0; r < 4; ++r) cfma(d, cconj(q[o][r]), q[c][r]);
        for (int r = 0; r < 4; ++r) q[c][r] = q[c][r] - d * q[o][r];
      }
    double nrm = 0.0;
    for (int r = 0; r < 4; ++r) nrm += cabs2(q[c][r]);
    const double inv = 1.0 / sqrt(nrm);
    for (int r = 0; r < 4; ++r) q[c][r] = cscale(q[c][r], inv);
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) u[r * 4 + c] = q[c][r];
}

}  // namespace

// ------------------------------------------------------------------ launchers
int launch_batch_setup(BProb *probs_dev, const int32_t *todo, int ntodo, const int32_t *m0s,
                       hipStream_t s) {
  if (ntodo <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_batch_setup, dim3(ntodo), dim3(256), 0, s, probs_dev, todo, ntodo, m0s, 0ull);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_batch_gates(BProb *probs_dev, const int32_t *prob_of, const int32_t *first_gate, int total,
                       hipStream_t s) {
  if (total <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_batch_gates, dim3((total + 127) / 128), dim3(128), 0, s, probs_dev, prob_of,
                     first_gate, total);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

template <typename R, int NT>
static int launch_sweep_t(const BatchArgs &a, int grid, size_t lds, hipStream_t s) {
  static size_t attr = 0;
  QFS_TRY(ensure_dynamic_lds(reinterpret_cast<const void *>(&k_batch_sweep<R, NT>), lds, &attr));
  hipLaunchKernelGGL((k_batch_sweep<R, NT>), dim3(grid), dim3(NT), lds, s, a);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_batch_sweep(const BatchArgs &a, bool fp64, int threads, int grid, size_t lds, hipStream_t s) {
  if (a.njobs <= 0) return QFS_OK;
  if (fp64) {
    switch (threads) {
      case 64: return launch_sweep_t<double, 64>(a, grid, lds, s);
      case 128: return launch_sweep_t<double, 128>(a, grid, lds, s);
      case 512: return launch_sweep_t<double, 512>(a, grid, lds, s);
      default: return launch_sweep_t<double, 256>(a, grid, lds, s);
    }
  }
  switch (threads) {
    case 64: return launch_sweep_t<float, 64>(a, grid, lds, s);
    case 128: return launch_sweep_t<float, 128>(a, grid, lds, s);
    case 512: return launch_sweep_t<float, 512>(a, grid, lds, s);
    default: return launch_sweep_t<float, 256>(a, grid, lds, s);
  }
}

}  // namespace qfs
