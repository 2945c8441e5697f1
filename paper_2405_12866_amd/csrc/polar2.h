// Update of a variable one-qubit gate, shared by the plain and the batched engines.
#pragma once

#include "qfs_internal.h"

namespace qfs {

// One-qubit gate update (one thread). The gate's slot holds v (x) I_2 on (a, spectator)
// and the 4x4 environment was reduced on that pair, so the 2x2 environment of v is its
// trace over the spectator: G1[q][p] = G[2q][2p] + G[2q+1][2p+1]. With X = (1 - beta) G1
// + beta v = W S V^dagger, the polar factor W V^dagger of a 2x2 matrix has the closed form
// (X + w adj(X)^dagger) / (s1 + s2), w = det X / |det X| (adj(X)^dagger scaled by w is
// W diag(s2, s1) V^dagger), and s1 + s2 is the Frobenius norm of the sum over sqrt 2. For
// a singular X any unit w gives a maximiser of Re Tr(X^dagger v) (w = 1 is taken); X = 0
// keeps v. The slot is rewritten as v (x) I_2 in FP64 (u64) and, when ur is given, in
// the state precision.
template <typename R>
__device__ inline void polar2_update(const c128 *G, double beta, c128 *u64, cx<R> *ur) {
  c128 x[4];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const c128 g1 = G[(2 * q) * 4 + 2 * p] + G[(2 * q + 1) * 4 + 2 * p + 1];
      x[q * 2 + p] = cscale(g1, 1.0 - beta) + cscale(u64[(2 * q) * 4 + 2 * p], beta);
    }
  const c128 det = x[0] * x[3] - x[1] * x[2];
  const double ad = sqrt(cabs2(det));
  const c128 w = ad > 0.0 ? cscale(det, 1.0 / ad) : cmake(1.0, 0.0);
  c128 y[4] = {x[0] + w * cconj(x[3]), x[1] - w * cconj(x[2]), x[2] - w * cconj(x[1]),
               x[3] + w * cconj(x[0])};
  const double nrm = sqrt((cabs2(y[0]) + cabs2(y[1]) + cabs2(y[2]) + cabs2(y[3])) * 0.5);
  if (!(nrm > 0.0)) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) y[e] = cscale(y[e], 1.0 / nrm);
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const c128 v = ((r & 1) == (c & 1)) ? y[(r >> 1) * 2 + (c >> 1)] : cmake(0.0, 0.0);
      u64[r * 4 + c] = v;
      if (ur) ur[r * 4 + c] = cmake<R>((R)v.re, (R)v.im);
    }
}

}  // namespace qfs
