/*
 * qfs_oracle.c -- FP64 CPU oracle of QFactor-Sample instantiation (arXiv 2405.12866).
 *
 * TEST INFRASTRUCTURE ONLY (see qfs_oracle.h): plain loops in complex128, written from
 * the paper's description of the method, with no blocking, fusion or reordering beyond
 * what the method states. Each function names the passage it follows. Conventions are
 * listed in qfs_oracle.h.
 */
#include "qfs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define QO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------
 * Random numbers. The method draws its training states, validation states and initial
 * gates at random (Sec. 3; App. A "multistarts and seed"). The paper uses SciPy's
 * unitary_group; here the same Haar distribution is built from Philox4x32-10, written
 * from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with a
 * Weyl-sequence key schedule.
 * ---------------------------------------------------------------------------------- */
void qo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u; /* golden ratio */
    k1 += 0xBB67AE85u; /* sqrt(3) - 1  */
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One complex standard normal per Philox block, by the Box-Muller transform:
 * two 53-bit uniforms u1 in (0,1], u2 in [0,1); |z|^2 = -ln u1 is Exp(1), so E|z|^2 = 1,
 * and arg z = 2 pi u2 is uniform. */
qo_cplx qo_cgauss(uint64_t seed, uint32_t role, uint32_t stream, uint64_t idx) {
  uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), role, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  qo_philox4x32_10(ctr, key, w);
  uint64_t a = (((uint64_t)w[1] << 32) | w[0]) >> 11;
  uint64_t b = (((uint64_t)w[3] << 32) | w[2]) >> 11;
  double u1 = ((double)a + 1.0) * 0x1.0p-53;
  double u2 = (double)b * 0x1.0p-53;
  double r = sqrt(-log(u1));
  double t = 2.0 * QO_PI * u2;
  return r * cos(t) + I * (r * sin(t));
}

void qo_ginibre(int64_t rows, int64_t cols, uint64_t seed, uint32_t role, uint32_t stream,
                qo_cplx *out) {
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i)
      out[j * rows + i] = qo_cgauss(seed, role, stream, (uint64_t)(j * rows + i));
}

/* Column j of Q is the part of column j of A orthogonal to columns 0..j-1, normalised
 * to unit length: the Q of A = QR with diag(R) real and positive, which makes Q Haar
 * distributed for Ginibre A (Mezzadri, "How to generate random matrices from the
 * classical compact groups", 2007). Gram-Schmidt with one re-orthogonalisation pass. */
static int qo_gram_schmidt_columns(int64_t rows, int64_t first, int64_t cols, qo_cplx *A) {
  for (int64_t j = first; j < cols; ++j) {
    qo_cplx *v = A + j * rows;
    double norm0 = 0.0;
    for (int64_t i = 0; i < rows; ++i) norm0 += creal(v[i] * conj(v[i]));
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t k = 0; k < j; ++k) {
        const qo_cplx *q = A + k * rows;
        qo_cplx r = 0.0;
        for (int64_t i = 0; i < rows; ++i) r += conj(q[i]) * v[i];
        for (int64_t i = 0; i < rows; ++i) v[i] -= r * q[i];
      }
    }
    double norm = 0.0;
    for (int64_t i = 0; i < rows; ++i) norm += creal(v[i] * conj(v[i]));
    norm = sqrt(norm);
    if (!(norm > 1e-12 * sqrt(norm0)) || norm == 0.0) return -1;
    for (int64_t i = 0; i < rows; ++i) v[i] /= norm;
  }
  return 0;
}

int qo_orthonormalize(int64_t rows, int64_t cols, qo_cplx *A) {
  return qo_gram_schmidt_columns(rows, 0, cols, A);
}

/* Sample states (Sec. 2.3 and Sec. 3: M mutually orthogonal Haar states; App. A: the
 * columns of a Haar unitary). Column j is drawn from Philox index j*N + i, so the first
 * M columns do not depend on how many more are drawn later. */
int qo_draw_states(int n, int M, uint64_t seed, uint32_t role, uint32_t stream,
                   qo_cplx *out) {
  const int64_t N = (int64_t)1 << n;
  qo_ginibre(N, M, seed, role, stream, out);
  return qo_gram_schmidt_columns(N, 0, M, out);
}

/* Extension on doubling (Sec. 3 "double-and-restart"; Fig. pre-comp: A and B_0 are
 * recomputed when the training set changes): columns m_old..m_new-1 of the same
 * Ginibre stream, orthogonalised against every earlier column. */
static int qo_extend_states(int n, int m_old, int m_new, uint64_t seed, qo_cplx *psi) {
  const int64_t N = (int64_t)1 << n;
  for (int64_t j = m_old; j < m_new; ++j)
    for (int64_t i = 0; i < N; ++i)
      psi[j * N + i] = qo_cgauss(seed, QO_ROLE_TRAIN, 0, (uint64_t)(j * N + i));
  return qo_gram_schmidt_columns(N, m_old, m_new, psi);
}

/* Initial gate of one start (App. A: random initial unitaries controlled by the seed):
 * Haar on U(4) from a 4x4 Ginibre block. Stored row-major u[q][p] = Q[q][p]. */
void qo_haar_gate(uint64_t seed, uint32_t start, uint32_t gate, qo_cplx u[16]) {
  qo_cplx cols[16]; /* column-major */
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i)
      cols[j * 4 + i] = qo_cgauss(seed, QO_ROLE_INIT, start, (uint64_t)gate * 16u + j * 4 + i);
  qo_gram_schmidt_columns(4, 0, 4, cols);
  for (int q = 0; q < 4; ++q)
    for (int p = 0; p < 4; ++p) u[q * 4 + p] = cols[p * 4 + q];
}

/* Initial one-qubit gate: Haar on U(2) from a 2x2 Ginibre block of the same stream
 * (indices 16*gate + 2*col + row), orthonormalised the same way. Row-major v[q][p]. */
void qo_haar_gate2(uint64_t seed, uint32_t start, uint32_t gate, qo_cplx v[4]) {
  qo_cplx cols[4]; /* column-major */
  for (int j = 0; j < 2; ++j)
    for (int i = 0; i < 2; ++i)
      cols[j * 2 + i] = qo_cgauss(seed, QO_ROLE_INIT, start, (uint64_t)gate * 16u + j * 2 + i);
  qo_gram_schmidt_columns(2, 0, 2, cols);
  for (int q = 0; q < 2; ++q)
    for (int p = 0; p < 2; ++p) v[q * 2 + p] = cols[p * 2 + q];
}

/* v (x) I_2 in the local basis 2*bit(qa) + bit(qb): entry (2q + x, 2p + y) is
 * v[q][p] when x = y, else 0. */
static void qo_kron_i2(const qo_cplx v[4], qo_cplx u[16]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      u[r * 4 + c] = ((r & 1) == (c & 1)) ? v[(r >> 1) * 2 + (c >> 1)] : 0.0;
}

void qo_initial_gate(uint64_t seed, uint32_t start, uint32_t gate, int kind,
                     const qo_cplx *fixed, qo_cplx u[16]) {
  if (kind == QO_GATE_FIXED) {
    memcpy(u, fixed + 16 * (size_t)gate, sizeof(qo_cplx) * 16);
  } else if (kind == QO_GATE_1Q) {
    qo_cplx v[4];
    qo_haar_gate2(seed, start, gate, v);
    qo_kron_i2(v, u);
  } else {
    qo_haar_gate(seed, start, gate, u);
  }
}

/* ------------------------------------------------------------------------------------
 * State simulation (Sec. 3, Fig. pre-comp: the B list holds C's intermediate states).
 * ---------------------------------------------------------------------------------- */
static void qo_group_indices(int n, int qa, int qb, int64_t base, int64_t idx[4]) {
  const int64_t ma = (int64_t)1 << (n - 1 - qa);
  const int64_t mb = (int64_t)1 << (n - 1 - qb);
  idx[0] = base;
  idx[1] = base | mb;
  idx[2] = base | ma;
  idx[3] = base | ma | mb;
}

static void qo_apply_gate_impl(int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx u[16],
                               int dagger) {
  const int64_t N = (int64_t)1 << n;
  const int64_t ma = (int64_t)1 << (n - 1 - qa);
  const int64_t mb = (int64_t)1 << (n - 1 - qb);
  qo_cplx m[16];
  for (int q = 0; q < 4; ++q)
    for (int p = 0; p < 4; ++p) m[q * 4 + p] = dagger ? conj(u[p * 4 + q]) : u[q * 4 + p];
  for (int64_t j = 0; j < M; ++j) {
    qo_cplx *s = st + j * N;
    for (int64_t i = 0; i < N; ++i) {
      if ((i & ma) || (i & mb)) continue;
      int64_t idx[4];
      qo_group_indices(n, qa, qb, i, idx);
      qo_cplx v[4], w[4];
      for (int p = 0; p < 4; ++p) v[p] = s[idx[p]];
      for (int q = 0; q < 4; ++q) {
        w[q] = 0.0;
        for (int p = 0; p < 4; ++p) w[q] += m[q * 4 + p] * v[p];
      }
      for (int q = 0; q < 4; ++q) s[idx[q]] = w[q];
    }
  }
}

void qo_apply_gate(int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx u[16]) {
  qo_apply_gate_impl(n, M, st, qa, qb, u, 0);
}

void qo_apply_gate_dag(int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx u[16]) {
  qo_apply_gate_impl(n, M, st, qa, qb, u, 1);
}

void qo_apply_circuit(int n, int M, qo_cplx *st, int L, const int32_t *pairs,
                      const qo_cplx *gates) {
  for (int k = 0; k < L; ++k)
    qo_apply_gate(n, M, st, pairs[2 * k], pairs[2 * k + 1], gates + 16 * k);
}

/* Output training states U psi_j for a dense target (Sec. 2.3: the training pairs are
 * (psi_j, U psi_j)). */
void qo_dense_apply(int n, int M, const qo_cplx *U, const qo_cplx *psi, qo_cplx *out) {
  const int64_t N = (int64_t)1 << n;
  for (int64_t j = 0; j < M; ++j)
    for (int64_t r = 0; r < N; ++r) {
      qo_cplx acc = 0.0;
      for (int64_t c = 0; c < N; ++c) acc += U[r * N + c] * psi[j * N + c];
      out[j * N + r] = acc;
    }
}

/* Environment of one two-qubit gate (Sec. 3, Eq. 10 and Fig. env_calc_tensor): the
 * contraction of the backward state a with the conjugate forward state B over every
 * sample j and every index r of the other n-2 qubits. */
void qo_environment(int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, int qb,
                    qo_cplx G[16]) {
  const int64_t N = (int64_t)1 << n;
  const int64_t ma = (int64_t)1 << (n - 1 - qa);
  const int64_t mb = (int64_t)1 << (n - 1 - qb);
  for (int e = 0; e < 16; ++e) G[e] = 0.0;
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = 0; i < N; ++i) {
      if ((i & ma) || (i & mb)) continue;
      int64_t idx[4];
      qo_group_indices(n, qa, qb, i, idx);
      for (int q = 0; q < 4; ++q)
        for (int p = 0; p < 4; ++p) G[q * 4 + p] += a[j * N + idx[q]] * conj(b[j * N + idx[p]]);
    }
}

/* Environment of a one-qubit gate on qubit qa (the same contraction with the gate's
 * single qubit): the sum over every sample j and every index r of the other n-1 qubits
 * of a_j(q, r) conj(b_j(p, r)). */
void qo_environment1(int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, qo_cplx G[4]) {
  const int64_t N = (int64_t)1 << n;
  const int64_t ma = (int64_t)1 << (n - 1 - qa);
  for (int e = 0; e < 4; ++e) G[e] = 0.0;
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = 0; i < N; ++i) {
      if (i & ma) continue;
      for (int q = 0; q < 2; ++q)
        for (int p = 0; p < 2; ++p)
          G[q * 2 + p] += a[j * N + i + q * ma] * conj(b[j * N + i + p * ma]);
    }
}

/* ------------------------------------------------------------------------------------
 * SVD and gate update (Sec. 2.1, Eq. 2: E = X D Y^dagger, u = Y X^dagger).
 * One-sided Jacobi (Hestenes 1958): rotate pairs of columns of G by 2x2 unitaries until
 * all columns are mutually orthogonal; then G V = W diag(s).
 * ---------------------------------------------------------------------------------- */
void qo_svd4(const qo_cplx Gin[16], qo_cplx W[16], double s[4], qo_cplx V[16]) {
  qo_cplx g[4][4], v[4][4]; /* [column][row] */
  for (int c = 0; c < 4; ++c)
    for (int r = 0; r < 4; ++r) {
      g[c][r] = Gin[r * 4 + c];
      v[c][r] = (r == c) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        double alpha = 0.0, beta = 0.0;
        qo_cplx gamma = 0.0;
        for (int r = 0; r < 4; ++r) {
          alpha += creal(g[p][r] * conj(g[p][r]));
          beta += creal(g[q][r] * conj(g[q][r]));
          gamma += conj(g[p][r]) * g[q][r];
        }
        double ag = cabs(gamma);
        if (ag == 0.0 || ag <= 1e-15 * sqrt(alpha * beta)) continue;
        rotated = 1;
        /* Hermitian 2x2 Gram block [[alpha, gamma], [conj(gamma), beta]] =
         * D R D^dagger with D = diag(1, e^{-i phi}), R real symmetric; J = D * (real
         * Jacobi rotation diagonalising R) (Golub & Van Loan, sym.schur2). */
        qo_cplx e = gamma / ag; /* e^{i phi} */
        double tau = (beta - alpha) / (2.0 * ag);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t);
        double sn = c * t;
        for (int r = 0; r < 4; ++r) {
          qo_cplx gp = g[p][r], gq = g[q][r];
          g[p][r] = c * gp - sn * conj(e) * gq;
          g[q][r] = sn * gp + c * conj(e) * gq;
          qo_cplx vp = v[p][r], vq = v[q][r];
          v[p][r] = c * vp - sn * conj(e) * vq;
          v[q][r] = sn * vp + c * conj(e) * vq;
        }
      }
    if (!rotated) break;
  }
  /* Singular values, and left vectors in decreasing-s order re-orthonormalised (and
   * completed with unit vectors where s is negligible), so that W is unitary. */
  double nrm[4];
  int order[4] = {0, 1, 2, 3};
  for (int c = 0; c < 4; ++c) {
    double acc = 0.0;
    for (int r = 0; r < 4; ++r) acc += creal(g[c][r] * conj(g[c][r]));
    nrm[c] = sqrt(acc);
  }
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b)
      if (nrm[order[b]] > nrm[order[a]]) {
        int tmp = order[a]; order[a] = order[b]; order[b] = tmp;
      }
  double smax = nrm[order[0]];
  qo_cplx w[4][4];
  int filled = 0;
  for (int k = 0; k < 4; ++k) {
    int c = order[k];
    s[k] = nrm[c];
    for (int r = 0; r < 4; ++r) V[r * 4 + k] = v[c][r];
    qo_cplx x[4];
    int ok = 0;
    if (nrm[c] > 1e-13 * smax && nrm[c] > 0.0) {
      for (int r = 0; r < 4; ++r) x[r] = g[c][r] / nrm[c];
      ok = 1;
    }
    if (ok) {
      for (int pass = 0; pass < 2; ++pass)
        for (int m = 0; m < filled; ++m) {
          qo_cplx d = 0.0;
          for (int r = 0; r < 4; ++r) d += conj(w[m][r]) * x[r];
          for (int r = 0; r < 4; ++r) x[r] -= d * w[m][r];
        }
      double l = 0.0;
      for (int r = 0; r < 4; ++r) l += creal(x[r] * conj(x[r]));
      l = sqrt(l);
      if (l > 0.5) {
        for (int r = 0; r < 4; ++r) x[r] /= l;
      } else {
        ok = 0;
      }
    }
    if (!ok) {
      /* complete with the unit vector that keeps the largest orthogonal part */
      double best = -1.0;
      qo_cplx bx[4];
      for (int e = 0; e < 4; ++e) {
        qo_cplx y[4] = {0, 0, 0, 0};
        y[e] = 1.0;
        for (int pass = 0; pass < 2; ++pass)
          for (int m = 0; m < filled; ++m) {
            qo_cplx d = 0.0;
            for (int r = 0; r < 4; ++r) d += conj(w[m][r]) * y[r];
            for (int r = 0; r < 4; ++r) y[r] -= d * w[m][r];
          }
        double l = 0.0;
        for (int r = 0; r < 4; ++r) l += creal(y[r] * conj(y[r]));
        if (l > best) {
          best = l;
          for (int r = 0; r < 4; ++r) bx[r] = y[r];
        }
      }
      best = sqrt(best);
      for (int r = 0; r < 4; ++r) x[r] = bx[r] / best;
    }
    for (int r = 0; r < 4; ++r) w[filled][r] = x[r];
    ++filled;
  }
  for (int k = 0; k < 4; ++k)
    for (int r = 0; r < 4; ++r) W[r * 4 + k] = w[k][r];
}

/* Gate update. The paper's update (Sec. 2.1, Eq. 2; Sec. 3 reuses it) is u = Y X^dagger
 * with E = X D Y^dagger; with Gamma = E^dagger this is u = W V^dagger for
 * Gamma = W S V^dagger. App. A's regularised form takes the SVD of (1-beta) E +
 * beta u^dagger, whose conjugate transpose is (1-beta) Gamma + beta u. */
void qo_update_gate(const qo_cplx G[16], double beta, qo_cplx u[16]) {
  qo_cplx X[16], W[16], V[16];
  double s[4];
  for (int e = 0; e < 16; ++e) X[e] = (1.0 - beta) * G[e] + beta * u[e];
  qo_svd4(X, W, s, V);
  for (int q = 0; q < 4; ++q)
    for (int p = 0; p < 4; ++p) {
      qo_cplx acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += W[q * 4 + k] * conj(V[p * 4 + k]);
      u[q * 4 + p] = acc;
    }
}

/* Update of a one-qubit gate (the same rule for a 2x2 environment). With X the 2x2
 * matrix (1-beta) G + beta v, the polar factor of the block-diagonal diag(X, I_2) is
 * diag(polar(X), I_2) (the polar factor of an invertible matrix is unique, and a block
 * diagonal SVD is one SVD of the whole), so the 4x4 routine gives polar(X) as its
 * leading block. The slot keeps the form v (x) I_2. */
void qo_update_gate1(const qo_cplx G[4], double beta, qo_cplx u[16]) {
  qo_cplx X[16], P[16];
  for (int e = 0; e < 16; ++e) X[e] = 0.0;
  for (int q = 0; q < 2; ++q)
    for (int p = 0; p < 2; ++p)
      X[q * 4 + p] = (1.0 - beta) * G[q * 2 + p] + beta * u[(2 * q) * 4 + 2 * p];
  X[10] = 1.0;
  X[15] = 1.0;
  for (int e = 0; e < 16; ++e) P[e] = 0.0;
  qo_update_gate(X, 0.0, P);
  qo_cplx v[4] = {P[0], P[1], P[4], P[5]};
  qo_kron_i2(v, u);
}

/* (1/M) sum_j ||x_j - y_j||^2: the QFactor-Sample cost (Sec. 3, Eq. 9, left side). */
double qo_state_distance(int n, int M, const qo_cplx *x, const qo_cplx *y) {
  const int64_t N = (int64_t)1 << n;
  double acc = 0.0;
  for (int64_t e = 0; e < (int64_t)M * N; ++e) {
    qo_cplx d = x[e] - y[e];
    acc += creal(d * conj(d));
  }
  return acc / (double)M;
}

static double qo_re_tr_gdag_u(const qo_cplx G[16], const qo_cplx u[16]) {
  double acc = 0.0;
  for (int e = 0; e < 16; ++e) acc += creal(conj(G[e]) * u[e]);
  return acc;
}

/* One sweep (Sec. 3; Fig. pre-comp; Fig. env_calc_tensor). The B list is computed
 * from the gates as they were before the sweep; the backward state a starts at
 * U psi (the A tensor) and is moved through each gate right after that gate has been
 * updated, so every environment mixes updated (left of the gate in time order, i.e.
 * later in the circuit) and not-yet-updated gates. Returns the cost (Eq. 9) of the
 * updated gates, computed from a_0 = C^dagger U psi. */
static double qo_re_tr_gdag_v(const qo_cplx G[4], const qo_cplx u[16]) {
  double acc = 0.0;
  for (int q = 0; q < 2; ++q)
    for (int p = 0; p < 2; ++p) acc += creal(conj(G[q * 2 + p]) * u[(2 * q) * 4 + 2 * p]);
  return acc;
}

/* A fixed gate is applied on both passes and never updated; a one-qubit gate is
 * updated from its 2x2 environment. */
double qo_sweep(int n, int L, const int32_t *pairs, const int32_t *kinds, int M,
                const qo_cplx *psi, const qo_cplx *phi, qo_cplx *gates, double beta,
                double gamma_scale, double *f_before, double *f_after, qo_cplx *gammas) {
  const int64_t N = (int64_t)1 << n;
  const int64_t S = (int64_t)M * N;
  qo_cplx *B = (qo_cplx *)malloc(sizeof(qo_cplx) * S * (size_t)L);
  qo_cplx *a = (qo_cplx *)malloc(sizeof(qo_cplx) * S);
  memcpy(B, psi, sizeof(qo_cplx) * S);
  for (int k = 1; k < L; ++k) {
    memcpy(B + (size_t)k * S, B + (size_t)(k - 1) * S, sizeof(qo_cplx) * S);
    qo_apply_gate(n, M, B + (size_t)k * S, pairs[2 * (k - 1)], pairs[2 * (k - 1) + 1],
                  gates + 16 * (k - 1));
  }
  memcpy(a, phi, sizeof(qo_cplx) * S);
  for (int k = L - 1; k >= 0; --k) {
    const int kind = kinds ? kinds[k] : QO_GATE_2Q;
    qo_cplx G[16], Gs[16];
    for (int e = 0; e < 16; ++e) G[e] = 0.0;
    if (kind == QO_GATE_2Q) {
      qo_environment(n, M, a, B + (size_t)k * S, pairs[2 * k], pairs[2 * k + 1], G);
      for (int e = 0; e < 16; ++e) Gs[e] = gamma_scale * G[e];
      if (f_before) f_before[k] = qo_re_tr_gdag_u(G, gates + 16 * k);
      qo_update_gate(Gs, beta, gates + 16 * k);
      if (f_after) f_after[k] = qo_re_tr_gdag_u(G, gates + 16 * k);
    } else if (kind == QO_GATE_1Q) {
      qo_environment1(n, M, a, B + (size_t)k * S, pairs[2 * k], G);
      for (int e = 0; e < 4; ++e) Gs[e] = gamma_scale * G[e];
      if (f_before) f_before[k] = qo_re_tr_gdag_v(G, gates + 16 * k);
      qo_update_gate1(Gs, beta, gates + 16 * k);
      if (f_after) f_after[k] = qo_re_tr_gdag_v(G, gates + 16 * k);
    } else {
      if (f_before) f_before[k] = NAN;
      if (f_after) f_after[k] = NAN;
    }
    if (gammas) memcpy(gammas + 16 * k, G, sizeof(G));
    qo_apply_gate_dag(n, M, a, pairs[2 * k], pairs[2 * k + 1], gates + 16 * k);
  }
  double c = qo_state_distance(n, M, a, psi);
  free(a);
  free(B);
  return c;
}

/* Cost of fixed gates on a state set: (1/M) sum ||U psi - C psi||^2 by simulation. */
static double qo_forward_cost(int n, int L, const int32_t *pairs, int M, const qo_cplx *psi,
                              const qo_cplx *phi, const qo_cplx *gates) {
  const int64_t S = (int64_t)M << n;
  qo_cplx *x = (qo_cplx *)malloc(sizeof(qo_cplx) * S);
  memcpy(x, psi, sizeof(qo_cplx) * S);
  qo_apply_circuit(n, M, x, L, pairs, gates);
  double c = qo_state_distance(n, M, phi, x);
  free(x);
  return c;
}

/* ------------------------------------------------------------------------------------
 * Qudits (Sec. 5: the method applies unchanged to d-level gates, where a sweep costs
 * O(M d^n) instead of QFactor's O(d^{2n})). n qudits of dimension d, N = d^n; qudit 0 is
 * the most significant base-d digit of the amplitude index (stride d^{n-1-q}); a
 * two-qudit gate on (qa, qb) is a D x D unitary, D = d^2, row-major u[q][p], with local
 * index d * digit(qa) + digit(qb). With d = 2 every function below computes what the
 * qubit functions above compute.
 * ---------------------------------------------------------------------------------- */
static int64_t qd_pow(int d, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= d;
  return r;
}

/* Amplitude indices of the D-group of base index i (digits of qa and qb zero). */
static void qd_group(int d, int n, int qa, int qb, int64_t i, int64_t *idx) {
  const int64_t sa = qd_pow(d, n - 1 - qa), sb = qd_pow(d, n - 1 - qb);
  for (int x = 0; x < d; ++x)
    for (int y = 0; y < d; ++y) idx[x * d + y] = i + x * sa + y * sb;
}

static int qd_is_base(int d, int n, int qa, int qb, int64_t i) {
  return (i / qd_pow(d, n - 1 - qa)) % d == 0 && (i / qd_pow(d, n - 1 - qb)) % d == 0;
}

/* st <- u st (or u^dagger st) on qudits (qa, qb), every sample. */
void qd_apply_gate(int d, int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx *u, int dagger) {
  const int D = d * d;
  const int64_t N = qd_pow(d, n);
  int64_t idx[16];
  qo_cplx in[16];
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = 0; i < N; ++i) {
      if (!qd_is_base(d, n, qa, qb, i)) continue;
      qd_group(d, n, qa, qb, i, idx);
      for (int p = 0; p < D; ++p) in[p] = st[j * N + idx[p]];
      for (int q = 0; q < D; ++q) {
        qo_cplx acc = 0.0;
        for (int p = 0; p < D; ++p) acc += (dagger ? conj(u[p * D + q]) : u[q * D + p]) * in[p];
        st[j * N + idx[q]] = acc;
      }
    }
}

/* Environment of a two-qudit gate: G[q][p] = sum_j sum_r a_j(q, r) conj(b_j(p, r)) over the
 * other n-2 qudits (the qubit environment above with base-d digits). */
void qd_environment(int d, int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, int qb,
                    qo_cplx *G) {
  const int D = d * d;
  const int64_t N = qd_pow(d, n);
  int64_t idx[16];
  for (int e = 0; e < D * D; ++e) G[e] = 0.0;
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = 0; i < N; ++i) {
      if (!qd_is_base(d, n, qa, qb, i)) continue;
      qd_group(d, n, qa, qb, i, idx);
      for (int q = 0; q < D; ++q)
        for (int p = 0; p < D; ++p) G[q * D + p] += a[j * N + idx[q]] * conj(b[j * N + idx[p]]);
    }
}

/* D x D complex SVD G = W diag(s) V^dagger (D <= 16) by one-sided Jacobi, the same
 * rotations as qo_svd4 on D columns; s in decreasing order, W completed to a unitary
 * where singular values are negligible. */
void qd_svd(int D, const qo_cplx *Gin, qo_cplx *W, double *s, qo_cplx *V) {
  qo_cplx g[16][16], v[16][16]; /* [column][row] */
  for (int c = 0; c < D; ++c)
    for (int r = 0; r < D; ++r) {
      g[c][r] = Gin[r * D + c];
      v[c][r] = (r == c) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 80; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < D - 1; ++p)
      for (int q = p + 1; q < D; ++q) {
        double alpha = 0.0, beta = 0.0;
        qo_cplx gamma = 0.0;
        for (int r = 0; r < D; ++r) {
          alpha += creal(g[p][r] * conj(g[p][r]));
          beta += creal(g[q][r] * conj(g[q][r]));
          gamma += conj(g[p][r]) * g[q][r];
        }
        double ag = cabs(gamma);
        if (ag == 0.0 || ag <= 1e-15 * sqrt(alpha * beta)) continue;
        rotated = 1;
        qo_cplx e = gamma / ag;
        double tau = (beta - alpha) / (2.0 * ag);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t);
        double sn = c * t;
        for (int r = 0; r < D; ++r) {
          qo_cplx gp = g[p][r], gq = g[q][r];
          g[p][r] = c * gp - sn * conj(e) * gq;
          g[q][r] = sn * gp + c * conj(e) * gq;
          qo_cplx vp = v[p][r], vq = v[q][r];
          v[p][r] = c * vp - sn * conj(e) * vq;
          v[q][r] = sn * vp + c * conj(e) * vq;
        }
      }
    if (!rotated) break;
  }
  double nrm[16];
  int order[16];
  for (int c = 0; c < D; ++c) {
    double acc = 0.0;
    for (int r = 0; r < D; ++r) acc += creal(g[c][r] * conj(g[c][r]));
    nrm[c] = sqrt(acc);
    order[c] = c;
  }
  for (int a = 0; a < D; ++a)
    for (int b = a + 1; b < D; ++b)
      if (nrm[order[b]] > nrm[order[a]]) {
        int tmp = order[a]; order[a] = order[b]; order[b] = tmp;
      }
  double smax = nrm[order[0]];
  qo_cplx w[16][16];
  for (int k = 0; k < D; ++k) {
    int c = order[k];
    s[k] = nrm[c];
    for (int r = 0; r < D; ++r) V[r * D + k] = v[c][r];
    qo_cplx x[16];
    int ok = 0;
    if (nrm[c] > 1e-13 * smax && nrm[c] > 0.0) {
      for (int r = 0; r < D; ++r) x[r] = g[c][r] / nrm[c];
      for (int pass = 0; pass < 2; ++pass)
        for (int m = 0; m < k; ++m) {
          qo_cplx dd = 0.0;
          for (int r = 0; r < D; ++r) dd += conj(w[m][r]) * x[r];
          for (int r = 0; r < D; ++r) x[r] -= dd * w[m][r];
        }
      double l = 0.0;
      for (int r = 0; r < D; ++r) l += creal(x[r] * conj(x[r]));
      l = sqrt(l);
      if (l > 0.5) {
        for (int r = 0; r < D; ++r) x[r] /= l;
        ok = 1;
      }
    }
    if (!ok) {
      double best = -1.0;
      qo_cplx bx[16];
      for (int e = 0; e < D; ++e) {
        qo_cplx y[16];
        for (int r = 0; r < D; ++r) y[r] = (r == e) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass)
          for (int m = 0; m < k; ++m) {
            qo_cplx dd = 0.0;
            for (int r = 0; r < D; ++r) dd += conj(w[m][r]) * y[r];
            for (int r = 0; r < D; ++r) y[r] -= dd * w[m][r];
          }
        double l = 0.0;
        for (int r = 0; r < D; ++r) l += creal(y[r] * conj(y[r]));
        if (l > best) {
          best = l;
          for (int r = 0; r < D; ++r) bx[r] = y[r];
        }
      }
      best = sqrt(best);
      for (int r = 0; r < D; ++r) x[r] = bx[r] / best;
    }
    for (int r = 0; r < D; ++r) w[k][r] = x[r];
  }
  for (int k = 0; k < D; ++k)
    for (int r = 0; r < D; ++r) W[r * D + k] = w[k][r];
}

/* u <- W V^dagger for (1 - beta) G + beta u = W S V^dagger (Eq. 2, App. A Beta). */
void qd_update_gate(int D, const qo_cplx *G, double beta, qo_cplx *u) {
  qo_cplx X[256], Wm[256], Vm[256];
  double sv[16];
  for (int e = 0; e < D * D; ++e) X[e] = (1.0 - beta) * G[e] + beta * u[e];
  qd_svd(D, X, Wm, sv, Vm);
  for (int q = 0; q < D; ++q)
    for (int p = 0; p < D; ++p) {
      qo_cplx acc = 0.0;
      for (int k = 0; k < D; ++k) acc += Wm[q * D + k] * conj(Vm[p * D + k]);
      u[q * D + p] = acc;
    }
}

/* Initial two-qudit gate: Haar on U(D) from a D x D Ginibre block of the start's
 * initial-gate stream (indices 256 gate + D col + row), orthonormalised by columns. */
void qd_haar_gate(int d, uint64_t seed, uint32_t start, uint32_t gate, qo_cplx *u) {
  const int D = d * d;
  qo_cplx cols[256];
  for (int j = 0; j < D; ++j)
    for (int i = 0; i < D; ++i)
      cols[j * D + i] = qo_cgauss(seed, QO_ROLE_INIT, start, (uint64_t)gate * 256u + (uint64_t)(j * D + i));
  qo_gram_schmidt_columns(D, 0, D, cols);
  for (int q = 0; q < D; ++q)
    for (int p = 0; p < D; ++p) u[q * D + p] = cols[p * D + q];
}

/* Environment of a one-qudit gate on qudit qa: the sum over every sample j and every
 * index r of the other n-1 qudits of a_j(x, r) conj(b_j(y, r)), d x d. */
void qd_environment1(int d, int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, qo_cplx *G) {
  const int64_t N = qd_pow(d, n), sa = qd_pow(d, n - 1 - qa);
  for (int e = 0; e < d * d; ++e) G[e] = 0.0;
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = 0; i < N; ++i) {
      if ((i / sa) % d != 0) continue;
      for (int x = 0; x < d; ++x)
        for (int y = 0; y < d; ++y) G[x * d + y] += a[j * N + i + x * sa] * conj(b[j * N + i + y * sa]);
    }
}

/* v (x) I_d in the local basis d digit(qa) + digit(qb): entry (d x + z, d y + w) is v[x][y]
 * when z = w, else 0. */
static void qd_kron_id(int d, const qo_cplx *v, qo_cplx *u) {
  const int D = d * d;
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) u[r * D + c] = (r % d == c % d) ? v[(r / d) * d + c / d] : 0.0;
}

/* Update of a one-qudit gate held as the slot v (x) I_d: v <- polar((1 - beta) G1 + beta v)
 * with the d x d environment G1 (the two-qudit rule on the gate's own d levels); the slot
 * keeps its form. */
void qd_update_gate1(int d, const qo_cplx *G1, double beta, qo_cplx *u) {
  const int D = d * d;
  qo_cplx v[16];
  for (int x = 0; x < d; ++x)
    for (int y = 0; y < d; ++y) v[x * d + y] = u[(d * x) * D + d * y];
  qd_update_gate(d, G1, beta, v);
  qd_kron_id(d, v, u);
}

/* Initial one-qudit gate: Haar on U(d) from the d x d Ginibre block at indices
 * 256 gate + d col + row of the start's initial-gate stream, as the slot v (x) I_d. */
void qd_haar_gate1(int d, uint64_t seed, uint32_t start, uint32_t gate, qo_cplx *u) {
  qo_cplx cols[16], v[16];
  for (int j = 0; j < d; ++j)
    for (int i = 0; i < d; ++i)
      cols[j * d + i] = qo_cgauss(seed, QO_ROLE_INIT, start, (uint64_t)gate * 256u + (uint64_t)(j * d + i));
  qo_gram_schmidt_columns(d, 0, d, cols);
  for (int q = 0; q < d; ++q)
    for (int p = 0; p < d; ++p) v[q * d + p] = cols[p * d + q];
  qd_kron_id(d, v, u);
}

static double qd_re_tr(int D, const qo_cplx *G, const qo_cplx *u) {
  double acc = 0.0;
  for (int e = 0; e < D * D; ++e) acc += creal(conj(G[e]) * u[e]);
  return acc;
}

/* One sweep on qudits (the qubit sweep with D x D gates): a constant gate is applied in
 * both passes and never updated; a one-qudit gate is updated from its d x d environment. */
double qd_sweep(int d, int n, int L, const int32_t *pairs, const int32_t *kinds, int M,
                const qo_cplx *psi, const qo_cplx *phi, qo_cplx *gates, double beta,
                double gamma_scale, double *f_before, double *f_after) {
  const int D = d * d, GS = D * D;
  const int64_t S = (int64_t)M * qd_pow(d, n);
  qo_cplx *B = (qo_cplx *)malloc(sizeof(qo_cplx) * S * (size_t)L);
  qo_cplx *a = (qo_cplx *)malloc(sizeof(qo_cplx) * S);
  qo_cplx G[256], Gs[256];
  memcpy(B, psi, sizeof(qo_cplx) * S);
  for (int k = 1; k < L; ++k) {
    memcpy(B + (size_t)k * S, B + (size_t)(k - 1) * S, sizeof(qo_cplx) * S);
    qd_apply_gate(d, n, M, B + (size_t)k * S, pairs[2 * (k - 1)], pairs[2 * (k - 1) + 1],
                  gates + GS * (k - 1), 0);
  }
  memcpy(a, phi, sizeof(qo_cplx) * S);
  for (int k = L - 1; k >= 0; --k) {
    const int kind = kinds ? kinds[k] : QO_GATE_2Q;
    if (kind == QO_GATE_2Q) {
      qd_environment(d, n, M, a, B + (size_t)k * S, pairs[2 * k], pairs[2 * k + 1], G);
      if (f_before) f_before[k] = qd_re_tr(D, G, gates + GS * k);
      for (int e = 0; e < GS; ++e) Gs[e] = gamma_scale * G[e];
      qd_update_gate(D, Gs, beta, gates + GS * k);
      if (f_after) f_after[k] = qd_re_tr(D, G, gates + GS * k);
    } else if (kind == QO_GATE_1Q) {
      qd_environment1(d, n, M, a, B + (size_t)k * S, pairs[2 * k], G);
      qo_cplx Gk[256];
      for (int e = 0; e < GS; ++e) Gk[e] = 0.0;
      for (int x = 0; x < d; ++x)
        for (int y = 0; y < d; ++y) Gk[(d * x) * D + d * y] = G[x * d + y];
      if (f_before) f_before[k] = qd_re_tr(D, Gk, gates + GS * k);
      for (int e = 0; e < d * d; ++e) Gs[e] = gamma_scale * G[e];
      qd_update_gate1(d, Gs, beta, gates + GS * k);
      if (f_after) f_after[k] = qd_re_tr(D, Gk, gates + GS * k);
    } else {
      if (f_before) f_before[k] = NAN;
      if (f_after) f_after[k] = NAN;
    }
    qd_apply_gate(d, n, M, a, pairs[2 * k], pairs[2 * k + 1], gates + GS * k, 1);
  }
  double c = 0.0;
  for (int64_t e = 0; e < S; ++e) {
    qo_cplx x = a[e] - psi[e];
    c += creal(x * conj(x));
  }
  free(a);
  free(B);
  return c / (double)M;
}

static double qd_forward_cost(int d, int n, int L, const int32_t *pairs, int M, const qo_cplx *psi,
                              const qo_cplx *phi, const qo_cplx *gates) {
  const int GS = d * d * d * d;
  const int64_t S = (int64_t)M * qd_pow(d, n);
  qo_cplx *x = (qo_cplx *)malloc(sizeof(qo_cplx) * S);
  memcpy(x, psi, sizeof(qo_cplx) * S);
  for (int k = 0; k < L; ++k) qd_apply_gate(d, n, M, x, pairs[2 * k], pairs[2 * k + 1], gates + GS * k, 0);
  double c = 0.0;
  for (int64_t e = 0; e < S; ++e) {
    qo_cplx y = x[e] - phi[e];
    c += creal(y * conj(y));
  }
  free(x);
  return c / (double)M;
}

/* ------------------------------------------------------------------------------------
 * The control loop (Sec. 3 "on-the-fly" generalisation check and double-and-restart;
 * the success relations of Eq. 12; App. A plateau test Eq. 13, min_iter, max_iter,
 * multistarts). Readings where the paper is silent are listed in the design notes:
 * validation set of size M drawn independently and redrawn on doubling; a doubling
 * extends the training set and keeps every gate; the iteration and plateau counters
 * restart after a doubling; at M = 2^n the training cost is the exact full distance
 * (Eq. 1 over 2^n), so the generalisation test is not applied there.
 * ---------------------------------------------------------------------------------- */
enum { ST_RUNNING = 0, ST_STOPPED = 1, ST_OVERTRAINED = 2 };

static double qo_now(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void qo_targets(int n, int kind, const qo_cplx *U, int Lt, const int32_t *tpairs,
                       const qo_cplx *tgates, int M, const qo_cplx *psi, qo_cplx *phi) {
  const int64_t S = (int64_t)M << n;
  if (kind == QO_TARGET_DENSE) {
    qo_dense_apply(n, M, U, psi, phi);
  } else {
    memcpy(phi, psi, sizeof(qo_cplx) * S);
    qo_apply_circuit(n, M, phi, Lt, tpairs, tgates);
  }
}

/* The same three steps on n qudits (Sec. 5: states and targets are those of the qubit
 * method with N = d^n amplitudes). States: column j of the N x M Ginibre matrix from
 * Philox index j N + i, orthonormalised in column order, so an extension draws the next
 * columns of the same stream. Targets: phi_j = U psi_j for a dense N x N target, or the
 * target circuit's D x D gates applied to psi_j in list order. */
int qd_draw_states(int d, int n, int M, uint64_t seed, uint32_t role, uint32_t stream,
                   qo_cplx *out) {
  const int64_t N = qd_pow(d, n);
  qo_ginibre(N, M, seed, role, stream, out);
  return qo_gram_schmidt_columns(N, 0, M, out);
}

static int qd_extend_states(int d, int n, int m_old, int m_new, uint64_t seed, qo_cplx *psi) {
  const int64_t N = qd_pow(d, n);
  for (int64_t j = m_old; j < m_new; ++j)
    for (int64_t i = 0; i < N; ++i)
      psi[j * N + i] = qo_cgauss(seed, QO_ROLE_TRAIN, 0, (uint64_t)(j * N + i));
  return qo_gram_schmidt_columns(N, m_old, m_new, psi);
}

static void qd_targets(int d, int n, int kind, const qo_cplx *U, int Lt, const int32_t *tpairs,
                       const qo_cplx *tgates, int M, const qo_cplx *psi, qo_cplx *phi) {
  const int64_t N = qd_pow(d, n);
  const int GS = d * d * d * d;
  if (kind == QO_TARGET_DENSE) {
    for (int64_t j = 0; j < M; ++j)
      for (int64_t r = 0; r < N; ++r) {
        qo_cplx acc = 0.0;
        for (int64_t c = 0; c < N; ++c) acc += U[r * N + c] * psi[j * N + c];
        phi[j * N + r] = acc;
      }
  } else {
    memcpy(phi, psi, sizeof(qo_cplx) * (size_t)M * N);
    for (int k = 0; k < Lt; ++k)
      qd_apply_gate(d, n, M, phi, tpairs[2 * k], tpairs[2 * k + 1], tgates + (size_t)GS * k, 0);
  }
}

/* Draws, extension and targets for either case: the qubit functions when d = 2. */
static int any_draw(int d, int n, int M, uint64_t seed, uint32_t role, uint32_t stream, qo_cplx *out) {
  return d == 2 ? qo_draw_states(n, M, seed, role, stream, out) : qd_draw_states(d, n, M, seed, role, stream, out);
}
static int any_extend(int d, int n, int m_old, int m_new, uint64_t seed, qo_cplx *psi) {
  return d == 2 ? qo_extend_states(n, m_old, m_new, seed, psi) : qd_extend_states(d, n, m_old, m_new, seed, psi);
}
static void any_targets(int d, int n, int kind, const qo_cplx *U, int Lt, const int32_t *tpairs,
                        const qo_cplx *tgates, int M, const qo_cplx *psi, qo_cplx *phi) {
  if (d == 2)
    qo_targets(n, kind, U, Lt, tpairs, tgates, M, psi, phi);
  else
    qd_targets(d, n, kind, U, Lt, tpairs, tgates, M, psi, phi);
}

static int instantiate_impl(int d, int n, int L, const int32_t *pairs, const int32_t *kinds,
                   const qo_cplx *fixed, int target_kind, const qo_cplx *U,
                   int Lt, const int32_t *tpairs, const qo_cplx *tgates,
                   const qo_cplx *samples_psi, const qo_cplx *samples_phi, int n_samples,
                   int n_val, const qo_params *p, const qo_cplx *gates_in,
                   qo_cplx *gates_out, qo_result *res, qo_trace *trace) {
  const double t0 = qo_now();
  if (n < 2 || n > 24 || L < 1 || !p || !gates_out || !res) return -1;
  const int GS = d * d * d * d; /* entries of one gate */
  for (int k = 0; k < L; ++k) {
    int a = pairs[2 * k], b = pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b) return -1;
    if (kinds && (kinds[k] < QO_GATE_2Q || kinds[k] > QO_GATE_FIXED)) return -1;
    if (kinds && kinds[k] == QO_GATE_FIXED && !fixed) return -1;
  }
  const int64_t N = qd_pow(d, n);
  const int S = p->multistarts > 0 ? p->multistarts : 1;
  int m_cap = (p->m_max > 0 && p->m_max < N) ? p->m_max : (int)N;
  int n_train = 0;
  if (target_kind == QO_TARGET_SAMPLES) {
    n_train = n_samples - n_val;
    if (n_train < 1 || n_val < 0) return -1;
    if (n_train < m_cap) m_cap = n_train;
  }
  int M = p->m_init < 1 ? 1 : p->m_init;
  if (M > m_cap) M = m_cap;
  if (p->fixed_m) m_cap = M;

  qo_cplx *psi = (qo_cplx *)malloc(sizeof(qo_cplx) * (size_t)m_cap * N);
  qo_cplx *phi = (qo_cplx *)malloc(sizeof(qo_cplx) * (size_t)m_cap * N);
  qo_cplx *psiv = NULL, *phiv = NULL;
  int Mv = 0, generation = 0;

  /* training set (A tensor = U Psi, computed once per training set: Fig. pre-comp) */
  if (target_kind == QO_TARGET_SAMPLES) {
    memcpy(psi, samples_psi, sizeof(qo_cplx) * (size_t)M * N);
    memcpy(phi, samples_phi, sizeof(qo_cplx) * (size_t)M * N);
  } else {
    if (any_draw(d, n, M, p->seed, QO_ROLE_TRAIN, 0, psi) != 0) return -2;
    any_targets(d, n, target_kind, U, Lt, tpairs, tgates, M, psi, phi);
  }
  /* validation set */
  if (target_kind == QO_TARGET_SAMPLES) {
    Mv = n_val;
    if (Mv > 0) {
      psiv = (qo_cplx *)malloc(sizeof(qo_cplx) * (size_t)Mv * N);
      phiv = (qo_cplx *)malloc(sizeof(qo_cplx) * (size_t)Mv * N);
      memcpy(psiv, samples_psi + (size_t)n_train * N, sizeof(qo_cplx) * (size_t)Mv * N);
      memcpy(phiv, samples_phi + (size_t)n_train * N, sizeof(qo_cplx) * (size_t)Mv * N);
    }
  } else {
    Mv = p->m_val > 0 ? p->m_val : M;
    psiv = (qo_cplx *)malloc(sizeof(qo_cplx) * (size_t)Mv * N);
    phiv = (qo_cplx *)malloc(sizeof(qo_cplx) * (size_t)Mv * N);
    if (any_draw(d, n, Mv, p->seed, QO_ROLE_VAL, (uint32_t)generation, psiv) != 0) return -2;
    any_targets(d, n, target_kind, U, Lt, tpairs, tgates, Mv, psiv, phiv);
  }

  qo_cplx *gates = (qo_cplx *)malloc(sizeof(qo_cplx) * GS * (size_t)L * S);
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < L; ++k) {
      const int kind = kinds ? kinds[k] : QO_GATE_2Q;
      qo_cplx *u = gates + GS * ((size_t)s * L + k);
      if (kind == QO_GATE_FIXED)
        memcpy(u, fixed + GS * (size_t)k, sizeof(qo_cplx) * GS);
      else if (gates_in)
        memcpy(u, gates_in + GS * ((size_t)s * L + k), sizeof(qo_cplx) * GS);
      else if (d != 2 && kind == QO_GATE_1Q)
        qd_haar_gate1(d, p->seed, (uint32_t)s, (uint32_t)k, u);
      else if (d != 2)
        qd_haar_gate(d, p->seed, (uint32_t)s, (uint32_t)k, u);
      else
        qo_initial_gate(p->seed, (uint32_t)s, (uint32_t)k, kind, fixed, u);
    }
#define FWD_COST(MM, PS, PH, G)                                                  \
  (d == 2 ? qo_forward_cost(n, L, pairs, (MM), (PS), (PH), (G))                  \
          : qd_forward_cost(d, n, L, pairs, (MM), (PS), (PH), (G)))

  int *status = (int *)calloc(S, sizeof(int));
  int *reason = (int *)calloc(S, sizeof(int));
  int *iter = (int *)calloc(S, sizeof(int));
  int *zcount = (int *)calloc(S, sizeof(int));
  int64_t *total = (int64_t *)calloc(S, sizeof(int64_t));
  double *c_prev = (double *)calloc(S, sizeof(double));
  double *c_tr = (double *)calloc(S, sizeof(double));
  double *c_v = (double *)calloc(S, sizeof(double));
  int *success = (int *)calloc(S, sizeof(int));

#pragma omp parallel for schedule(dynamic)
  for (int s = 0; s < S; ++s) {
    c_prev[s] = FWD_COST(M, psi, phi, gates + GS * (size_t)s * L);
    c_tr[s] = c_prev[s];
    c_v[s] = Mv > 0 ? FWD_COST(Mv, psiv, phiv, gates + GS * (size_t)s * L) : c_tr[s];
  }

  int restarts = 0, m_total = M, chosen = -1;
  for (;;) {
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < S; ++s) {
      if (status[s] != ST_RUNNING) continue;
      qo_cplx *g = gates + GS * (size_t)s * L;
      if (d == 2)
        c_tr[s] = qo_sweep(n, L, pairs, kinds, M, psi, phi, g, p->beta,
                           p->beta_normalized ? 1.0 / (double)M : 1.0, NULL, NULL, NULL);
      else
        c_tr[s] = qd_sweep(d, n, L, pairs, kinds, M, psi, phi, g, p->beta,
                           p->beta_normalized ? 1.0 / (double)M : 1.0, NULL, NULL);
      c_v[s] = Mv > 0 ? FWD_COST(Mv, psiv, phiv, g) : c_tr[s];
    }
    const int full = (M == (int)N);
    int any_success = 0, any_over = 0, any_running = 0;
    for (int s = 0; s < S; ++s) {
      if (status[s] != ST_RUNNING) continue;
      iter[s] += 1;
      total[s] += 1;
      int t = -1;
      if (trace && trace->count < trace->capacity) {
        t = trace->count++;
        trace->start[t] = s;
        trace->sweep[t] = (int32_t)total[s];
        trace->m[t] = M;
        trace->c_train[t] = c_tr[s];
        trace->c_val[t] = c_v[s];
        if (trace->iter) trace->iter[t] = iter[s];
      }
      int ev = QO_EV_RUN;
      /* App. A, Eq. 13: relative improvement test over consecutive iterations. */
      int improved = fabs(c_prev[s]) - fabs(c_tr[s]) > p->diff_tol_r * fabs(c_tr[s]);
      zcount[s] = improved ? 0 : zcount[s] + 1;
      c_prev[s] = c_tr[s];
      /* Sec. 3, success relations: c_train < dist_tol and c_val / c_train <= 1 + otr. */
      int gen_ok = full || Mv == 0 || c_v[s] <= (1.0 + p->overtrain_ratio) * c_tr[s];
      if (c_tr[s] < p->dist_tol && gen_ok) {
        status[s] = ST_STOPPED;
        reason[s] = QO_SUCCESS;
        success[s] = 1;
        any_success = 1;
        ev = QO_EV_SUCCESS;
      } else if (iter[s] >= p->min_iter && !gen_ok && M < m_cap) {
        status[s] = ST_OVERTRAINED;
        any_over = 1;
        ev = QO_EV_OVERTRAINED;
      } else if (iter[s] >= p->min_iter && !gen_ok && c_tr[s] < p->dist_tol) {
        status[s] = ST_STOPPED;
        reason[s] = QO_NOT_GENERALIZED;
        ev = QO_EV_NOT_GEN;
      } else if (iter[s] >= p->min_iter && zcount[s] >= p->plateau_window) {
        status[s] = ST_STOPPED;
        reason[s] = QO_PLATEAU;
        ev = QO_EV_PLATEAU;
      } else if (total[s] >= p->max_iter) {
        status[s] = ST_STOPPED;
        reason[s] = QO_MAX_ITER;
        ev = QO_EV_MAX_ITER;
      }
      if (t >= 0 && trace->event) trace->event[t] = ev;
    }
    if (any_success) {
      double best = INFINITY;
      for (int s = 0; s < S; ++s)
        if (success[s] && c_tr[s] < best) {
          best = c_tr[s];
          chosen = s;
        }
      break;
    }
    if (any_over) {
      /* double-and-restart: extend the training set, keep every gate (App. A) */
      int M_new = 2 * M < m_cap ? 2 * M : m_cap;
      const int rec = trace && trace->dbl_count < trace->dbl_capacity ? trace->dbl_count++ : -1;
      const size_t all_gates = GS * (size_t)L * S;
      if (rec >= 0) {
        trace->dbl_m_old[rec] = M;
        trace->dbl_m_new[rec] = M_new;
        if (trace->dbl_gates_before)
          memcpy(trace->dbl_gates_before + rec * all_gates, gates, sizeof(qo_cplx) * all_gates);
      }
      if (target_kind == QO_TARGET_SAMPLES) {
        memcpy(psi, samples_psi, sizeof(qo_cplx) * (size_t)M_new * N);
        memcpy(phi, samples_phi, sizeof(qo_cplx) * (size_t)M_new * N);
      } else {
        if (any_extend(d, n, M, M_new, p->seed, psi) != 0) return -2;
        any_targets(d, n, target_kind, U, Lt, tpairs, tgates, M_new - M, psi + (size_t)M * N,
                    phi + (size_t)M * N);
        ++generation;
        Mv = p->m_val > 0 ? p->m_val : M_new;
        psiv = (qo_cplx *)realloc(psiv, sizeof(qo_cplx) * (size_t)Mv * N);
        phiv = (qo_cplx *)realloc(phiv, sizeof(qo_cplx) * (size_t)Mv * N);
        if (any_draw(d, n, Mv, p->seed, QO_ROLE_VAL, (uint32_t)generation, psiv) != 0)
          return -2;
        any_targets(d, n, target_kind, U, Lt, tpairs, tgates, Mv, psiv, phiv);
      }
      M = M_new;
      m_total += M;
      ++restarts;
#pragma omp parallel for schedule(dynamic)
      for (int s = 0; s < S; ++s) {
        if (status[s] == ST_STOPPED) continue;
        status[s] = ST_RUNNING;
        iter[s] = 0;
        zcount[s] = 0;
        c_prev[s] = FWD_COST(M, psi, phi, gates + GS * (size_t)s * L);
      }
      if (rec >= 0) {
        if (trace->dbl_gates_after)
          memcpy(trace->dbl_gates_after + rec * all_gates, gates, sizeof(qo_cplx) * all_gates);
        const int rows = M < trace->dbl_rows ? M : trace->dbl_rows;
        const size_t stride = (size_t)trace->dbl_rows * N;
        if (trace->dbl_psi) memcpy(trace->dbl_psi + rec * stride, psi, sizeof(qo_cplx) * (size_t)rows * N);
        if (trace->dbl_phi) memcpy(trace->dbl_phi + rec * stride, phi, sizeof(qo_cplx) * (size_t)rows * N);
        if (trace->dbl_c_prev)
          for (int s = 0; s < S; ++s)
            trace->dbl_c_prev[(size_t)rec * S + s] = status[s] == ST_STOPPED ? NAN : c_prev[s];
      }
      continue;
    }
    for (int s = 0; s < S; ++s)
      if (status[s] == ST_RUNNING) any_running = 1;
    if (!any_running) {
      double best = INFINITY;
      for (int s = 0; s < S; ++s)
        if (c_tr[s] < best) {
          best = c_tr[s];
          chosen = s;
        }
      break;
    }
  }

#undef FWD_COST
  memcpy(gates_out, gates + GS * (size_t)chosen * L, sizeof(qo_cplx) * GS * (size_t)L);
  res->reason = reason[chosen];
  res->m_final = M;
  res->sweeps = (int32_t)total[chosen];
  res->restarts = restarts;
  res->best_start = chosen;
  res->m_total = m_total;
  res->c_train = c_tr[chosen];
  res->c_val = c_v[chosen];
  res->seconds = qo_now() - t0;

  free(status); free(reason); free(iter); free(zcount); free(total);
  free(c_prev); free(c_tr); free(c_v); free(success);
  free(gates); free(psi); free(phi); free(psiv); free(phiv);
  return 0;
}

int qo_instantiate(int n, int L, const int32_t *pairs, const int32_t *kinds, const qo_cplx *fixed,
                   int target_kind, const qo_cplx *U, int Lt, const int32_t *tpairs,
                   const qo_cplx *tgates, const qo_cplx *samples_psi, const qo_cplx *samples_phi,
                   int n_samples, int n_val, const qo_params *p, const qo_cplx *gates_in,
                   qo_cplx *gates_out, qo_result *res, qo_trace *trace) {
  return instantiate_impl(2, n, L, pairs, kinds, fixed, target_kind, U, Lt, tpairs, tgates,
                          samples_psi, samples_phi, n_samples, n_val, p, gates_in, gates_out, res,
                          trace);
}

int qd_instantiate_target(int d, int n, int L, const int32_t *pairs, const int32_t *kinds,
                          const qo_cplx *fixed, int target_kind, const qo_cplx *U, int Lt,
                          const int32_t *tpairs, const qo_cplx *tgates, const qo_params *p,
                          const qo_cplx *gates_in, qo_cplx *gates_out, qo_result *res,
                          qo_trace *trace) {
  if (d < 2 || d > 4 || (target_kind != QO_TARGET_DENSE && target_kind != QO_TARGET_CIRCUIT)) return -1;
  if (target_kind == QO_TARGET_DENSE && !U) return -1;
  if (target_kind == QO_TARGET_CIRCUIT) {
    if (Lt < 0 || (Lt > 0 && (!tpairs || !tgates))) return -1;
    for (int k = 0; k < Lt; ++k) {
      const int a = tpairs[2 * k], b = tpairs[2 * k + 1];
      if (a < 0 || b < 0 || a >= n || b >= n || a == b) return -1;
    }
  }
  return instantiate_impl(d, n, L, pairs, kinds, fixed, target_kind, U, Lt, tpairs, tgates, NULL, NULL,
                          0, 0, p, gates_in, gates_out, res, trace);
}

int qd_instantiate(int d, int n, int L, const int32_t *pairs, const int32_t *kinds,
                   const qo_cplx *fixed, const qo_cplx *samples_psi, const qo_cplx *samples_phi,
                   int n_samples, int n_val, const qo_params *p, const qo_cplx *gates_in,
                   qo_cplx *gates_out, qo_result *res, qo_trace *trace) {
  if (d < 2 || d > 4) return -1;
  return instantiate_impl(d, n, L, pairs, kinds, fixed, QO_TARGET_SAMPLES, NULL, 0, NULL, NULL,
                          samples_psi, samples_phi, n_samples, n_val, p, gates_in, gates_out, res,
                          trace);
}
