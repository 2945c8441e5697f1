/*
 * qfs_oracle.h -- FP64 CPU oracle of QFactor-Sample instantiation
 * (Kukliansky et al., "Leveraging Quantum Machine Learning Generalization to
 * Significantly Speed-up Quantum Compilation", arXiv 2405.12866).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, obviously-correct reference used
 * by the test-suite, the smoke check and the CPU-baseline leg of the benchmark. It
 * shares no code, header, table or helper with the HIP implementation, and the
 * product path never loads it.
 *
 * Conventions (the paper fixes none of them; chosen once and pinned by the dense
 * brute-force tests):
 *   - n qubits, N = 2^n amplitudes. Qubit 0 is the MOST significant bit of the
 *     amplitude index (textbook Kronecker order): bit position of qubit q is n-1-q.
 *   - A two-qubit gate acts on the ordered pair (qa, qb), qa != qb. Its 4x4 matrix
 *     u[q][p] is row-major, q = output local index, p = input local index, and the
 *     local index of an amplitude is 2*bit(qa) + bit(qb).
 *   - Gates are applied in list order: C = u_{L-1} ... u_1 u_0.
 *   - A state set is [M][N] complex128 (sample-major, each state contiguous).
 *   - Environment Gamma_k[q][p] = sum_j sum_r a_j(q,r) conj(B_j(p,r)); the paper's
 *     environment E (Sec. 3, Eq. 10 and Sec. 2.1, Eq. 2) is Gamma^dagger, so the
 *     update u = Y X^dagger with E = X D Y^dagger is u = W V^dagger with
 *     Gamma = W S V^dagger, i.e. the unitary polar factor of Gamma.
 */
#ifndef QFS_ORACLE_H
#define QFS_ORACLE_H

#include <complex.h>
#include <stdint.h>

typedef double _Complex qo_cplx;

/* Random-number roles (counter word 2 of Philox). */
enum { QO_ROLE_TRAIN = 1, QO_ROLE_VAL = 2, QO_ROLE_INIT = 3 };

/* Target kinds. */
enum { QO_TARGET_DENSE = 0, QO_TARGET_CIRCUIT = 1, QO_TARGET_SAMPLES = 2 };

/* Gate kinds of a template (Sec. 2.1: QFactor updates gates of any size directly as
 * unitaries; Sec. 4: the evaluated circuits hold U3 and CNOT gates).
 *   QO_GATE_2Q:    variable two-qubit gate on (qa, qb), any 4x4 unitary.
 *   QO_GATE_1Q:    variable one-qubit gate v on qubit qa; qb is a spectator qubit and the
 *                  gate's 4x4 slot holds v (x) I_2 in the local basis of (qa, qb).
 *   QO_GATE_FIXED: constant 4x4 gate on (qa, qb): applied, never updated.
 * A NULL kinds array means every gate is QO_GATE_2Q. */
enum { QO_GATE_2Q = 0, QO_GATE_1Q = 1, QO_GATE_FIXED = 2 };

/* Termination reasons (the paper's termination kinds, Sec. 4 per-run runtimes). */
enum {
  QO_SUCCESS = 0,
  QO_PLATEAU = 1,
  QO_MAX_ITER = 2,
  QO_NOT_GENERALIZED = 3,
  QO_TIMEOUT = 4
};

typedef struct {
  double dist_tol;        /* App. A: dist_tol                                  */
  double diff_tol_r;      /* App. A: diff_tol_r (plateau relative improvement) */
  int32_t plateau_window; /* App. A: plateau_windows_size                      */
  int32_t min_iter;       /* App. A: min_iter                                  */
  int64_t max_iter;       /* App. A: max_iter (total sweeps per start)         */
  int32_t m_init;         /* App. A: number_of_training_states                 */
  int32_t m_max;          /* cap on M; 0 means 2^n (Sec. 3)                    */
  double overtrain_ratio; /* App. A: overtrain_ratio                           */
  int32_t multistarts;    /* App. A: multistarts                               */
  double beta;            /* App. A: Beta (regularised update)                 */
  uint64_t seed;          /* App. A: seed                                      */
  int32_t fixed_m;        /* 1: never double M                                 */
  int32_t m_val;          /* validation-set size; 0 means M                    */
  int32_t beta_normalized; /* 1: mix the environment divided by M with u       */
} qo_params;

typedef struct {
  int32_t reason;
  int32_t m_final;
  int32_t sweeps;     /* sweeps of the returned start                          */
  int32_t restarts;   /* number of doublings                                   */
  int32_t best_start;
  int32_t m_total;    /* sum of the M values used, one entry per training set  */
  double c_train;
  double c_val;
  double seconds;
} qo_result;

/* Control decision taken for a start after one of its sweeps (trace->event). */
enum {
  QO_EV_RUN = 0,         /* keeps running                                         */
  QO_EV_SUCCESS = 1,     /* success relations of Sec. 3 hold                      */
  QO_EV_OVERTRAINED = 2, /* generalisation test failed while M may still grow     */
  QO_EV_NOT_GEN = 3,     /* generalisation test failed at the M cap below dist_tol */
  QO_EV_PLATEAU = 4,
  QO_EV_MAX_ITER = 5
};

/* Optional per-sweep trace: one row per (start, sweep). Every array except the first
 * five may be NULL. */
typedef struct {
  int32_t capacity;
  int32_t count;
  int32_t *start;     /* [capacity] */
  int32_t *sweep;     /* [capacity] total sweep index of that start (1-based) */
  int32_t *m;         /* [capacity] */
  double *c_train;    /* [capacity] */
  double *c_val;      /* [capacity] */
  int32_t *iter;      /* [capacity] sweep index since the last restart (1-based)   */
  int32_t *event;     /* [capacity] QO_EV_* decision taken after that sweep        */
  /* Record of each double-and-restart (Sec. 3; App. A), up to dbl_capacity of them.
   * gates: [dbl_capacity][multistarts][L][D*D] (D = d^2); states: [dbl_capacity]
   * [dbl_rows][N] (the first min(M_new, dbl_rows) rows are written). */
  int32_t dbl_capacity;
  int32_t dbl_count;
  int32_t dbl_rows;
  int32_t *dbl_m_old;         /* [dbl_capacity] M before the doubling               */
  int32_t *dbl_m_new;         /* [dbl_capacity] M after it                          */
  qo_cplx *dbl_gates_before;  /* every start's gates when the doubling is decided   */
  qo_cplx *dbl_gates_after;   /* every start's gates when the new set's sweeps begin */
  qo_cplx *dbl_psi;           /* training states after the doubling                 */
  qo_cplx *dbl_phi;           /* U psi of those states                              */
  double *dbl_c_prev;         /* [dbl_capacity][multistarts] plateau reference c_0 on
                                 the new set (NaN for a start that had stopped)     */
} qo_trace;

/* Counter-based generator Philox4x32-10 (Salmon et al., SC'11). */
void qo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Standard complex normal (E|z|^2 = 1) for (seed, role, stream, index). */
qo_cplx qo_cgauss(uint64_t seed, uint32_t role, uint32_t stream, uint64_t idx);
/* Complex Ginibre matrix, column-major rows x cols: entry (i, j) uses index j*rows+i. */
void qo_ginibre(int64_t rows, int64_t cols, uint64_t seed, uint32_t role, uint32_t stream,
                qo_cplx *out /* [cols][rows] */);
/* Q of the QR factorisation with real positive diag(R) (Mezzadri 2007), in place on
 * column-major columns; returns 0, or -1 if a column is numerically dependent. */
int qo_orthonormalize(int64_t rows, int64_t cols, qo_cplx *cols_inout);
/* Training / validation sample states: first M columns of a Haar unitary (Sec. 3,
 * App. A). Training columns come from one fixed Ginibre stream so that the set for
 * 2M extends the set for M. Validation uses stream `generation`. */
int qo_draw_states(int n, int M, uint64_t seed, uint32_t role, uint32_t stream,
                   qo_cplx *out /* [M][N] */);
/* Haar-random 4x4 initial gate (App. A, multistarts and seed). */
void qo_haar_gate(uint64_t seed, uint32_t start, uint32_t gate, qo_cplx u[16]);
/* Haar-random 2x2 initial gate of a one-qubit gate, row-major. */
void qo_haar_gate2(uint64_t seed, uint32_t start, uint32_t gate, qo_cplx v[4]);
/* Initial 4x4 slot of gate `gate` of start `start` by kind: a Haar 4x4, v (x) I_2 with a
 * Haar 2x2 v, or the constant gate fixed[gate] (fixed: [L][16], read for FIXED only). */
void qo_initial_gate(uint64_t seed, uint32_t start, uint32_t gate, int kind,
                     const qo_cplx *fixed, qo_cplx u[16]);

void qo_apply_gate(int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx u[16]);
void qo_apply_gate_dag(int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx u[16]);
void qo_apply_circuit(int n, int M, qo_cplx *st, int L, const int32_t *pairs,
                      const qo_cplx *gates);
void qo_dense_apply(int n, int M, const qo_cplx *U /*[N][N] row-major*/,
                    const qo_cplx *psi, qo_cplx *out);
void qo_environment(int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, int qb,
                    qo_cplx G[16]);
/* Environment of a one-qubit gate on qubit qa: G[q][p] = sum_j sum_r a_j(q,r) conj(b_j(p,r))
 * over the other n-1 qubits r (2x2, row-major). */
void qo_environment1(int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, qo_cplx G[4]);
/* 4x4 complex SVD G = W diag(s) V^dagger by one-sided (Hestenes) Jacobi. */
void qo_svd4(const qo_cplx G[16], qo_cplx W[16], double s[4], qo_cplx V[16]);
/* Update of one gate: u <- polar((1-beta) Gamma + beta u). */
void qo_update_gate(const qo_cplx G[16], double beta, qo_cplx u[16]);
/* Update of a one-qubit gate stored as v (x) I_2 in u: v <- polar((1-beta) G + beta v). */
void qo_update_gate1(const qo_cplx G[4], double beta, qo_cplx u[16]);
double qo_state_distance(int n, int M, const qo_cplx *x, const qo_cplx *y);

/* One sweep (forward B list, right-to-left update). Returns c_train after the sweep.
 * kinds: [L] or NULL (all QO_GATE_2Q). gamma_scale multiplies each environment before the
 * regularised mix (1: the paper's form; 1/M: normalised). Optional outputs: per gate
 * f = Re Tr(G^dagger u)
 * before/after its update (NaN for a fixed gate), and each environment G ([L][16]; a
 * one-qubit gate's 2x2 in the first 4 entries, a fixed gate's all zero). */
double qo_sweep(int n, int L, const int32_t *pairs, const int32_t *kinds, int M,
                const qo_cplx *psi, const qo_cplx *phi, qo_cplx *gates, double beta,
                double gamma_scale, double *f_before, double *f_after, qo_cplx *gammas);

/* Qudits (n of dimension d, 2 <= d <= 4; N = d^n, qudit 0 the most significant base-d
 * digit; a two-qudit gate on (qa, qb) is D x D, D = d^2, local index d digit(qa) +
 * digit(qb)). With d = 2 these compute what the qubit functions compute. */
void qd_apply_gate(int d, int n, int M, qo_cplx *st, int qa, int qb, const qo_cplx *u, int dagger);
void qd_environment(int d, int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, int qb,
                    qo_cplx *G /* [D][D] */);
void qd_svd(int D, const qo_cplx *G, qo_cplx *W, double *s, qo_cplx *V);
void qd_update_gate(int D, const qo_cplx *G, double beta, qo_cplx *u);
/* Haar D x D initial gate from indices 256 gate + D col + row of the start's stream. */
void qd_haar_gate(int d, uint64_t seed, uint32_t start, uint32_t gate, qo_cplx *u);
/* Gate kinds on qudits (the qubit kinds with d levels): a one-qudit gate v on qa with qb a
 * spectator is held as the D x D slot v (x) I_d (entry (d x + z, d y + w) = v[x][y] when
 * z = w), updated from its d x d environment; a constant gate is applied, never updated.
 * qd_environment1: G[x][y] = sum_j sum_r a_j(x, r) conj(b_j(y, r)) over the other n-1
 * qudits. qd_haar_gate1: Haar on U(d) from the d x d Ginibre block at indices
 * 256 gate + d col + row of the start's stream, as a slot. */
void qd_environment1(int d, int n, int M, const qo_cplx *a, const qo_cplx *b, int qa, qo_cplx *G);
void qd_update_gate1(int d, const qo_cplx *G1, double beta, qo_cplx *u);
void qd_haar_gate1(int d, uint64_t seed, uint32_t start, uint32_t gate, qo_cplx *u);
/* kinds: [L] or NULL (all QO_GATE_2Q); f_before/f_after as for qo_sweep. */
double qd_sweep(int d, int n, int L, const int32_t *pairs, const int32_t *kinds, int M,
                const qo_cplx *psi, const qo_cplx *phi, qo_cplx *gates, double beta,
                double gamma_scale, double *f_before, double *f_after);
/* Instantiation on a fixed sample set (rows 0 .. n_samples - n_val - 1 train, the last
 * n_val validate), the same control loop as qo_instantiate. */
int qd_instantiate(int d, int n, int L, const int32_t *pairs, const int32_t *kinds,
                   const qo_cplx *fixed, const qo_cplx *samples_psi, const qo_cplx *samples_phi,
                   int n_samples, int n_val, const qo_params *p, const qo_cplx *gates_in,
                   qo_cplx *gates_out, qo_result *res, qo_trace *trace);

/* M orthonormal Haar states on N = d^n amplitudes, drawn as qo_draw_states draws them for
 * N = 2^n (column j of the Ginibre matrix from Philox index j N + i, orthonormalised in
 * column order). out: [M][N]. */
int qd_draw_states(int d, int n, int M, uint64_t seed, uint32_t role, uint32_t stream,
                   qo_cplx *out);
/* Instantiation against a dense target U ([N][N] row-major) or a target circuit
 * of Lt two-qudit gates (tpairs [Lt][2], tgates [Lt][D][D]) with states drawn as in
 * qo_instantiate (N = d^n amplitudes, the same Philox roles, streams and indices),
 * the same control loop. kinds and fixed ([L][D][D], read for QO_GATE_FIXED) as for
 * qo_instantiate. */
int qd_instantiate_target(int d, int n, int L, const int32_t *pairs, const int32_t *kinds,
                          const qo_cplx *fixed, int target_kind, const qo_cplx *U, int Lt,
                          const int32_t *tpairs, const qo_cplx *tgates, const qo_params *p,
                          const qo_cplx *gates_in, qo_cplx *gates_out, qo_result *res,
                          qo_trace *trace);

/* Full instantiation with the paper's control loop. kinds: [L] or NULL; fixed: [L][16]
 * constant gates (read for QO_GATE_FIXED; replace those slots of gates_in too). */
int qo_instantiate(int n, int L, const int32_t *pairs, const int32_t *kinds,
                   const qo_cplx *fixed, int target_kind,
                   const qo_cplx *U, int Lt, const int32_t *tpairs, const qo_cplx *tgates,
                   const qo_cplx *samples_psi, const qo_cplx *samples_phi, int n_samples,
                   int n_val, const qo_params *p, const qo_cplx *gates_in,
                   qo_cplx *gates_out, qo_result *res, qo_trace *trace);

#endif
