/*
 * qfs.h -- C ABI of the MI355X (gfx950) implementation of QFactor-Sample instantiation
 * (Kukliansky et al., "Leveraging Quantum Machine Learning Generalization to
 * Significantly Speed-up Quantum Compilation", arXiv 2405.12866).
 *
 * Library: libqfs_hip.so (HIP, gfx950). Plain C types only; no exception crosses this
 * boundary; every function returns an error code (QFS_OK = 0) unless stated.
 *
 * Conventions, shared by every entry point:
 *   - n qubits, N = 2^n amplitudes; qubit 0 is the MOST significant bit of the
 *     amplitude index (textbook Kronecker order).
 *   - A template is an ordered list of L two-qubit gates; gate k acts on the ordered
 *     qubit pair (pairs[2k], pairs[2k+1]), distinct and in [0, n). Gates are applied
 *     in list order: C = u_{L-1} ... u_0.
 *   - A gate is a 4x4 complex matrix stored row-major, u[q][p] (q output, p input
 *     local index), local index = 2*bit(first qubit) + bit(second qubit). Gate
 *     tensors are [L][4][4] qfs_c128 (interleaved re, im doubles).
 *   - A state set is [M][N] qfs_c128, sample-major (each state contiguous).
 *   - "device" pointers are HIP device memory of the current device; "host" pointers
 *     are ordinary host memory. Every pointer is caller-owned, used only during the
 *     call and never retained. Outputs are defined only when the call returns QFS_OK.
 *   - Calls are stream-ordered on params->hip_stream (or the stream argument; NULL is
 *     the null stream) and return after the work has completed unless stated.
 *   - Random draws use the counter-based generator Philox4x32-10 (Salmon et al., SC'11)
 *     keyed by the 64-bit seed; a complex standard normal is formed from one Philox
 *     block by the Box-Muller transform. Counter words: (index lo, index hi, role,
 *     stream). Ginibre entry (row i, column j) of an R-row matrix has index j*R + i.
 */
#ifndef QFS_H
#define QFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} qfs_c128;

/* ---------------------------------------------------------------- error codes */
enum {
  QFS_OK = 0,
  QFS_EINVAL = 1,       /* bad argument: n < 2 or n > 24, pair out of range or equal,
                           M > 2^n, non-finite or non-unitary input gate, ...        */
  QFS_ENOMEM = 2,       /* does not fit the device-memory budget even with one start */
  QFS_EDEVICE = 3,      /* a HIP runtime error; see qfs_last_error_detail()          */
  QFS_EUNSUPPORTED = 4, /* a combination the library does not implement             */
  QFS_ENUMERIC = 5      /* orthonormalisation of a drawn sample set failed            */
};

/* Human-readable text of an error code (static storage). */
const char *qfs_strerror(int code);
/* Detail of the most recent error on the calling thread (static per thread). */
const char *qfs_last_error_detail(void);
/* Library version string. */
const char *qfs_version(void);
/* Device memory kept between calls. When a call of qfs_instantiate (and of the entry
 * points built on it: qfs_instantiate_samples, the learned single-problem entry) ends, the
 * library keeps its device buffers, up to an eighth of the device's memory, and reuses
 * them in later calls that need buffers of the same sizes, instead of freeing and
 * allocating them again. An allocation that fails frees the kept buffers first, and the
 * free-memory budget of a call counts them as free. This frees the buffers kept for the
 * current device and stores their total size in *bytes_freed (may be null). Blocks are
 * kept only once the device has finished with them, so it may be called at any time, from
 * any thread. Returns QFS_OK or QFS_EDEVICE. */
int qfs_release_device_cache(size_t *bytes_freed);

/* ---------------------------------------------------------------- problem */
/* Gate kinds (Sec. 2.1: QFactor updates gates of any size directly as unitaries;
 * Sec. 4: the instantiated partitions are U3 + CNOT circuits).
 *   QFS_GATE_2Q:    variable two-qubit gate on (a, b): any 4x4 unitary, updated to the
 *                   polar factor of its 4x4 environment.
 *   QFS_GATE_1Q:    variable one-qubit gate v on qubit a; b is any other qubit (a
 *                   spectator). Its 4x4 slot holds v (x) I_2 in the local basis of
 *                   (a, b) and keeps that form: v is updated to the polar factor of the
 *                   2x2 environment sum_j sum_r a_j(q, r) conj(B_j(p, r)) over the other
 *                   n-1 qubits (read v as slot[2q][2p]).
 *   QFS_GATE_FIXED: constant 4x4 gate on (a, b) (a CNOT; a constant one-qubit gate as
 *                   w (x) I_2): applied in both passes, never updated. */
enum { QFS_GATE_2Q = 0, QFS_GATE_1Q = 1, QFS_GATE_FIXED = 2 };

/* Circuit template: L gates applied in list order, gate k on the ordered qubit pair
 * pairs[k] (a != b; local index 2 bit(a) + bit(b), qubit 0 the most significant bit).
 * kinds == NULL means every gate is QFS_GATE_2Q. fixed_gates holds the constant gates
 * (device [n_gates][4][4]; only the QFS_GATE_FIXED entries are read, every start gets
 * them); it may be NULL when no gate is constant. A target circuit's kinds and
 * fixed_gates are ignored (its gates are all given). */
typedef struct {
  int32_t n_qubits;
  int32_t n_gates;
  const int32_t *pairs;         /* host, [n_gates][2]                        */
  const int32_t *kinds;         /* host, [n_gates] or NULL                   */
  const qfs_c128 *fixed_gates;  /* device, [n_gates][4][4] or NULL           */
} qfs_template;

enum { QFS_TARGET_DENSE = 0, QFS_TARGET_CIRCUIT = 1, QFS_TARGET_SAMPLES = 2 };

/* Target of an instantiation (Sec. 2.3: training pairs (psi, U psi)).
 *   DENSE:   U, device [N][N] row-major.
 *   CIRCUIT: circuit (host template) + circuit_gates (device [Lt][4][4]); U psi is
 *            formed by simulating that circuit.
 *   SAMPLES: psi, phi device [n_samples][N]; rows 0 .. n_samples-n_val-1 are the
 *            training pairs (used in order; doubling takes more of them), the last
 *            n_val rows the validation pairs (n_val = 0: no generalisation test). */
typedef struct {
  int32_t kind;
  const qfs_c128 *U;
  const qfs_template *circuit;
  const qfs_c128 *circuit_gates;
  const qfs_c128 *psi;
  const qfs_c128 *phi;
  int32_t n_samples;
  int32_t n_val;
} qfs_target;

enum { QFS_PREC_FP64 = 0, QFS_PREC_MIXED = 1 };

/* Hyperparameters (App. A; defaults are the paper's recommended values) plus the
 * execution controls of this implementation. */
typedef struct {
  double dist_tol;           /* success threshold on c_train (App. A: dist_tol)      */
  double diff_tol_r;         /* plateau relative improvement (App. A, Eq. 13)        */
  int32_t plateau_window;    /* consecutive non-improving sweeps (App. A)            */
  int32_t min_iter;          /* sweeps before plateau/overtraining tests (App. A)    */
  int64_t max_iter;          /* total sweeps per start (App. A)                      */
  int32_t m_init;            /* initial number of training states (App. A)           */
  int32_t m_max;             /* cap on M; 0 = 2^n (Sec. 3)                           */
  double overtrain_ratio;    /* c_val / c_train - 1 threshold (Sec. 3, App. A)       */
  int32_t multistarts;       /* independent random starts (App. A)                   */
  double beta;               /* regularised update (App. A); 0 = full update         */
  uint64_t seed;             /* seeds states, validation states and initial gates    */
  int32_t fixed_m;           /* 1: never double M                                    */
  int32_t m_val;             /* validation-set size; 0 = M                           */
  int32_t precision;         /* QFS_PREC_FP64: complex128 states throughout.
                                QFS_PREC_MIXED: complex64 states with FP64
                                environment sums, polar update and cost, and
                                complex128 refinement sweeps once the best running
                                start's c_train drops below refine_below.           */
  double refine_below;       /* MIXED: refinement threshold (default 1e-5)           */
  uint64_t device_mem_budget;/* bytes the call may allocate; 0 = free device memory  */
  double time_budget_s;      /* wall-clock budget; 0 = none (reason TIMEOUT)         */
  void *hip_stream;          /* hipStream_t for all work; NULL = null stream          */
  int32_t timing;            /* 1: time every sweep kernel with hipEvents on
                                hip_stream and report it in qfs_result             */
  int32_t batch_sweeps;      /* qfs_instantiate_batch: sweeps per persistent launch
                                (0 = automatic: 8, doubled up to 256 while fewer
                                than 1/4, 1/8, ... of the jobs still run; 1 keeps
                                every start of a problem in lock step, as
                                qfs_instantiate does)                               */
  int32_t batch_threads;     /* qfs_instantiate_batch: work-group size 64, 128 or 256
                                (0 = chosen by the built-in autotuner, cached per
                                precision and state-size class for the process)     */
  int32_t graphs;            /* qfs_instantiate: 1 replays each sweep's launches as
                                a captured HIP graph on an internal stream
                                (re-captured when the running starts, M or the
                                precision change); 0 (default) launches every
                                kernel, which measured faster on MI355X / ROCm 7   */
  int32_t full_unitary;      /* qfs_instantiate: 1 runs full-unitary QFactor
                                (Sec. 2.1): the training set is the complete
                                computational basis (M = 2^n, no validation set),
                                so c_train is the full distance (Eq. 1 / 2^n) and
                                each sweep is QFactor's; DENSE and CIRCUIT targets
                                only; m_init, fixed_m and m_val are ignored        */
  int32_t beta_normalized;   /* 1: the regularised update (App. A Beta) mixes the
                                environment divided by the current M with the gate,
                                polar((1 - beta) Gamma / M + beta u), so beta keeps
                                its meaning as M changes; 0: the paper's form       */
  int32_t backward_mode;     /* QFS_BWD_GROUPED (default): consecutive gates whose
                                qubits fit in four share one pass over the backward
                                state (Sec. 3 right-to-left update, Fig.
                                env_calc_tensor): the pass reduces one 16 x 16
                                second-moment matrix of the state entering the group
                                and the forward state before it, and every gate's
                                environment follows from it in order; the forward
                                pass stores one B list entry per group.
                                QFS_BWD_PER_GATE: one pass per gate. Both give the
                                same gates to rounding; templates on fewer than 3
                                qubits always take the per-gate passes.             */
} qfs_params;

enum { QFS_BWD_GROUPED = 0, QFS_BWD_PER_GATE = 1 };

/* Termination reasons (the paper's run outcomes: success, distance not reached,
 * timeout). */
enum {
  QFS_SUCCESS = 0,
  QFS_PLATEAU = 1,
  QFS_MAX_ITER = 2,
  QFS_NOT_GENERALIZED = 3, /* c_train < dist_tol but c_val / c_train > 1 + otr at m_max */
  QFS_TIMEOUT = 4
};

typedef struct {
  int32_t reason;
  int32_t m_final;           /* M of the last training set                         */
  int32_t sweeps;            /* sweeps run by the returned start                   */
  int32_t restarts;          /* doublings                                          */
  int32_t best_start;        /* index of the returned start                        */
  int32_t m_total;           /* sum of M over the training sets used               */
  int32_t start_groups;      /* multistart groups run (> 1 when memory was split)  */
  int32_t refined;           /* 1 if complex128 refinement sweeps ran              */
  double c_train;            /* Eq. 9 cost of the returned gates on the training set */
  double c_val;              /* same on the validation set                         */
  double seconds;            /* wall time of the call                              */
  int64_t start_sweeps;      /* sum over starts of sweeps run (throughput count)   */
  double sweep_seconds;      /* device time spent in sweeps (hipEvent)             */
  /* With params->timing: per kernel class, launches, summed hipEvent durations and
   * the bytes the kernels must move (state reads + writes). Class 0: backward step
   * (apply u^dagger + environment partial sums); class 1: forward pass (B list and
   * validation states); class 2: distance (cost) kernels; class 3: environment
   * reduction + FP64 polar update. */
  int64_t kernel_launches[4];
  double kernel_seconds[4];
  double kernel_bytes[4];
  /* Learned entries only (qfs_instantiate_learned, qfs_instantiate_batch_learned):
   * the predicted initial M, the starts run (learned run plus fallback), and 1 when the
   * learned run did not succeed and the plain method was run after it. */
  int32_t m_predicted;
  int32_t starts_run;
  int32_t fallback;
  /* Device work of the call (or of the problem, batched): sum over start-sweeps of
   * (M + M_val) 2^n L, the amplitude-gate updates of one sweep's forward and backward
   * passes at the M of that sweep. */
  double amp_updates;
} qfs_result;

/* Fill *p with the defaults: dist_tol 1e-8, diff_tol_r 1e-5, plateau_window 5,
 * min_iter 6, max_iter 1e4, m_init 2, overtrain_ratio 0.1, multistarts 16, beta 0
 * (App. A recommended values); precision MIXED, refine_below 1e-5, seed 0. */
void qfs_default_params(qfs_params *p);

/* QFactor-Sample instantiation with the paper's control loop (Sec. 3, App. A):
 * draw M orthonormal Haar sample states, form U psi, and sweep every running start
 * right to left (environment, SVD, unitary polar update) until success, plateau,
 * max_iter or timeout; double M and restart (keeping the gates) when the
 * normalised generalisation error exceeds overtrain_ratio. When the plan does not
 * fit device_mem_budget the multistarts are run in halves, recursively (App. A).
 *   gates_in:  device [multistarts][L][4][4], or NULL for Haar-random initial gates
 *              drawn from params->seed (role 3, stream = start, index 16*gate + 4*col
 *              + row of a column-major 4x4 Ginibre block; a one-qubit gate takes
 *              v (x) I_2 with v from the 2x2 block at indices 16*gate + 2*col + row).
 *              Constant gates always come from tmpl->fixed_gates; a one-qubit gate's
 *              entry must have the form v (x) I_2 (to 1e-10) and is used as exactly
 *              that form, v taken from its entries (2i, 2j).
 *   gates_out: device [L][4][4]: the returned start's gates (complex128).
 *   res:       host.
 * Errors: QFS_EINVAL (invalid template/target/params, or gates_in not unitary to
 * 1e-10), QFS_ENOMEM, QFS_EDEVICE, QFS_ENUMERIC. */
int qfs_instantiate(const qfs_template *tmpl, const qfs_target *target,
                    const qfs_params *params, const qfs_c128 *gates_in,
                    qfs_c128 *gates_out, qfs_result *res);

/* Batched instantiation of P independent problems, each with params->multistarts
 * starts (Sec. 3 and App. A per problem), in persistent launches: every
 * (problem, start) job is one work-group that keeps its two working state sets in LDS
 * (per-work-group global scratch when they exceed 128 KB) and recovers the forward
 * intermediate states during the backward pass with the gates as they were before the
 * sweep. Control decisions run on the device after every sweep; doublings and the
 * complex128 refinement switch happen between launches. Problem p uses seed
 * params->seed + p. With batch_sweeps = 1 every problem follows qfs_instantiate's
 * lock-step control flow; with batch_sweeps = K > 1 the starts of a problem advance up
 * to K sweeps independently, a success or overtraining found by one start at its sweep
 * count t takes effect at t (slower starts run on to t), and the decision at t is lock
 * step's; a start that had already run past t resumes from its later state after a
 * doubling. MIXED precision switches each start to complex128 on its own
 * (qfs_instantiate switches all starts together).
 *   tmpl, targets: host arrays [P] (targets' device pointers as in qfs_instantiate).
 *   gates_out: host array [P] of device pointers [L_p][4][4] (NULL entries skipped).
 *   res: host [P].
 * Templates may hold one-qubit and constant gates (kinds, fixed_gates as in
 * qfs_instantiate; initial one-qubit gates drawn the same way).
 * Limits: 2 <= n_qubits <= 10 per problem (QFS_EUNSUPPORTED above). */
int qfs_instantiate_batch(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                          const qfs_params *params, qfs_c128 *const *gates_out, qfs_result *res);

/* qfs_instantiate_batch with per-problem initial M and start counts: m_init host [P]
 * (NULL: params->m_init for every problem; each entry >= 1, capped at m_max and 2^n)
 * and starts host [P] (NULL: params->multistarts; problem p runs its first starts[p]
 * starts, 1 <= starts[p] <= multistarts). QFS_EINVAL for an entry out of range. */
int qfs_instantiate_batch_ex(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                             const qfs_params *params, const int32_t *m_init,
                             const int32_t *starts, qfs_c128 *const *gates_out,
                             qfs_result *res);

/* Labelling runs for the sample-count predictor: every problem at a fixed M =
 * params->m_init (no doubling), every start run to its own stop (no start waits for or
 * stops at another's success), Sec. 3 success relation per start. successes: host [P],
 * the number of starts that succeeded; res: host [P] (reason and costs of the best
 * start). Other arguments and limits as qfs_instantiate_batch. */
int qfs_label_batch(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                    const qfs_params *params, int32_t *successes, qfs_result *res);

/* ------------------------------------------- learned initial M and start pruning */
/* The paper leaves the initial number of training states open (Sec. 3, Sec. 5) and
 * relates the number needed to the parameter count per amplitude (Sec. 4). A network
 * 64 -> 128 -> 128 -> 2 (ReLU; bfloat16 weights, FP32 accumulation; process-wide, one
 * per process, guarded by a mutex) maps structural template features to
 *   y0: log2 of the smallest power-of-two M at which a start succeeds, and
 *   y1: the logit of the chance that one random start succeeds at that M.
 * The network was fitted on templates of two-qubit gates: every entry below that takes
 * a template returns QFS_EUNSUPPORTED for one with other gate kinds. */

/* The 64 features of a template (host; no device work). out: host [64]. */
int qfs_features(const qfs_template *tmpl, float *out);

/* Number of FP32 parameters: W1 [128][64], b1 [128], W2 [128][128], b2 [128],
 * W3 [2][128], b3 [2], in this order. */
int qfs_mlp_num_params(void);

/* He-uniform weights from a seed; resets the optimiser state. */
int qfs_mlp_init(uint64_t seed);

/* Copy the FP32 master weights out (host [num_params]) or in (resets the optimiser). */
int qfs_mlp_get(float *host_params);
int qfs_mlp_set(const float *host_params);

/* Weight file: 8-byte magic "QFSMLP1\0" then num_params little-endian FP32. */
int qfs_mlp_save(const char *path);
int qfs_mlp_load(const char *path);

/* Forward pass: features device [count][64] -> out device [count][2]. */
int qfs_mlp_forward(int32_t count, const float *features, float *out, void *hip_stream);

/* Gradient of the mean loss over count rows (no update): targets device [count][2] =
 * (log2 M label, NaN when there is none; success fraction in [0, 1]). Loss per row:
 * (y0 - t0)^2 / 2 when t0 is finite, plus the binary cross-entropy of logit y1 against
 * t1. grad_host: host [num_params] or NULL; loss_host: host or NULL. */
int qfs_mlp_grad(int32_t count, const float *features, const float *targets,
                 float *grad_host, float *loss_host, void *hip_stream);

/* Adam (0.9, 0.999, 1e-8) on shuffled mini-batches of `batch` rows for `epochs`
 * passes; features / targets as in qfs_mlp_grad (device). epoch_loss: host [epochs]
 * (mean mini-batch loss before each step) or NULL. */
int qfs_mlp_train(int32_t count, const float *features, const float *targets,
                  int32_t epochs, int32_t batch, float lr, uint64_t seed, float *epoch_loss,
                  void *hip_stream);

/* Predicted initial M (a power of two in [2, 2^n]) and the starts to keep: with the
 * predicted per-start success rate p, the number k of leading starts (1 <= k <=
 * params->multistarts = S) that minimises k + (1 - p)^k (S - k), the expected start-runs
 * when the pruned starts run only if all kept ones fail. keep_mask bit s = start s kept
 * (nullable). QFS_EINVAL when no weights are loaded. */
int qfs_predict_m(const qfs_template *tmpl, const qfs_params *params, int32_t *m0,
                  uint32_t *keep_mask);
int qfs_predict_batch(int32_t P, const qfs_template *tmpl, const qfs_params *params,
                      int32_t *m0, int32_t *starts);

/* qfs_instantiate with M starting at max(m_init, predicted M) (doubling on the
 * validation cost as usual, Sec. 3) and a number of leading starts chosen for wall time:
 * one problem's starts run together, so a sweep takes about T0 + k b / BW for k starts
 * (T0 the sweep's serial chain, about 17.5 us per gate; BW about 3.7 TB/s; b = (2L + 1)
 * M 2^n 8 bytes per start), and k minimises the expected time with the predicted
 * per-start success rate (the pruned starts run after a failed first run), pruning only
 * when that saves at least a tenth of the time of all starts. When
 * that run does not succeed and starts were pruned, the pruned starts run after it
 * with the plain method's control from the M the first run ended at (their own initial
 * gates), fallback = 1, and the better of the two runs is returned (success first, then
 * lower c_train). Counters in res (start_sweeps, m_total, sweep_seconds, seconds) cover
 * both runs. */
int qfs_instantiate_learned(const qfs_template *tmpl, const qfs_target *target,
                            const qfs_params *params, qfs_c128 *gates_out, qfs_result *res);

/* The same for qfs_instantiate_batch, in one batched run: each problem starts with its
 * predicted M and kept starts; its pruned starts are parked and woken inside the run
 * (from the problem's current training set, their own initial gates) as soon as every
 * kept start has stopped without success, or for every problem at once when fewer jobs
 * than two per compute unit are left running (the device would otherwise idle).
 * fallback = 1 when they were woken. */
int qfs_instantiate_batch_learned(int32_t P, const qfs_template *tmpl,
                                  const qfs_target *targets, const qfs_params *params,
                                  qfs_c128 *const *gates_out, qfs_result *res);

/* Minimal entry: fixed sample set of M pairs (psi, phi = U psi; device [M][N]), one
 * start, App. A defaults, no validation set, FP64 states, dist_tol = tol. Writes the
 * gates (device [L][4][4]) and the final Eq. 9 cost (host double). */
int qfs_instantiate_samples(const qfs_template *tmpl, const qfs_c128 *psi,
                            const qfs_c128 *phi, int32_t M, double tol,
                            qfs_c128 *gates_out, double *cost_out);

/* ------------------------------------------------------------------ qudits */
/* QFactor-Sample on n qudits of dimension d (Sec. 5: the method applies unchanged to
 * d-level gates; a sweep costs O(M d^n) where QFactor's costs O(d^{2n})). Qudit 0 is the
 * most significant base-d digit of the amplitude index (N = d^n); tmpl->n_qubits is the
 * qudit count, tmpl->pairs the ordered qudit pairs; a gate is a D x D unitary, D = d^2,
 * row-major u[q][p] with local index d digit(a) + digit(b). d = 2, 3 or 4; d^n <= 2^24.
 * Gate kinds as for qubits (tmpl->kinds, NULL: every gate QFS_GATE_2Q): a QFS_GATE_1Q gate
 * v on qudit a (b a spectator) is held as the slot v (x) I_d (entry (d x + z, d y + w) is
 * v[x][y] when z = w) and updated to polar((1 - beta) G1 + beta v) of its d x d
 * environment G1[x][y] = sum_z Gamma[d x + z][d y + z]; a QFS_GATE_FIXED gate takes
 * tmpl->fixed_gates (device [L][D][D], read for those entries; they replace the same slots
 * of gates_in) and is never updated. Drawn one-qudit gates are Haar on U(d) from the d x d
 * Ginibre block at indices 256 gate + d col + row of the start's stream.
 *
 * Instantiation on a fixed sample set with the paper's control loop (Sec. 3, App. A), the
 * SAMPLES semantics of qfs_instantiate: psi, phi device [n_samples][N] (phi = U psi);
 * rows 0 .. n_samples - n_val - 1 train (M from params->m_init, doubling takes more rows,
 * capped by m_max), the last n_val rows validate (n_val = 0: no generalisation test).
 * gates_in: device [multistarts][L][D][D] or NULL for Haar-random D x D initial gates
 * drawn from params->seed (role 3, stream = start, index 256 gate + D col + row of a
 * column-major Ginibre block). gates_out: device [L][D][D]. Precision FP64 or MIXED
 * (complex64 states, complex128 sweeps once the best running c_train < refine_below).
 * params->timing and full_unitary are not supported here (full_unitary: QFS_EINVAL). When
 * the starts' sets and B lists do not fit (device out of memory, or more than
 * params->device_mem_budget bytes when that is set) the starts run as two halves,
 * recursively, each with its own control loop (App. A), and the better result is returned
 * (success first, then lower c_train; res->start_groups counts the groups).
 * Errors: QFS_EINVAL, QFS_EUNSUPPORTED, QFS_ENOMEM (one start does not fit), QFS_EDEVICE. */
int qfs_qudit_instantiate(int32_t d, const qfs_template *tmpl, const qfs_c128 *psi,
                          const qfs_c128 *phi, int32_t n_samples, int32_t n_val,
                          const qfs_params *params, const qfs_c128 *gates_in,
                          qfs_c128 *gates_out, qfs_result *res);

/* The same with a target as for qfs_instantiate: DENSE (U device [N][N] row-major,
 * N = d^n <= 2^16) or CIRCUIT (target->circuit a host template on the same n qudits, its
 * kinds ignored; target->circuit_gates device [Lt][D][D]), with the training and
 * validation states drawn on the device as qfs_instantiate draws them for qubits (Sec. 3,
 * App. A: columns of a Haar unitary; Philox role 1 stream 0 for training, role 2 stream =
 * generation for validation, index j N + i; M_val = params->m_val or M, capped at N), the
 * targets formed on the device (U psi by the dense product, or the target circuit's
 * gates applied in order); a doubling extends the training set by the next columns of
 * its stream, orthonormal to the earlier ones, keeps every gate, and draws the next
 * validation generation. SAMPLES forwards to qfs_qudit_instantiate. Errors as there, plus
 * QFS_ENUMERIC when a drawn set fails to orthonormalise. */
int qfs_qudit_instantiate_target(int32_t d, const qfs_template *tmpl, const qfs_target *target,
                                 const qfs_params *params, const qfs_c128 *gates_in,
                                 qfs_c128 *gates_out, qfs_result *res);

/* P qudit problems (templates tmpls[i], targets targets[i] in any form) with the same
 * params, each as qfs_qudit_instantiate_target, run side by side on up to eight streams of
 * their own (the qudit path is bound by the latency of its small kernels, so problems on
 * separate streams fill the device together); each problem's sweeps keep to its stream.
 * gates_out: host array of P device pointers ([L_i][D][D] each); res: host [P]. The
 * caller's stream (params->hip_stream) is synchronised first. On an error no further
 * problem starts and the first error is returned (its detail names the problem). */
int qfs_qudit_instantiate_batch(int32_t d, int32_t P, const qfs_template *tmpls,
                                const qfs_target *targets, const qfs_params *params,
                                qfs_c128 *const *gates_out, qfs_result *res);

/* One qudit sweep for `starts` starts sharing a training set, as qfs_sweep: psi, phi
 * device [M][N]; kinds host [L] or NULL (constant gates are the gates' own slots, applied
 * and kept); gates device [starts][L][D][D] updated in place; c_train host [starts] (Eq. 9
 * cost of the updated gates). */
int qfs_qudit_sweep(int32_t d, int32_t n, int32_t L, const int32_t *pairs, const int32_t *kinds,
                    int32_t M, const qfs_c128 *psi, const qfs_c128 *phi, int32_t starts,
                    qfs_c128 *gates, int32_t precision, double beta, double *c_train,
                    void *hip_stream);

/* ------------------------------------------------- steps of the method (device) */
/* M orthonormal Haar states (Sec. 3; App. A: columns of a Haar unitary): the Q of the
 * QR factorisation, with real positive diag(R), of the N x M complex Ginibre matrix
 * drawn with (seed, role, stream). out: device [M][N]. M <= 2^n. */
int qfs_draw_states(int32_t n, int32_t M, uint64_t seed, uint32_t role, uint32_t stream,
                    qfs_c128 *out, void *hip_stream);

/* Haar-random 4x4 initial gates for `starts` starts of L gates each (App. A,
 * multistarts and seed). out: device [starts][L][4][4]. */
int qfs_haar_gates(uint64_t seed, int32_t starts, int32_t L, qfs_c128 *out,
                   void *hip_stream);

/* Apply a gate list in order to M states in place (Fig. pre-comp, the B list; the
 * circuit form of the target). states: device [M][N]; pairs: host [L][2];
 * gates: device [L][4][4]. dagger = 1 applies u^dagger of each gate instead. */
int qfs_apply_gates(int32_t n, int32_t M, qfs_c128 *states, int32_t L,
                    const int32_t *pairs, const qfs_c128 *gates, int32_t dagger,
                    void *hip_stream);

/* out = U psi for a dense target (Sec. 2.3). U: device [N][N] row-major; psi, out:
 * device [M][N]. */
int qfs_dense_apply(int32_t n, int32_t M, const qfs_c128 *U, const qfs_c128 *psi,
                    qfs_c128 *out, void *hip_stream);

/* Environment of the gate on qubits (qa, qb) (Sec. 3, Eq. 10; Fig. env_calc_tensor):
 * Gamma[q][p] = sum_j sum_r a_j(q, r) conj(b_j(p, r)) over the M samples and the
 * other n-2 qubits r. The paper's E is Gamma^dagger. a, b: device [M][N];
 * gamma: device [4][4]. */
int qfs_environment(int32_t n, int32_t M, const qfs_c128 *a, const qfs_c128 *b,
                    int32_t qa, int32_t qb, qfs_c128 *gamma, void *hip_stream);

/* qfs_environment for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same Gamma, computed
 * from the row-major states directly, with its work-group partial sums in a fixed array of
 * this library (256 KiB per GPU, held until the process ends); no allocation, no
 * memset, no synchronisation (gamma is ready in stream order). Limit: M 2^(n-2) <= 2^28,
 * else QFS_EINVAL. Every call on a GPU shares that array: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller. a, b: device
 * [M][N]; gamma: device [4][4]. */
int qfs_environment_noalloc(int32_t n, int32_t M, const qfs_c128 *a, const qfs_c128 *b,
                            int32_t qa, int32_t qb, qfs_c128 *gamma, void *hip_stream);

/* Gate update (Sec. 2.1, Eq. 2; App. A Beta): u <- W V^dagger where
 * (1 - beta) Gamma + beta u = W S V^dagger (FP64 one-sided Jacobi SVD). count
 * independent 4x4 problems; gamma: device [count][4][4]; u: device [count][4][4]
 * (read when beta != 0, always written). */
int qfs_polar_update(int32_t count, const qfs_c128 *gamma, double beta, qfs_c128 *u,
                     void *hip_stream);

/* One sweep for `starts` starts sharing a training set (Sec. 3; Fig. pre-comp;
 * Fig. env_calc_tensor): forward B list from the current gates, then right to left
 * environment, polar update, and backward propagation through the updated gate;
 * returns the Eq. 9 cost of the updated gates per start.
 *   kinds:     host [L] gate kinds, or NULL (every gate QFS_GATE_2Q); constant gates
 *              are the gates' own entries and are left unchanged; a one-qubit
 *              gate's entry must have the form v (x) I_2 exactly (the forward pass
 *              skips the products with its zero entries).
 *   psi, phi:  device [M][N] (training states and U psi).
 *   gates:     device [starts][L][4][4], updated in place (complex128 master).
 *   precision: QFS_PREC_FP64 or QFS_PREC_MIXED (complex64 states).
 *   backward_mode: QFS_BWD_GROUPED or QFS_BWD_PER_GATE (as qfs_params.backward_mode).
 *   c_train:   host [starts]. */
int qfs_sweep(int32_t n, int32_t L, const int32_t *pairs, const int32_t *kinds, int32_t M,
              const qfs_c128 *psi, const qfs_c128 *phi, int32_t starts, qfs_c128 *gates,
              int32_t precision, double beta, int32_t backward_mode, double *c_train,
              void *hip_stream);

/* (1/M) sum_j ||x_j - y_j||^2 accumulated in FP64 (Sec. 3, Eq. 9). x, y: device
 * [M][N]; result: host. */
int qfs_state_distance(int32_t n, int32_t M, const qfs_c128 *x, const qfs_c128 *y,
                       double *result, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QFS_H */
