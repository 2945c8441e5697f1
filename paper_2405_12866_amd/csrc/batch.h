// Device-side structures of the batched engine (batch.hip, batch_engine.hip).
#pragma once

#include "qfs_internal.h"

namespace qfs {

// Job status (per problem x start).
enum {
  BJ_RUN = 0,
  BJ_SUCCESS = 1,
  BJ_PLATEAU = 2,
  BJ_MAX_ITER = 3,
  BJ_NOT_GEN = 4,
  BJ_OVER = 5,     // overtrained: waits for the problem's doubling
  BJ_PAUSED = 6,   // reached a sweep the problem already decided on
  BJ_REFINE = 7,   // complex64 job below refine_below: continue in complex128
  BJ_TIMEOUT = 8,
  BJ_SKIP = 9,      // start not run (pruned by the caller)
  BJ_PARKED = 10    // pruned start that runs only if every other start stops unsuccessfully
};

constexpr int kNoSweep = 0x3fffffff;

struct BProb {
  int32_t n, L, M, Mv, mcap, full;
  int32_t kind;         // QFS_TARGET_*
  int32_t Lt;           // target circuit length
  int32_t generation;   // validation stream
  int32_t n_train;      // SAMPLES: training rows available
  uint64_t seed;
  const int32_t *pairs;   // device [L][2]
  const int32_t *kinds;   // device [L] gate kinds (nullptr: all two-qubit)
  const c128 *fixed;      // device [L][16] constant gates (read at QFS_GATE_FIXED)
  const int32_t *tpairs;  // device [Lt][2]
  const c128 *tgates;     // device [Lt][16]
  const c128 *U;          // DENSE target
  const c128 *s_psi, *s_phi;  // SAMPLES target rows
  c128 *psi, *phi, *psiv, *phiv;  // FP64 masters, sample-major [M][N]
  c128 *coef;             // Gram-Schmidt scratch [mcap]
  c128 *g64;              // [S][L][16]
  c128 *vst;              // [S][L][16] Jacobi warm start
  int32_t done_sweep;     // smallest sweep count at which a start succeeded
  int32_t over_sweep;     // smallest sweep count at which a start was overtrained
};

struct BJob {
  int32_t prob, start;
  int32_t status;
  int32_t iter, z, total;
  int32_t need_c0;
  int32_t fp64;
  double c_prev, c_train, c_val;
  double work;  // sum over this job's sweeps of (M + Mv) 2^n L
};

struct BParams {
  double dist_tol, diff_tol_r, overtrain_ratio, beta, refine_below;
  int32_t plateau_window, min_iter;
  int64_t max_iter;
  int32_t mixed;
  int32_t independent;  // every start runs to its own stop (no problem-level pause)
  int32_t beta_normalized;  // mix Gamma / M (effective_beta of the problem's M)
};

struct BatchArgs {
  BJob *jobs;
  BProb *probs;
  const int32_t *queue;   // job ids, longest first
  int32_t njobs;
  int32_t *queue_head;    // zeroed before each launch
  int32_t sweeps_per_launch;
  BParams hp;
  char *scratch;          // per-work-group state slots (nullptr: states in LDS)
  size_t scratch_slot_bytes;
};

// Per-problem options of the batched engine (all nullable / zero = the plain method).
struct BatchOpts {
  const int32_t *m_init = nullptr;  // [P] initial sample count per problem
  const int32_t *starts = nullptr;  // [P] problem p runs starts [start_lo[p], starts[p])
  const int32_t *start_lo = nullptr;  // [P] first start to run (default 0)
  const uint64_t *seeds = nullptr;  // [P] per-problem seeds (default params->seed + p)
  int independent = 0;              // starts do not stop at another start's success
  int park_rest = 0;                // starts beyond starts[p] are parked, not skipped
  int32_t *fallback_used = nullptr; // [P] out: 1 when parked starts were run
  int32_t *successes = nullptr;     // [P] out: number of starts that succeeded
};

int batch_instantiate(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                      const qfs_params *params, qfs_c128 *const *gates_out, qfs_result *res,
                      const BatchOpts &opts);

int launch_batch_setup(BProb *probs_dev, const int32_t *todo, int ntodo, const int32_t *m0s,
                       hipStream_t s);
int launch_batch_gates(BProb *probs_dev, const int32_t *prob_of, const int32_t *first_gate,
                       int total, hipStream_t s);
int launch_batch_sweep(const BatchArgs &a, bool fp64, int threads, int grid, size_t lds,
                       hipStream_t s);

}  // namespace qfs
