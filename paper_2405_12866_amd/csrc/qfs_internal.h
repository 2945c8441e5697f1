// Internal declarations of the HIP implementation (not part of the C ABI).
//
// Device state layout ("amplitude-major"): a set of M states of N = 2^n amplitudes is
// an N x ld row-major matrix, element (i, j) = amplitude i of sample j, ld >= M even,
// columns M..ld-1 zero. Columns are states, so the linear algebra of the sample
// draw works on it directly, and every two-qubit gate touches four rows whose
// sample runs are contiguous: loads are 16-byte vectors over consecutive samples
// whatever qubits the gate acts on.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qfs.h"

namespace qfs {

// ------------------------------------------------------------------ complex helpers
template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__host__ __device__ inline cx<R> cmake(R re, R im) {
  cx<R> z;
  z.re = re;
  z.im = im;
  return z;
}
template <typename R>
__host__ __device__ inline cx<R> operator+(cx<R> a, cx<R> b) {
  return cmake<R>(a.re + b.re, a.im + b.im);
}
template <typename R>
__host__ __device__ inline cx<R> operator-(cx<R> a, cx<R> b) {
  return cmake<R>(a.re - b.re, a.im - b.im);
}
template <typename R>
__host__ __device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
  return cmake<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ inline cx<R> cscale(cx<R> a, R s) {
  return cmake<R>(a.re * s, a.im * s);
}
template <typename R>
__host__ __device__ inline cx<R> cconj(cx<R> a) {
  return cmake<R>(a.re, -a.im);
}
template <typename R>
__host__ __device__ inline R cabs2(cx<R> a) {
  return a.re * a.re + a.im * a.im;
}
// acc += a * b
template <typename R>
__host__ __device__ inline void cfma(cx<R> &acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += a * conj(b)
template <typename R>
__host__ __device__ inline void cfma_conj(cx<R> &acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.im, b.re, acc.im);
  acc.im = fma(-a.re, b.im, acc.im);
}

using c64 = cx<float>;
using c128 = cx<double>;

// ------------------------------------------------------------------ errors
struct Status {
  int code = QFS_OK;
};

void set_error_detail(const std::string &s);

// Process-wide pool of non-blocking streams (default priority) on the current device,
// created on first use and kept until the process ends: creating streams per call costs
// far more than a small instantiation. Index 0..15.
int pool_stream(int index, hipStream_t *out);

#define QFS_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e__ = (call);                                                           \
    if (e__ != hipSuccess) {                                                           \
      ::qfs::set_error_detail(std::string(#call) + ": " + hipGetErrorString(e__) +     \
                              " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
      return QFS_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)

#define QFS_TRY(expr)         \
  do {                        \
    int rc__ = (expr);        \
    if (rc__ != QFS_OK) return rc__; \
  } while (0)

// ------------------------------------------------------------------ device buffers
// Blocks that calls of the single-problem engine give back when they end, kept for the
// next call of the same size instead of hipFree (engine.hip). Every block in the cache is
// idle: a call gives its blocks back only after the device has drained.
void *device_cache_take(int dev, size_t bytes);
size_t device_cache_held(int dev);
size_t device_cache_trim(int dev);  // frees the device's cached blocks; returns the bytes freed

// A simple owning device allocation; the engine keeps a few of these per call. An
// allocator that takes blocks back (the engine's per-call Arena) sets give_back, and
// release() then hands the block to it instead of freeing it.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  void (*give_back)(void *owner, void *ptr, size_t bytes) = nullptr;
  void *owner = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  int alloc(size_t b) {
    release();
    if (b == 0) return QFS_OK;
    hipError_t e = hipMalloc(&ptr, b);
    if (e == hipErrorOutOfMemory) {
      // blocks held for later calls go first
      (void)hipGetLastError();
      int dev = 0;
      if (hipGetDevice(&dev) == hipSuccess && device_cache_trim(dev) > 0) e = hipMalloc(&ptr, b);
    }
    if (e != hipSuccess) {
      ptr = nullptr;
      (void)hipGetLastError();
      set_error_detail(std::string("hipMalloc(") + std::to_string(b) + "): " + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? QFS_ENOMEM : QFS_EDEVICE;
    }
    bytes = b;
    return QFS_OK;
  }
  void release() {
    if (ptr) {
      if (give_back)
        give_back(owner, ptr, bytes);
      else
        (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
    give_back = nullptr;
    owner = nullptr;
  }
  void swap(DevBuf &o) {
    std::swap(ptr, o.ptr);
    std::swap(bytes, o.bytes);
    std::swap(give_back, o.give_back);
    std::swap(owner, o.owner);
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(ptr);
  }
};

// ------------------------------------------------------------------ kernels (host API)
// Random numbers (rng.hip). Philox roles of the drawn sets: training states, validation
// states (stream = the validation set's generation), initial gates (stream = start).
enum { kRoleTrain = 1, kRoleVal = 2, kRoleInit = 3 };
// Raise kernel fn's dynamic-LDS limit to at least `bytes` (above 64 KB it must be asked
// for per kernel); *have caches what was set. Serialised across threads: problems may be
// run from several host threads at once.
int ensure_dynamic_lds(const void *fn, size_t bytes, size_t *have);
int launch_ginibre(int64_t rows, int64_t col0, int64_t col1, int64_t ld, uint64_t seed,
                   uint32_t role, uint32_t stream, c128 *A, hipStream_t s);
int launch_haar_gates(uint64_t seed, int32_t start0, int32_t starts, int32_t L, c128 *out,
                      hipStream_t s);
// Gate kinds applied to [starts][L] slots: constant gates copied from fixed, and, when the
// slots were drawn, one-qubit gates redrawn as v (x) I_2. kinds: device [L] (NULL: no-op).
int launch_kind_gates(uint64_t seed, int32_t start0, int32_t starts, int32_t L,
                      const int32_t *kinds, const c128 *fixed, bool drawn, c128 *out,
                      hipStream_t s);

// Linear algebra (linalg.hip), all complex FP64, row-major with leading dimensions.
// C[m x n] = alpha * op(A) * B + beta * C, op(A) = A (m x k) or A^H (A is k x m).
int launch_zgemm(bool conjtrans_a, int m, int n, int k, c128 alpha, const c128 *A, int lda,
                 const c128 *B, int ldb, c128 beta, c128 *C, int ldc, hipStream_t s);
// Orthonormalise columns [c0, c1) of the rows x ld matrix A against columns [0, c0)
// and among themselves: QR with real positive diag(R) (CholeskyQR2 after two block
// Gram-Schmidt projections). Uses `work` (device, >= work_bytes_orth(rows, c1)). With
// flag_dev null it waits for the stream and returns QFS_ENUMERIC on a non-positive
// Cholesky pivot; else it returns at once and sets *flag_dev (device, zeroed by the caller)
// to 1 on such a pivot.
size_t work_bytes_orth(int64_t rows, int64_t cols);
int orthonormalize_columns(int64_t rows, int64_t ld, int64_t c0, int64_t c1, c128 *A,
                           void *work, hipStream_t s, int *flag_dev = nullptr);

// Layout conversions (linalg.hip)
// sample-major [M][N] c128  <->  chunked amplitude-major layout in R (zero padding).
template <typename R>
int launch_to_internal(int n, int64_t M, int logC, int64_t nch, const c128 *src, cx<R> *dst,
                       hipStream_t s);
template <typename R>
int launch_from_internal(int n, int64_t M, int logC, const cx<R> *src, c128 *dst, hipStream_t s);
int launch_narrow(int64_t count, const c128 *src, c64 *dst, hipStream_t s);
// Per-start copies between buffers of layout [S][units] (16-byte units; src and dst 16-byte
// aligned), for the starts slots[0 .. nslots) (device list): up to kBufs buffers per launch,
// units 0 for an unused one.
struct SlotCopy {
  static constexpr int kBufs = 3;
  const uint4 *src[kBufs] = {};
  uint4 *dst[kBufs] = {};
  int64_t units[kBufs] = {};
};
int launch_copy_slots(const int32_t *slots, int nslots, const SlotCopy &c, hipStream_t s);
int launch_zero(void *p, size_t bytes, hipStream_t s);
// A[i][i] = 1 for i < N in an N x ld complex128 matrix (the computational basis as columns).
int launch_unit_columns(int64_t N, int64_t ld, c128 *A, hipStream_t s);

// Host check of gate slots [count][4][4] (gate gi % L of a template with the given kinds):
// unitary to 1e-10 and, for one-qubit gates, of the form v (x) I_2. fixed_only: only the
// constant gates; else every gate but those. QFS_EINVAL with a detail naming `what`.
int check_gates_unitary(const qfs_c128 *gates_dev, size_t count, int L, const int32_t *kinds,
                        bool fixed_only, const char *what, hipStream_t s);

// Control of one running start after a sweep (Sec. 3 success relations, Eq. 12; App. A:
// plateau test Eq. 13 over plateau_window sweeps after min_iter, max_iter, time budget).
// ct, cv: training and validation cost after the sweep; no_gen_test: the training set is
// the full basis or there is no validation set; can_double: M may still grow. Updates the
// counters and returns ST_STOP (reason set), ST_OVER (overtrained, M may double) or ST_RUN.
enum { ST_RUN = 0, ST_STOP = 1, ST_OVER = 2 };
inline int control_step(const qfs_params &p, double ct, double cv, bool no_gen_test, bool can_double,
                        bool timed_out, int &iter, int &z, int64_t &total, double &c_prev, int &reason) {
  iter += 1;
  total += 1;
  const bool improved = std::fabs(c_prev) - std::fabs(ct) > p.diff_tol_r * std::fabs(ct);
  z = improved ? 0 : z + 1;
  c_prev = ct;
  const bool gen_ok = no_gen_test || cv <= (1.0 + p.overtrain_ratio) * ct;
  if (ct < p.dist_tol && gen_ok) return reason = QFS_SUCCESS, ST_STOP;
  if (iter >= p.min_iter && !gen_ok) {
    if (can_double) return ST_OVER;
    if (ct < p.dist_tol) return reason = QFS_NOT_GENERALIZED, ST_STOP;
  }
  if (iter >= p.min_iter && z >= p.plateau_window) return reason = QFS_PLATEAU, ST_STOP;
  if (total >= p.max_iter) return reason = QFS_MAX_ITER, ST_STOP;
  if (timed_out) return reason = QFS_TIMEOUT, ST_STOP;
  return ST_RUN;
}

// The regularised update with the environment normalised by M, polar((1 - beta) G / M +
// beta u), is the paper's unnormalised form polar((1 - b) G + b u) at
// b = beta M / ((1 - beta) + beta M): the two mixes differ by the positive factor
// (1 - beta) + beta M, and the polar factor ignores a positive scale.
__host__ __device__ inline double effective_beta(double beta, bool normalized, int M) {
  if (!normalized || beta <= 0.0 || beta >= 1.0) return beta;
  const double bm = beta * (double)M;
  return bm / ((1.0 - beta) + bm);
}

// Capacity, in blocks, of the per-start environment partials of a backward step: start s
// owns blocks [s kPcap, s kPcap + P) whatever the block count P of a launch, so launches on
// different streams over different start sets (with different P) never share partials.
constexpr int kPcap = 4096;

// ------------------------------------------------------------------ sweep kernels
// Per-start addressing for the sweep kernels: a buffer of starts is at
// base + stride * start (elements); stride 0 means shared by all starts.
template <typename R>
struct SBuf {
  cx<R> *base;
  int64_t stride;
};

struct GateRef {
  const c128 *g64;   // [S][L][16]
  const void *gR;    // [S][L][16] in state precision (c64 copy or the c128 master)
  int32_t gstride;   // L * 16
};

// A chunked state set: nch chunks of C = 2^logC samples, each chunk N x C row-major;
// element (i, j) at (j >> logC) * N * C + i * C + (j & (C - 1)). M live samples, the
// padding samples are zero.
struct Geometry {
  int32_t n;       // qubits
  int32_t N;       // 2^n
  int32_t logC;    // log2 chunk width (>= 1)
  int32_t nch;     // chunks
  int32_t M;       // live samples
  int64_t elems() const { return (int64_t)nch << (n + logC); }
};

// Chunk width: the fused forward pass needs a whole chunk in LDS (N * C complex);
// otherwise chunks of up to 32 samples keep rows coalesced.
int choose_log_chunk(int n, int M, size_t rbytes, bool fused, int starts, size_t lds_max);
bool forward_fusable(int n, size_t rbytes, size_t lds_max);
size_t forward_lds_bytes(int n, int logC, size_t rbytes);

// Per-gate apply: dst_s = op(u_s[k]) src_s on qubits (qa, qb), for the slots
// [0, nslots) mapped to starts by slot_to_start (device).
template <typename R>
int launch_apply(const Geometry &g, int qa, int qb, int k, bool dagger, GateRef gates,
                 SBuf<R> src, SBuf<R> dst, const int32_t *slot_to_start, int nslots,
                 hipStream_t s);

// Fused forward pass for every slot: B list (B_{k+1} at list index k, k < L-1) from
// psi; optionally the Eq. 9 distance of the full circuit against phi_ref (block
// partials [S][g.nch]); optionally the validation set through all L gates with its
// distance partials [S][gv->nch]. pairs_dev: device [L][2]. kinds_dev: device [L] gate
// kinds or nullptr; the B list entry before a constant gate is not stored (no environment
// reads it). bneed_dev: device [L], when given B_j is stored iff bneed_dev[j] != 0 (the
// grouped backward pass reads one entry per group).
template <typename R>
int launch_forward_fused(const Geometry &g, const Geometry *gv, const int32_t *pairs_dev, int L,
                         GateRef gates, const cx<R> *psi, cx<R> *blist, int64_t bstride,
                         const cx<R> *phi_ref, double *c0_partials, const cx<R> *psiv,
                         const cx<R> *phiv, double *val_partials, const int32_t *slot_to_start,
                         int nslots, const int32_t *kinds_dev, hipStream_t s,
                         const int32_t *bneed_dev = nullptr);

template <typename R>
int launch_pack(const Geometry &g, int64_t ld, const c128 *master, cx<R> *dst, hipStream_t s);

// Backward step: optionally a_s <- u_s[k_apply]^dagger a_s (qubits of k_apply; with
// k_apply2 >= 0, a gate on the same two qubits, a_s <- u_s[k_apply]^dagger
// u_s[k_apply2]^dagger a_s), then the environment of gate k_env from a_s and b_s as
// per-block FP64 partial sums
// [S][kPcap][16] (blocks 0 .. P-1 of each start; P returned). launch_env_finalize (one
// wave per start) reduces them in a fixed order and writes u_s[k_env] <- polar((1-beta) Gamma + beta u) to both gate
// copies (kind QFS_GATE_1Q: the one-qubit update of a v (x) I_2 slot); optionally stores
// Gamma (FP64) to gamma_out[s].
template <typename R>
int launch_bwd_step(const Geometry &g, const int32_t *pairs_host, int k_apply, int k_env,
                    GateRef gates, SBuf<R> a_in, SBuf<R> a_out, SBuf<R> b,
                    const int32_t *slot_to_start, int nslots, c128 *partials, int *P_out,
                    hipStream_t s, int k_apply2 = -1);
// vstore (nullable, [S][L][16]): right singular vectors of each gate's last update,
// used to warm-start the Jacobi iteration and updated in place.
int launch_env_finalize(int P, const c128 *partials, const int32_t *slot_to_start, int nslots,
                        c128 *gamma_out, bool do_update, double beta, c128 *g64, c64 *g32,
                        int32_t gstride, int32_t k_env, c128 *vstore, int kind, hipStream_t s);
// count 4x4 identity matrices.
int launch_identity4(int64_t count, c128 *v, hipStream_t s);

// Block partials of sum ||op(u_s[k]) x_s - ref_s||^2 (k < 0: no gate), P returned;
// launch_dist_finalize writes out[s] = (1/M) * (fixed-order sum of partials[s stride + b],
// b < P; stride 0 means P).
template <typename R>
int launch_apply_dist(const Geometry &g, int qa, int qb, int k, bool dagger, GateRef gates,
                      SBuf<R> x, SBuf<R> ref, const int32_t *slot_to_start, int nslots,
                      double *partials, int *P_out, hipStream_t s);
int launch_dist_finalize(int P, const double *partials, const int32_t *slot_to_start, int nslots,
                         int M, double *out, hipStream_t s, int stride = 0);

// Batched polar update on device (count problems).
int launch_polar_batch(int count, const c128 *gamma, double beta, c128 *u, hipStream_t s);

// ------------------------------------------------------------------ grouped backward pass
// Consecutive gates whose qubits fit in four slots share one pass over the backward state
// (group.hip): the pass reduces a 16 x 16 second-moment matrix of the state entering the
// group and the forward state before it, and a finalize kernel derives every environment
// of the group from it and updates the gates in order.
constexpr int kGroupMaxGates = 16;
// Most blocks per start of a grouped pass (second-moment partials [S][stride][256] c128,
// stride = group_partials_stride(g) <= kGPcap).
constexpr int kGPcap = 512;
struct GateGroup {
  int32_t k_hi, k_lo;  // gates k_lo .. k_hi
  int32_t nq;          // distinct qubits of the group (<= 4)
  int32_t q[4];        // those qubits: slots 0 .. nq-1 of the second-moment index
  int32_t nvar;        // variable (updated) gates in the group
};
// Groups from the last gate down, each as long as its qubits fit in four (fewest groups).
// Start/stop events recorded by a launch itself (see launch_group_pass).
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
std::vector<GateGroup> plan_gate_groups(int L, const int32_t *pairs, const int32_t *kinds);
bool group_path_supported(const Geometry &g, size_t rbytes);
// Blocks per start any grouped pass over geometry g uses at most (the partials' stride).
int group_partials_stride(const Geometry &g, size_t rbytes);
// One pass: a_in <- Vop a_in with prev's operator (vop [S][256], from prev's finalize; when
// prev), stored to a_out (when given), then either the second-moment block partials of cur
// against b (gpartials) or, with dist, the block partials of sum |a - b|^2 ([S][P] in
// dpartials). P returned.
// (ev: start/stop events the launch records itself, hipExtLaunchKernelGGL, so that they
// bracket the kernel's own execution; both null: a plain launch.)
template <typename R>
int launch_group_pass(const Geometry &g, const int32_t *pairs, const GateGroup *prev,
                      const GateGroup *cur, bool dist, const c128 *vop, SBuf<R> a_in, SBuf<R> a_out,
                      SBuf<R> b, const int32_t *slot_to_start, int nslots, int blocks_per_start,
                      c128 *gpartials, int pstride, double *dpartials, int *P_out, hipStream_t s,
                      LaunchEvents ev = {});
// Forward pass by gate groups (the groups in forward order, one LDS round trip per group;
// complex64 states, the products on the matrix cores):
// plan [ngroups][8] and per-gate entries [L][kFwdGS] (the slots of the gate's two qubits and
// how it is applied) from build_forward_plan (host; bneed_host [L] marks the B entries the
// backward pass reads; mode_host [L] from forward_gate_modes, or null: every gate dense),
// copied to the device by the caller.
enum { kFwdGS = 4 };
enum { kFwdDense = 0, kFwd1Q = 1, kFwdCnotA = 2, kFwdCnotB = 3 };
// How each gate is applied in the grouped forward pass: one-qubit gates (v (x) I_2) as 2x2
// products, constant gates that are exactly a CNOT (in every one of `copies` host copies of
// the gates, [copies][L][16]) as an exchange of amplitudes, the rest as dense 4x4 products.
// launch_forward_groups takes forms = any gate not dense (a kernel built for the forms).
std::vector<int32_t> forward_gate_modes(int L, const int32_t *kinds, const c128 *gates_host, int copies);
int build_forward_plan(const Geometry &g, int L, const int32_t *pairs, const std::vector<GateGroup> &groups,
                       const int32_t *bneed_host, const int32_t *mode_host, std::vector<int32_t> &plan,
                       std::vector<int32_t> &gslot);
template <typename R>
int launch_forward_groups(const Geometry &g, const Geometry *gv, int L, GateRef gates, const cx<R> *psi,
                          cx<R> *blist, int64_t bstride, const cx<R> *phi_ref, double *c0_partials,
                          const cx<R> *psiv, const cx<R> *phiv, double *val_partials,
                          const int32_t *slot_to_start, int nslots, const int32_t *plan_dev, int ngroups,
                          const int32_t *gslot_dev, bool forms, hipStream_t s);
// Work-groups per start of a grouped pass when `running_starts` starts sweep together
// (whatever streams they are split over).
int group_blocks_per_start(int running_starts);
// Per start: sum the P partials in a fixed order and update cur's variable gates from the top
// down (both gate copies, warm-start vectors as launch_env_finalize); then write cur's
// operator Vop = u_{k_lo}^dag ... u_{k_hi}^dag over its four slots to vop [S][256].
int launch_group_finalize(int P, const c128 *gpartials, int pstride, const int32_t *slot_to_start,
                          int nslots,
                          const GateGroup &cur, const int32_t *pairs, const int32_t *kinds,
                          double beta, c128 *g64, c64 *g32, int32_t gstride, c128 *vstore,
                          c128 *vop, hipStream_t s, LaunchEvents ev = {});

}  // namespace qfs
