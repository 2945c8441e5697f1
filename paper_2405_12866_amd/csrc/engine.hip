// Host runtime and C ABI of the HIP implementation: the instantiation control loop
// (Sec. 3 on-the-fly generalisation check and double-and-restart, Eq. 12 success
// relations; App. A plateau test, min_iter/max_iter, multistarts and the recursive
// half-multistart retry on device out-of-memory), device memory management and the
// per-step entry points declared in include/qfs.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <vector>

#include "qfs_internal.h"

namespace qfs {

static thread_local std::string g_detail;
void set_error_detail(const std::string &s) { g_detail = s; }

namespace {

enum { kRoleTrain = 1, kRoleVal = 2 };

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

hipStream_t as_stream(void *p) { return static_cast<hipStream_t>(p); }

int64_t even_up(int64_t m) { return (m + 1) & ~int64_t(1); }

int validate_template(const qfs_template *t) {
  if (!t || t->n_qubits < 2 || t->n_qubits > 24 || t->n_gates < 1 || !t->pairs) {
    set_error_detail("template: need 2 <= n_qubits <= 24, n_gates >= 1, pairs != NULL");
    return QFS_EINVAL;
  }
  for (int k = 0; k < t->n_gates; ++k) {
    const int a = t->pairs[2 * k], b = t->pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= t->n_qubits || b >= t->n_qubits || a == b) {
      set_error_detail("template: gate " + std::to_string(k) + " has an invalid qubit pair");
      return QFS_EINVAL;
    }
  }
  return QFS_OK;
}

// Memory accounting for one call: every allocation goes through here so that the
// budget (device_mem_budget or the free memory) is enforced before hipMalloc.
struct Arena {
  size_t budget = 0, used = 0;
  int alloc(DevBuf &b, size_t bytes) {
    const size_t old = b.bytes;
    if (used - old + bytes > budget) {
      set_error_detail("device memory budget exceeded: need " + std::to_string(used - old + bytes) +
                       " of " + std::to_string(budget) + " bytes");
      return QFS_ENOMEM;
    }
    used -= old;
    b.release();
    QFS_TRY(b.alloc(bytes));
    used += bytes;
    return QFS_OK;
  }
  void free(DevBuf &b) {
    used -= b.bytes;
    b.release();
  }
};

struct GroupResult {
  int rc = QFS_OK;
  int reason = QFS_MAX_ITER;
  int best = -1;  // absolute start index
  double c_train = INFINITY, c_val = INFINITY;
  int m_final = 0, sweeps = 0, restarts = 0, m_total = 0;
  int64_t success_round = -1;  // sweep round at which the success was found
  int refined = 0;
  int64_t start_sweeps = 0;
  double sweep_seconds = 0.0;
  int64_t kl[3] = {0, 0, 0};
  double ks[3] = {0, 0, 0}, kb[3] = {0, 0, 0};
  std::vector<qfs_c128> gates;  // [L][16] of the chosen start (host copy)
};

// Optional per-kernel timing: a start/stop hipEvent pair around every timed launch on
// the call's stream, read back after the next stream synchronisation.
class KernelTimer {
 public:
  ~KernelTimer() {
    for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
  }
  bool on = false;
  int begin(hipStream_t s) {
    if (!on) return QFS_OK;
    if (ev_.size() < 2 * (used_ + 1)) {
      hipEvent_t a, b;
      QFS_HIP(hipEventCreate(&a));
      QFS_HIP(hipEventCreate(&b));
      ev_.push_back(a);
      ev_.push_back(b);
    }
    QFS_HIP(hipEventRecord(ev_[2 * used_], s));
    return QFS_OK;
  }
  int end(hipStream_t s, int cls, double bytes) {
    if (!on) return QFS_OK;
    QFS_HIP(hipEventRecord(ev_[2 * used_ + 1], s));
    if (cls_.size() <= used_) {
      cls_.resize(used_ + 1);
      bytes_.resize(used_ + 1);
    }
    cls_[used_] = cls;
    bytes_[used_] = bytes;
    ++used_;
    return QFS_OK;
  }
  // Call only after the stream has been synchronised.
  int flush(GroupResult &r) {
    for (size_t i = 0; i < used_; ++i) {
      float ms = 0.f;
      QFS_HIP(hipEventElapsedTime(&ms, ev_[2 * i], ev_[2 * i + 1]));
      r.kl[cls_[i]] += 1;
      r.ks[cls_[i]] += 1e-3 * ms;
      r.kb[cls_[i]] += bytes_[i];
    }
    used_ = 0;
    return QFS_OK;
  }

 private:
  std::vector<hipEvent_t> ev_;
  std::vector<int> cls_;
  std::vector<double> bytes_;
  size_t used_ = 0;
};

enum { ST_RUN = 0, ST_STOP = 1, ST_OVER = 2 };

// One independent QFactor-Sample run over starts [start0, start0 + S).
class Group {
 public:
  Group(const qfs_template *t, const qfs_target *tg, const qfs_params &p, const qfs_c128 *gates_in,
        int start0, int S, Arena &arena)
      : tgt_(tg), p_(p), gates_in_(gates_in), start0_(start0), S_(S), arena_(arena) {
    n_ = t->n_qubits;
    L_ = t->n_gates;
    N_ = int64_t(1) << n_;
    pairs_.assign(t->pairs, t->pairs + 2 * L_);
    stream_ = as_stream(p.hip_stream);
  }
  ~Group() {
    if (h_costs_) (void)hipHostFree(h_costs_);
    if (ev0_) (void)hipEventDestroy(ev0_);
    if (ev1_) (void)hipEventDestroy(ev1_);
  }

  int run(GroupResult &out, double t_start);

 private:
  const qfs_target *tgt_;
  qfs_params p_;
  const qfs_c128 *gates_in_;
  int start0_, S_;
  Arena &arena_;
  int n_ = 0, L_ = 0;
  int64_t N_ = 0;
  std::vector<int32_t> pairs_;
  hipStream_t stream_ = nullptr;

  int M_ = 0, ld_ = 0, Mv_ = 0, ldv_ = 0, m_cap_ = 0, n_train_ = 0, generation_ = 0;
  bool fp64_ = true;
  DevBuf psi64_, phi64_, psiv64_, phiv64_;  // complex128 masters
  DevBuf psi32_, phi32_, psiv32_, phiv32_;  // complex64 working copies (MIXED)
  DevBuf blist_, astate_, vstate_;          // sized for complex128
  DevBuf g64_, g32_;
  DevBuf partials_, dpart_, costs_, slots_, work_;
  double *h_costs_ = nullptr;  // pinned [3 S]: c_train, c_val, c_0
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
  int nslots_ = 0;
  KernelTimer timer_;
  GroupResult *res_ = nullptr;
  double state_bytes(int ld) const {
    return (double)N_ * ld * (fp64_ ? sizeof(c128) : sizeof(c64)) * (double)nslots_;
  }

  int draw_training(int c0, int c1);
  int make_targets(DevBuf &psi, DevBuf &phi, int M, int ld);
  int draw_validation();
  int alloc_states();
  int refresh_working_copies();
  int set_slots(const std::vector<int> &active);
  template <typename R>
  int forward(bool with_c0);
  template <typename R>
  int backward();
  int forward_any(bool with_c0) { return fp64_ ? forward<double>(with_c0) : forward<float>(with_c0); }
  int backward_any() { return fp64_ ? backward<double>() : backward<float>(); }
  int read_costs(std::vector<double> &ct, std::vector<double> &cv, std::vector<double> *c0);
};

int Group::draw_training(int c0, int c1) {
  QFS_TRY(launch_ginibre(N_, c0, c1, ld_, p_.seed, kRoleTrain, 0, psi64_.as<c128>(), stream_));
  QFS_TRY(arena_.alloc(work_, work_bytes_orth(N_, c1)));
  QFS_TRY(orthonormalize_columns(N_, ld_, c0, c1, psi64_.as<c128>(), work_.ptr, stream_));
  arena_.free(work_);
  return QFS_OK;
}

// phi = U psi (dense product, or simulation of the target circuit), FP64.
int Group::make_targets(DevBuf &psi, DevBuf &phi, int M, int ld) {
  const size_t bytes = sizeof(c128) * (size_t)N_ * ld;
  if (tgt_->kind == QFS_TARGET_DENSE) {
    QFS_TRY(launch_zgemm(false, (int)N_, M, (int)N_, cmake(1.0, 0.0),
                         reinterpret_cast<const c128 *>(tgt_->U), (int)N_, psi.as<c128>(), ld,
                         cmake(0.0, 0.0), phi.as<c128>(), ld, stream_));
    return QFS_OK;
  }
  QFS_HIP(hipMemcpyAsync(phi.ptr, psi.ptr, bytes, hipMemcpyDeviceToDevice, stream_));
  const qfs_template *ct = tgt_->circuit;
  Geometry g{n_, (int32_t)N_, ld, M};
  int32_t zero = 0;
  DevBuf slot;
  QFS_TRY(slot.alloc(sizeof(int32_t)));
  QFS_HIP(hipMemcpyAsync(slot.ptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice, stream_));
  GateRef gr{reinterpret_cast<const c128 *>(tgt_->circuit_gates),
             reinterpret_cast<const c128 *>(tgt_->circuit_gates), 0};
  for (int k = 0; k < ct->n_gates; ++k) {
    QFS_TRY(launch_apply<double>(g, ct->pairs[2 * k], ct->pairs[2 * k + 1], k, false, gr,
                                 SBuf<double>{phi.as<c128>(), 0}, SBuf<double>{phi.as<c128>(), 0},
                                 slot.as<int32_t>(), 1, stream_));
  }
  QFS_HIP(hipStreamSynchronize(stream_));
  return QFS_OK;
}

int Group::draw_validation() {
  if (tgt_->kind == QFS_TARGET_SAMPLES) {
    Mv_ = tgt_->n_val;
    ldv_ = (int)even_up(std::max(Mv_, 1));
    if (Mv_ == 0) return QFS_OK;
    QFS_TRY(arena_.alloc(psiv64_, sizeof(c128) * N_ * ldv_));
    QFS_TRY(arena_.alloc(phiv64_, sizeof(c128) * N_ * ldv_));
    const c128 *ps = reinterpret_cast<const c128 *>(tgt_->psi) + (size_t)n_train_ * N_;
    const c128 *ph = reinterpret_cast<const c128 *>(tgt_->phi) + (size_t)n_train_ * N_;
    QFS_TRY(launch_to_internal<double>(N_, Mv_, ldv_, ps, psiv64_.as<c128>(), stream_));
    QFS_TRY(launch_to_internal<double>(N_, Mv_, ldv_, ph, phiv64_.as<c128>(), stream_));
    return QFS_OK;
  }
  Mv_ = p_.m_val > 0 ? p_.m_val : M_;
  if (Mv_ > N_) Mv_ = (int)N_;
  ldv_ = (int)even_up(Mv_);
  QFS_TRY(arena_.alloc(psiv64_, sizeof(c128) * N_ * ldv_));
  QFS_TRY(arena_.alloc(phiv64_, sizeof(c128) * N_ * ldv_));
  QFS_TRY(launch_zero(psiv64_.ptr, psiv64_.bytes, stream_));
  QFS_TRY(launch_ginibre(N_, 0, Mv_, ldv_, p_.seed, kRoleVal, (uint32_t)generation_,
                         psiv64_.as<c128>(), stream_));
  QFS_TRY(arena_.alloc(work_, work_bytes_orth(N_, Mv_)));
  QFS_TRY(orthonormalize_columns(N_, ldv_, 0, Mv_, psiv64_.as<c128>(), work_.ptr, stream_));
  arena_.free(work_);
  return make_targets(psiv64_, phiv64_, Mv_, ldv_);
}

int Group::alloc_states() {
  const size_t state = sizeof(c128) * (size_t)N_ * ld_;
  QFS_TRY(arena_.alloc(blist_, state * (size_t)S_ * (size_t)std::max(L_ - 1, 1)));
  QFS_TRY(arena_.alloc(astate_, state * (size_t)S_));
  QFS_TRY(arena_.alloc(vstate_, sizeof(c128) * (size_t)N_ * ldv_ * (size_t)S_));
  return QFS_OK;
}

int Group::refresh_working_copies() {
  if (p_.precision != QFS_PREC_MIXED) return QFS_OK;
  QFS_TRY(arena_.alloc(psi32_, sizeof(c64) * N_ * ld_));
  QFS_TRY(arena_.alloc(phi32_, sizeof(c64) * N_ * ld_));
  QFS_TRY(launch_narrow(N_ * ld_, psi64_.as<c128>(), psi32_.as<c64>(), stream_));
  QFS_TRY(launch_narrow(N_ * ld_, phi64_.as<c128>(), phi32_.as<c64>(), stream_));
  if (Mv_ > 0) {
    QFS_TRY(arena_.alloc(psiv32_, sizeof(c64) * N_ * ldv_));
    QFS_TRY(arena_.alloc(phiv32_, sizeof(c64) * N_ * ldv_));
    QFS_TRY(launch_narrow(N_ * ldv_, psiv64_.as<c128>(), psiv32_.as<c64>(), stream_));
    QFS_TRY(launch_narrow(N_ * ldv_, phiv64_.as<c128>(), phiv32_.as<c64>(), stream_));
  }
  return QFS_OK;
}

int Group::set_slots(const std::vector<int> &active) {
  nslots_ = (int)active.size();
  if (nslots_ == 0) return QFS_OK;
  QFS_HIP(hipMemcpyAsync(slots_.ptr, active.data(), sizeof(int32_t) * active.size(),
                         hipMemcpyHostToDevice, stream_));
  return QFS_OK;
}

template <typename R>
static cx<R> *cast_state(const DevBuf &b) {
  return static_cast<cx<R> *>(b.ptr);
}

// Forward pass (Fig. pre-comp): B_k = u_k B_{k-1}, k = 1 .. L-1, from the gates as
// they are before the sweep; the validation states go through every gate and their
// Eq. 9 cost is taken against U psi_val (c_val of the current gates). with_c0 also
// takes the training cost of the current gates (needed once per training set).
template <typename R>
int Group::forward(bool with_c0) {
  Geometry g{n_, (int32_t)N_, ld_, M_};
  Geometry gv{n_, (int32_t)N_, ldv_, Mv_};
  const bool f32 = sizeof(R) == 4;
  GateRef gr{g64_.as<c128>(), f32 ? g32_.ptr : g64_.ptr, L_ * 16};
  cx<R> *psi = f32 ? reinterpret_cast<cx<R> *>(psi32_.ptr) : reinterpret_cast<cx<R> *>(psi64_.ptr);
  cx<R> *phi = f32 ? reinterpret_cast<cx<R> *>(phi32_.ptr) : reinterpret_cast<cx<R> *>(phi64_.ptr);
  cx<R> *psiv = f32 ? reinterpret_cast<cx<R> *>(psiv32_.ptr) : reinterpret_cast<cx<R> *>(psiv64_.ptr);
  cx<R> *phiv = f32 ? reinterpret_cast<cx<R> *>(phiv32_.ptr) : reinterpret_cast<cx<R> *>(phiv64_.ptr);
  const int64_t sN = N_ * (int64_t)ld_;
  const int64_t bstride = sN * std::max(L_ - 1, 1);
  cx<R> *B = cast_state<R>(blist_);
  cx<R> *V = cast_state<R>(vstate_);
  const int64_t vstride = N_ * (int64_t)ldv_;
  const int32_t *slots = slots_.as<int32_t>();
  for (int k = 1; k < L_; ++k) {
    const int qa = pairs_[2 * (k - 1)], qb = pairs_[2 * (k - 1) + 1];
    SBuf<R> src = k == 1 ? SBuf<R>{psi, 0} : SBuf<R>{B + (k - 2) * sN, bstride};
    QFS_TRY(timer_.begin(stream_));
    QFS_TRY(launch_apply<R>(g, qa, qb, k - 1, false, gr, src, SBuf<R>{B + (k - 1) * sN, bstride},
                            slots, nslots_, stream_));
    QFS_TRY(timer_.end(stream_, 1, 2.0 * state_bytes(ld_)));
    if (Mv_ > 0) {
      QFS_TRY(timer_.begin(stream_));
      QFS_TRY(launch_apply<R>(gv, qa, qb, k - 1, false, gr,
                              k == 1 ? SBuf<R>{psiv, 0} : SBuf<R>{V, vstride}, SBuf<R>{V, vstride},
                              slots, nslots_, stream_));
      QFS_TRY(timer_.end(stream_, 1, 2.0 * state_bytes(ldv_)));
    }
  }
  const int qa = pairs_[2 * (L_ - 1)], qb = pairs_[2 * (L_ - 1) + 1];
  double *costs = costs_.as<double>();
  if (Mv_ > 0) {
    QFS_TRY(timer_.begin(stream_));
    QFS_TRY(launch_apply_dist<R>(gv, qa, qb, L_ - 1, false, gr,
                                 L_ == 1 ? SBuf<R>{psiv, 0} : SBuf<R>{V, vstride},
                                 SBuf<R>{phiv, 0}, slots, nslots_, 0, dpart_.as<double>(),
                                 costs + S_, stream_));
    QFS_TRY(timer_.end(stream_, 2, 2.0 * state_bytes(ldv_)));
  }
  if (with_c0)
    QFS_TRY(launch_apply_dist<R>(g, qa, qb, L_ - 1, false, gr,
                                 L_ == 1 ? SBuf<R>{psi, 0} : SBuf<R>{B + (L_ - 2) * sN, bstride},
                                 SBuf<R>{phi, 0}, slots, nslots_, 0, dpart_.as<double>(),
                                 costs + 2 * S_, stream_));
  return QFS_OK;
}

// Right-to-left update (Sec. 3; Fig. env_calc_tensor): for k = L-1 .. 0 the backward
// state is moved through the just-updated gate k+1, the environment of gate k is
// reduced against B_k, and gate k is replaced by its polar factor. Then the Eq. 9
// cost of the updated gates from a_0 = C^dagger U psi.
template <typename R>
int Group::backward() {
  Geometry g{n_, (int32_t)N_, ld_, M_};
  const bool f32 = sizeof(R) == 4;
  GateRef gr{g64_.as<c128>(), f32 ? g32_.ptr : g64_.ptr, L_ * 16};
  cx<R> *psi = f32 ? reinterpret_cast<cx<R> *>(psi32_.ptr) : reinterpret_cast<cx<R> *>(psi64_.ptr);
  cx<R> *phi = f32 ? reinterpret_cast<cx<R> *>(phi32_.ptr) : reinterpret_cast<cx<R> *>(phi64_.ptr);
  const int64_t sN = N_ * (int64_t)ld_;
  const int64_t bstride = sN * std::max(L_ - 1, 1);
  cx<R> *B = cast_state<R>(blist_);
  cx<R> *A = cast_state<R>(astate_);
  const int32_t *slots = slots_.as<int32_t>();
  StepScratch sc{partials_.as<c128>(), nullptr};
  for (int k = L_ - 1; k >= 0; --k) {
    const int k_apply = (k == L_ - 1) ? -1 : k + 1;
    SBuf<R> a_in = (k >= L_ - 2) ? SBuf<R>{phi, 0} : SBuf<R>{A, sN};
    SBuf<R> b = k == 0 ? SBuf<R>{psi, 0} : SBuf<R>{B + (k - 1) * sN, bstride};
    QFS_TRY(timer_.begin(stream_));
    QFS_TRY(launch_bwd_step<R>(g, pairs_.data(), k_apply, k, gr, g64_.as<c128>(),
                               f32 ? g32_.ptr : nullptr, p_.beta, a_in, SBuf<R>{A, sN}, b, slots,
                               nslots_, 0, sc, true, stream_));
    QFS_TRY(timer_.end(stream_, 0, (k_apply < 0 ? 2.0 : 3.0) * state_bytes(ld_)));
  }
  const int qa = pairs_[0], qb = pairs_[1];
  QFS_TRY(timer_.begin(stream_));
  QFS_TRY(launch_apply_dist<R>(g, qa, qb, 0, true, gr, L_ == 1 ? SBuf<R>{phi, 0} : SBuf<R>{A, sN},
                               SBuf<R>{psi, 0}, slots, nslots_, 0, dpart_.as<double>(),
                               costs_.as<double>(), stream_));
  QFS_TRY(timer_.end(stream_, 2, 2.0 * state_bytes(ld_)));
  return QFS_OK;
}

int Group::read_costs(std::vector<double> &ct, std::vector<double> &cv, std::vector<double> *c0) {
  QFS_HIP(hipMemcpyAsync(h_costs_, costs_.ptr, sizeof(double) * 3 * S_, hipMemcpyDeviceToHost, stream_));
  QFS_HIP(hipStreamSynchronize(stream_));
  if (res_) QFS_TRY(timer_.flush(*res_));
  for (int s = 0; s < S_; ++s) {
    ct[s] = h_costs_[s];
    cv[s] = h_costs_[S_ + s];
    if (c0) (*c0)[s] = h_costs_[2 * S_ + s];
  }
  return QFS_OK;
}

int Group::run(GroupResult &out, double t_start) {
  const bool samples = tgt_->kind == QFS_TARGET_SAMPLES;
  m_cap_ = (p_.m_max > 0 && p_.m_max < N_) ? p_.m_max : (int)N_;
  if (samples) {
    n_train_ = tgt_->n_samples - tgt_->n_val;
    m_cap_ = std::min(m_cap_, n_train_);
  }
  M_ = std::max(1, std::min(p_.m_init, m_cap_));
  if (p_.fixed_m) m_cap_ = M_;
  ld_ = (int)even_up(M_);
  fp64_ = p_.precision != QFS_PREC_MIXED;
  timer_.on = p_.timing != 0;
  res_ = &out;

  QFS_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_costs_), sizeof(double) * 3 * S_));
  QFS_HIP(hipEventCreate(&ev0_));
  QFS_HIP(hipEventCreate(&ev1_));
  const int Pcap = 4096;
  QFS_TRY(arena_.alloc(partials_, sizeof(c128) * 16 * (size_t)Pcap * S_));
  QFS_TRY(arena_.alloc(dpart_, sizeof(double) * (size_t)Pcap * S_));
  QFS_TRY(arena_.alloc(costs_, sizeof(double) * 3 * S_));
  QFS_TRY(arena_.alloc(slots_, sizeof(int32_t) * S_));

  // training set and A tensor (computed once per training set)
  QFS_TRY(arena_.alloc(psi64_, sizeof(c128) * N_ * ld_));
  QFS_TRY(arena_.alloc(phi64_, sizeof(c128) * N_ * ld_));
  QFS_TRY(launch_zero(psi64_.ptr, psi64_.bytes, stream_));
  if (samples) {
    QFS_TRY(launch_to_internal<double>(N_, M_, ld_, reinterpret_cast<const c128 *>(tgt_->psi),
                                       psi64_.as<c128>(), stream_));
    QFS_TRY(launch_to_internal<double>(N_, M_, ld_, reinterpret_cast<const c128 *>(tgt_->phi),
                                       phi64_.as<c128>(), stream_));
  } else {
    QFS_TRY(draw_training(0, M_));
    QFS_TRY(make_targets(psi64_, phi64_, M_, ld_));
  }
  QFS_TRY(draw_validation());
  QFS_TRY(alloc_states());
  QFS_TRY(refresh_working_copies());

  // initial gates (App. A: random per start from the seed, or given)
  QFS_TRY(arena_.alloc(g64_, sizeof(c128) * 16 * (size_t)L_ * S_));
  QFS_TRY(arena_.alloc(g32_, sizeof(c64) * 16 * (size_t)L_ * S_));
  if (gates_in_) {
    QFS_HIP(hipMemcpyAsync(g64_.ptr, gates_in_ + (size_t)start0_ * L_ * 16,
                           sizeof(c128) * 16 * (size_t)L_ * S_, hipMemcpyDeviceToDevice, stream_));
  } else {
    QFS_TRY(launch_haar_gates(p_.seed, start0_, S_, L_, g64_.as<c128>(), stream_));
  }
  QFS_TRY(launch_narrow((int64_t)16 * L_ * S_, g64_.as<c128>(), g32_.as<c64>(), stream_));

  std::vector<int> status(S_, ST_RUN), reason(S_, QFS_MAX_ITER), iter(S_, 0), z(S_, 0);
  std::vector<int64_t> total(S_, 0);
  std::vector<double> c_prev(S_), ct(S_), cv(S_), c0(S_);
  std::vector<int> active;
  for (int s = 0; s < S_; ++s) active.push_back(s);
  QFS_TRY(set_slots(active));
  int restarts = 0, m_total = M_;
  int64_t round = 0;

  QFS_TRY(forward_any(true));
  QFS_TRY(read_costs(ct, cv, &c0));
  for (int s = 0; s < S_; ++s) {
    c_prev[s] = c0[s];
    ct[s] = c0[s];
    if (Mv_ == 0) cv[s] = ct[s];
  }

  int chosen = -1;
  for (;;) {
    // one sweep of every running start, then the next forward pass (which also gives
    // the validation cost of the post-sweep gates)
    QFS_HIP(hipEventRecord(ev0_, stream_));
    QFS_TRY(backward_any());
    QFS_TRY(forward_any(false));
    QFS_HIP(hipEventRecord(ev1_, stream_));
    std::vector<double> nct(S_), ncv(S_);
    QFS_TRY(read_costs(nct, ncv, nullptr));
    float ms = 0.f;
    QFS_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
    out.sweep_seconds += 1e-3 * ms;
    ++round;
    out.start_sweeps += (int64_t)active.size();

    const bool full = (int64_t)M_ == N_;
    bool any_success = false, any_over = false;
    const bool timed_out = p_.time_budget_s > 0 && now_s() - t_start > p_.time_budget_s;
    for (int s : active) {
      ct[s] = nct[s];
      cv[s] = Mv_ > 0 ? ncv[s] : nct[s];
      iter[s] += 1;
      total[s] += 1;
      const bool improved = std::fabs(c_prev[s]) - std::fabs(ct[s]) > p_.diff_tol_r * std::fabs(ct[s]);
      z[s] = improved ? 0 : z[s] + 1;
      c_prev[s] = ct[s];
      const bool gen_ok = full || Mv_ == 0 || cv[s] <= (1.0 + p_.overtrain_ratio) * ct[s];
      if (ct[s] < p_.dist_tol && gen_ok) {
        status[s] = ST_STOP;
        reason[s] = QFS_SUCCESS;
        any_success = true;
        continue;
      }
      if (iter[s] >= p_.min_iter && !gen_ok) {
        if (M_ < m_cap_) {
          status[s] = ST_OVER;
          any_over = true;
          continue;
        }
        if (ct[s] < p_.dist_tol) {
          status[s] = ST_STOP;
          reason[s] = QFS_NOT_GENERALIZED;
          continue;
        }
      }
      if (iter[s] >= p_.min_iter && z[s] >= p_.plateau_window) {
        status[s] = ST_STOP;
        reason[s] = QFS_PLATEAU;
        continue;
      }
      if (total[s] >= p_.max_iter) {
        status[s] = ST_STOP;
        reason[s] = QFS_MAX_ITER;
        continue;
      }
      if (timed_out) {
        status[s] = ST_STOP;
        reason[s] = QFS_TIMEOUT;
        continue;
      }
    }
    if (any_success) {
      double best = INFINITY;
      for (int s : active)
        if (reason[s] == QFS_SUCCESS && status[s] == ST_STOP && ct[s] < best) {
          best = ct[s];
          chosen = s;
        }
      out.success_round = round;
      break;
    }
    if (any_over) {
      // double-and-restart: extend the training set, keep every gate (App. A)
      const int M_new = std::min(2 * M_, m_cap_);
      const int ld_new = (int)even_up(M_new);
      DevBuf npsi, nphi;
      QFS_TRY(arena_.alloc(npsi, sizeof(c128) * N_ * ld_new));
      QFS_TRY(arena_.alloc(nphi, sizeof(c128) * N_ * ld_new));
      QFS_TRY(launch_zero(npsi.ptr, npsi.bytes, stream_));
      QFS_HIP(hipMemcpy2DAsync(npsi.ptr, sizeof(c128) * ld_new, psi64_.ptr, sizeof(c128) * ld_,
                               sizeof(c128) * M_, N_, hipMemcpyDeviceToDevice, stream_));
      arena_.free(psi64_);
      arena_.free(phi64_);
      std::swap(psi64_.ptr, npsi.ptr);
      std::swap(psi64_.bytes, npsi.bytes);
      std::swap(phi64_.ptr, nphi.ptr);
      std::swap(phi64_.bytes, nphi.bytes);
      const int M_old = M_;
      M_ = M_new;
      ld_ = ld_new;
      if (samples) {
        QFS_TRY(launch_to_internal<double>(N_, M_, ld_, reinterpret_cast<const c128 *>(tgt_->psi),
                                           psi64_.as<c128>(), stream_));
        QFS_TRY(launch_to_internal<double>(N_, M_, ld_, reinterpret_cast<const c128 *>(tgt_->phi),
                                           phi64_.as<c128>(), stream_));
      } else {
        QFS_TRY(draw_training(M_old, M_));
        QFS_TRY(make_targets(psi64_, phi64_, M_, ld_));
        ++generation_;
        arena_.free(psiv64_);
        arena_.free(phiv64_);
        QFS_TRY(draw_validation());
      }
      QFS_TRY(alloc_states());
      QFS_TRY(refresh_working_copies());
      m_total += M_;
      ++restarts;
      active.clear();
      for (int s = 0; s < S_; ++s)
        if (status[s] != ST_STOP) {
          status[s] = ST_RUN;
          iter[s] = 0;
          z[s] = 0;
          active.push_back(s);
        }
      QFS_TRY(set_slots(active));
      QFS_TRY(forward_any(true));
      QFS_TRY(read_costs(nct, ncv, &c0));
      for (int s : active) c_prev[s] = c0[s];
      continue;
    }
    std::vector<int> next;
    for (int s : active)
      if (status[s] == ST_RUN) next.push_back(s);
    if (next.empty()) {
      double best = INFINITY;
      for (int s = 0; s < S_; ++s)
        if (ct[s] < best || chosen < 0) {
          best = ct[s];
          chosen = s;
        }
      break;
    }
    // precision policy: complex128 refinement once the best running start is close
    bool switch_now = false;
    if (!fp64_) {
      double best = INFINITY;
      for (int s : next) best = std::min(best, ct[s]);
      switch_now = best < p_.refine_below;
    }
    if (next.size() != active.size()) {
      // the forward pass just run already holds valid B lists for the survivors
      active = next;
      QFS_TRY(set_slots(active));
    }
    if (switch_now) {
      fp64_ = true;
      out.refined = 1;
      QFS_TRY(forward_any(false));  // B lists again, in complex128, from the FP64 gates
    }
  }

  out.best = start0_ + chosen;
  out.reason = reason[chosen];
  out.c_train = ct[chosen];
  out.c_val = cv[chosen];
  out.m_final = M_;
  out.sweeps = (int)total[chosen];
  out.restarts = restarts;
  out.m_total = m_total;
  out.gates.resize((size_t)L_ * 16);
  QFS_HIP(hipMemcpyAsync(out.gates.data(), g64_.as<c128>() + (size_t)chosen * L_ * 16,
                         sizeof(c128) * 16 * L_, hipMemcpyDeviceToHost, stream_));
  QFS_HIP(hipStreamSynchronize(stream_));
  return QFS_OK;
}

bool better(const GroupResult &a, const GroupResult &b) {
  // success first, then the earlier success round, then the lower training cost
  const bool sa = a.reason == QFS_SUCCESS, sb = b.reason == QFS_SUCCESS;
  if (sa != sb) return sa;
  if (sa && a.success_round != b.success_round) return a.success_round < b.success_round;
  return a.c_train < b.c_train;
}

// App. A: on device out-of-memory, run the starts as two halves (recursively).
int run_split(const qfs_template *t, const qfs_target *tg, const qfs_params &p,
              const qfs_c128 *gates_in, int start0, int S, size_t budget, double t0,
              std::vector<GroupResult> &results) {
  GroupResult r;
  {
    Arena arena;
    arena.budget = budget;
    Group grp(t, tg, p, gates_in, start0, S, arena);
    r.rc = grp.run(r, t0);
  }
  if (r.rc == QFS_ENOMEM && S > 1) {
    (void)hipGetLastError();
    const int h = S / 2;
    QFS_TRY(run_split(t, tg, p, gates_in, start0, h, budget, t0, results));
    return run_split(t, tg, p, gates_in, start0 + h, S - h, budget, t0, results);
  }
  if (r.rc != QFS_OK) return r.rc;
  results.push_back(std::move(r));
  return QFS_OK;
}

int check_gates_unitary(const qfs_c128 *gates_dev, size_t count, hipStream_t s) {
  std::vector<qfs_c128> h(count * 16);
  QFS_HIP(hipMemcpyAsync(h.data(), gates_dev, sizeof(qfs_c128) * h.size(), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  for (size_t gi = 0; gi < count; ++gi) {
    const qfs_c128 *u = h.data() + gi * 16;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < 4; ++k) {
          const qfs_c128 a = u[k * 4 + i], b = u[k * 4 + j];  // conj(u[k][i]) u[k][j]
          re += a.re * b.re + a.im * b.im;
          im += a.re * b.im - a.im * b.re;
        }
        re -= (i == j) ? 1.0 : 0.0;
        if (!std::isfinite(re) || !std::isfinite(im) || std::fabs(re) > 1e-10 || std::fabs(im) > 1e-10) {
          set_error_detail("gates_in: gate " + std::to_string(gi) + " is not unitary to 1e-10");
          return QFS_EINVAL;
        }
      }
  }
  return QFS_OK;
}

}  // namespace
}  // namespace qfs

using namespace qfs;

extern "C" {

const char *qfs_strerror(int code) {
  switch (code) {
    case QFS_OK: return "ok";
    case QFS_EINVAL: return "invalid argument";
    case QFS_ENOMEM: return "device memory budget exceeded";
    case QFS_EDEVICE: return "HIP runtime error";
    case QFS_EUNSUPPORTED: return "unsupported combination";
    case QFS_ENUMERIC: return "orthonormalisation of the sample states failed";
    default: return "unknown error";
  }
}

const char *qfs_last_error_detail(void) { return g_detail.c_str(); }

const char *qfs_version(void) { return "qfs-hip 0.1 (gfx950)"; }

void qfs_default_params(qfs_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dist_tol = 1e-8;
  p->diff_tol_r = 1e-5;
  p->plateau_window = 5;
  p->min_iter = 6;
  p->max_iter = 10000;
  p->m_init = 2;
  p->m_max = 0;
  p->overtrain_ratio = 0.1;
  p->multistarts = 16;
  p->beta = 0.0;
  p->seed = 0;
  p->fixed_m = 0;
  p->m_val = 0;
  p->precision = QFS_PREC_MIXED;
  p->refine_below = 1e-5;
  p->device_mem_budget = 0;
  p->time_budget_s = 0.0;
  p->hip_stream = nullptr;
}

int qfs_instantiate(const qfs_template *tmpl, const qfs_target *target, const qfs_params *params,
                    const qfs_c128 *gates_in, qfs_c128 *gates_out, qfs_result *res) {
  const double t0 = now_s();
  QFS_TRY(validate_template(tmpl));
  if (!target || !params || !gates_out || !res) {
    set_error_detail("null target, params, gates_out or res");
    return QFS_EINVAL;
  }
  const qfs_params &p = *params;
  const int64_t N = int64_t(1) << tmpl->n_qubits;
  if (p.multistarts < 1 || p.m_init < 1 || p.m_init > N || p.max_iter < 1 || p.plateau_window < 1 ||
      !(p.dist_tol >= 0) || !(p.diff_tol_r >= 0) || !(p.overtrain_ratio >= 0) || !(p.beta >= 0) ||
      !(p.beta <= 1) || (p.precision != QFS_PREC_FP64 && p.precision != QFS_PREC_MIXED) ||
      p.m_val < 0 || p.m_val > N) {
    set_error_detail("params out of range");
    return QFS_EINVAL;
  }
  switch (target->kind) {
    case QFS_TARGET_DENSE:
      if (!target->U) return set_error_detail("DENSE target needs U"), QFS_EINVAL;
      break;
    case QFS_TARGET_CIRCUIT:
      QFS_TRY(validate_template(target->circuit));
      if (target->circuit->n_qubits != tmpl->n_qubits || !target->circuit_gates)
        return set_error_detail("CIRCUIT target: qubit count mismatch or no gates"), QFS_EINVAL;
      break;
    case QFS_TARGET_SAMPLES:
      if (!target->psi || !target->phi || target->n_val < 0 || target->n_samples - target->n_val < 1 ||
          target->n_samples - target->n_val > N)
        return set_error_detail("SAMPLES target: bad psi/phi/n_samples/n_val"), QFS_EINVAL;
      break;
    default:
      return set_error_detail("unknown target kind"), QFS_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(p.hip_stream);
  if (gates_in) QFS_TRY(check_gates_unitary(gates_in, (size_t)p.multistarts * tmpl->n_gates, s));
  size_t budget = p.device_mem_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    QFS_HIP(hipMemGetInfo(&fr, &tot));
    budget = (size_t)(0.92 * (double)fr);
  }
  std::vector<GroupResult> results;
  QFS_TRY(run_split(tmpl, target, p, gates_in, 0, p.multistarts, budget, t0, results));
  size_t bi = 0;
  for (size_t i = 1; i < results.size(); ++i)
    if (better(results[i], results[bi])) bi = i;
  const GroupResult &r = results[bi];
  QFS_HIP(hipMemcpyAsync(gates_out, r.gates.data(), sizeof(qfs_c128) * r.gates.size(),
                         hipMemcpyHostToDevice, s));
  QFS_HIP(hipStreamSynchronize(s));
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
    for (int c = 0; c < 3; ++c) {
      res->kernel_launches[c] += x.kl[c];
      res->kernel_seconds[c] += x.ks[c];
      res->kernel_bytes[c] += x.kb[c];
    }
  }
  res->seconds = now_s() - t0;
  return QFS_OK;
}

int qfs_instantiate_samples(const qfs_template *tmpl, const qfs_c128 *psi, const qfs_c128 *phi,
                            int32_t M, double tol, qfs_c128 *gates_out, double *cost_out) {
  qfs_params p;
  qfs_default_params(&p);
  p.multistarts = 1;
  p.m_init = M;
  p.fixed_m = 1;
  p.dist_tol = tol;
  p.precision = QFS_PREC_FP64;
  qfs_target t;
  std::memset(&t, 0, sizeof(t));
  t.kind = QFS_TARGET_SAMPLES;
  t.psi = psi;
  t.phi = phi;
  t.n_samples = M;
  t.n_val = 0;
  qfs_result r;
  QFS_TRY(qfs_instantiate(tmpl, &t, &p, nullptr, gates_out, &r));
  if (cost_out) *cost_out = r.c_train;
  return QFS_OK;
}

// ------------------------------------------------------------------ step entry points
int qfs_draw_states(int32_t n, int32_t M, uint64_t seed, uint32_t role, uint32_t stream,
                    qfs_c128 *out, void *hip_stream) {
  if (n < 1 || n > 24 || M < 1 || (int64_t)M > (int64_t(1) << n) || !out) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = even_up(M);
  DevBuf A, W;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(launch_zero(A.ptr, A.bytes, s));
  QFS_TRY(launch_ginibre(N, 0, M, ld, seed, role, stream, A.as<c128>(), s));
  QFS_TRY(W.alloc(work_bytes_orth(N, M)));
  QFS_TRY(orthonormalize_columns(N, ld, 0, M, A.as<c128>(), W.ptr, s));
  QFS_TRY(launch_from_internal<double>(N, M, ld, A.as<c128>(), reinterpret_cast<c128 *>(out), s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_haar_gates(uint64_t seed, int32_t starts, int32_t L, qfs_c128 *out, void *hip_stream) {
  if (starts < 1 || L < 1 || !out) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  QFS_TRY(launch_haar_gates(seed, 0, starts, L, reinterpret_cast<c128 *>(out), s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

static int one_slot(DevBuf &slot, hipStream_t s) {
  int32_t zero = 0;
  QFS_TRY(slot.alloc(sizeof(int32_t)));
  QFS_HIP(hipMemcpyAsync(slot.ptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
  return QFS_OK;
}

int qfs_apply_gates(int32_t n, int32_t M, qfs_c128 *states, int32_t L, const int32_t *pairs,
                    const qfs_c128 *gates, int32_t dagger, void *hip_stream) {
  qfs_template t{n, L, pairs};
  QFS_TRY(validate_template(&t));
  if (M < 1 || !states || !gates) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = even_up(M);
  DevBuf A, slot;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(one_slot(slot, s));
  QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(states), A.as<c128>(), s));
  Geometry g{n, (int32_t)N, (int32_t)ld, M};
  GateRef gr{reinterpret_cast<const c128 *>(gates), gates, 0};
  for (int i = 0; i < L; ++i) {
    const int k = dagger ? L - 1 - i : i;
    QFS_TRY(launch_apply<double>(g, pairs[2 * k], pairs[2 * k + 1], k, dagger != 0, gr,
                                 SBuf<double>{A.as<c128>(), 0}, SBuf<double>{A.as<c128>(), 0},
                                 slot.as<int32_t>(), 1, s));
  }
  QFS_TRY(launch_from_internal<double>(N, M, ld, A.as<c128>(), reinterpret_cast<c128 *>(states), s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_dense_apply(int32_t n, int32_t M, const qfs_c128 *U, const qfs_c128 *psi, qfs_c128 *out,
                    void *hip_stream) {
  if (n < 1 || n > 16 || M < 1 || !U || !psi || !out) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = even_up(M);
  DevBuf A, B;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(B.alloc(sizeof(c128) * N * ld));
  QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(psi), A.as<c128>(), s));
  QFS_TRY(launch_zgemm(false, (int)N, (int)ld, (int)N, cmake(1.0, 0.0), reinterpret_cast<const c128 *>(U),
                       (int)N, A.as<c128>(), (int)ld, cmake(0.0, 0.0), B.as<c128>(), (int)ld, s));
  QFS_TRY(launch_from_internal<double>(N, M, ld, B.as<c128>(), reinterpret_cast<c128 *>(out), s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_environment(int32_t n, int32_t M, const qfs_c128 *a, const qfs_c128 *b, int32_t qa,
                    int32_t qb, qfs_c128 *gamma, void *hip_stream) {
  const int32_t pr[2] = {qa, qb};
  qfs_template t{n, 1, pr};
  QFS_TRY(validate_template(&t));
  if (M < 1 || !a || !b || !gamma) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = even_up(M);
  DevBuf A, B, slot, part;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(B.alloc(sizeof(c128) * N * ld));
  QFS_TRY(part.alloc(sizeof(c128) * 16 * 4096));
  QFS_TRY(one_slot(slot, s));
  QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(a), A.as<c128>(), s));
  QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(b), B.as<c128>(), s));
  Geometry g{n, (int32_t)N, (int32_t)ld, M};
  GateRef gr{nullptr, nullptr, 0};
  StepScratch sc{part.as<c128>(), reinterpret_cast<c128 *>(gamma)};
  QFS_TRY(launch_bwd_step<double>(g, pr, -1, 0, gr, nullptr, nullptr, 0.0,
                                  SBuf<double>{A.as<c128>(), 0}, SBuf<double>{A.as<c128>(), 0},
                                  SBuf<double>{B.as<c128>(), 0}, slot.as<int32_t>(), 1, 0, sc,
                                  false, s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_polar_update(int32_t count, const qfs_c128 *gamma, double beta, qfs_c128 *u,
                     void *hip_stream) {
  if (count < 0 || (count > 0 && (!gamma || !u)) || !(beta >= 0.0 && beta <= 1.0)) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  QFS_TRY(launch_polar_batch(count, reinterpret_cast<const c128 *>(gamma), beta,
                             reinterpret_cast<c128 *>(u), s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_state_distance(int32_t n, int32_t M, const qfs_c128 *x, const qfs_c128 *y, double *result,
                       void *hip_stream) {
  if (n < 2 || n > 24 || M < 1 || !x || !y || !result) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = even_up(M);
  DevBuf A, B, slot, part, out;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(B.alloc(sizeof(c128) * N * ld));
  QFS_TRY(part.alloc(sizeof(double) * 4096));
  QFS_TRY(out.alloc(16));
  QFS_TRY(one_slot(slot, s));
  QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(x), A.as<c128>(), s));
  QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(y), B.as<c128>(), s));
  Geometry g{n, (int32_t)N, (int32_t)ld, M};
  GateRef gr{nullptr, nullptr, 0};
  QFS_TRY(launch_apply_dist<double>(g, 0, 1, -1, false, gr, SBuf<double>{A.as<c128>(), 0},
                                    SBuf<double>{B.as<c128>(), 0}, slot.as<int32_t>(), 1, 0,
                                    part.as<double>(), out.as<double>(), s));
  QFS_HIP(hipMemcpyAsync(result, out.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_sweep(int32_t n, int32_t L, const int32_t *pairs, int32_t M, const qfs_c128 *psi,
              const qfs_c128 *phi, int32_t starts, qfs_c128 *gates, int32_t precision, double beta,
              double *c_train, void *hip_stream) {
  qfs_template t{n, L, pairs};
  QFS_TRY(validate_template(&t));
  if (M < 1 || (int64_t)M > (int64_t(1) << n) || starts < 1 || !psi || !phi || !gates || !c_train ||
      (precision != QFS_PREC_FP64 && precision != QFS_PREC_MIXED) || !(beta >= 0 && beta <= 1))
    return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = even_up(M);
  const bool f32 = precision == QFS_PREC_MIXED;
  const size_t b = f32 ? sizeof(c64) : sizeof(c128);
  DevBuf ps, ph, Bl, As, g32, slots, part, dpart, costs;
  QFS_TRY(ps.alloc(b * N * ld));
  QFS_TRY(ph.alloc(b * N * ld));
  QFS_TRY(Bl.alloc(b * N * ld * (size_t)std::max(L - 1, 1) * starts));
  QFS_TRY(As.alloc(b * N * ld * starts));
  QFS_TRY(g32.alloc(sizeof(c64) * 16 * (size_t)L * starts));
  QFS_TRY(slots.alloc(sizeof(int32_t) * starts));
  QFS_TRY(part.alloc(sizeof(c128) * 16 * 4096 * (size_t)starts));
  QFS_TRY(dpart.alloc(sizeof(double) * 4096 * (size_t)starts));
  QFS_TRY(costs.alloc(sizeof(double) * starts));
  std::vector<int32_t> sl(starts);
  for (int i = 0; i < starts; ++i) sl[i] = i;
  QFS_HIP(hipMemcpyAsync(slots.ptr, sl.data(), sizeof(int32_t) * starts, hipMemcpyHostToDevice, s));
  if (f32) {
    QFS_TRY(launch_to_internal<float>(N, M, ld, reinterpret_cast<const c128 *>(psi), ps.as<c64>(), s));
    QFS_TRY(launch_to_internal<float>(N, M, ld, reinterpret_cast<const c128 *>(phi), ph.as<c64>(), s));
    QFS_TRY(launch_narrow((int64_t)16 * L * starts, reinterpret_cast<const c128 *>(gates), g32.as<c64>(), s));
  } else {
    QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(psi), ps.as<c128>(), s));
    QFS_TRY(launch_to_internal<double>(N, M, ld, reinterpret_cast<const c128 *>(phi), ph.as<c128>(), s));
  }
  Geometry g{n, (int32_t)N, (int32_t)ld, M};
  c128 *g64 = reinterpret_cast<c128 *>(gates);
  GateRef gr{g64, f32 ? g32.ptr : static_cast<void *>(g64), L * 16};
  const int64_t sN = N * ld;
  const int64_t bstride = sN * std::max(L - 1, 1);
  const int32_t *sp = slots.as<int32_t>();
  StepScratch sc{part.as<c128>(), nullptr};
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    cx<R> *P0 = static_cast<cx<R> *>(ps.ptr), *F0 = static_cast<cx<R> *>(ph.ptr);
    cx<R> *Bp = static_cast<cx<R> *>(Bl.ptr), *Ap = static_cast<cx<R> *>(As.ptr);
    for (int k = 1; k < L; ++k) {
      SBuf<R> src = k == 1 ? SBuf<R>{P0, 0} : SBuf<R>{Bp + (k - 2) * sN, bstride};
      QFS_TRY(launch_apply<R>(g, pairs[2 * (k - 1)], pairs[2 * (k - 1) + 1], k - 1, false, gr, src,
                              SBuf<R>{Bp + (k - 1) * sN, bstride}, sp, starts, s));
    }
    for (int k = L - 1; k >= 0; --k) {
      const int ka = (k == L - 1) ? -1 : k + 1;
      SBuf<R> a_in = (k >= L - 2) ? SBuf<R>{F0, 0} : SBuf<R>{Ap, sN};
      SBuf<R> bb = k == 0 ? SBuf<R>{P0, 0} : SBuf<R>{Bp + (k - 1) * sN, bstride};
      QFS_TRY(launch_bwd_step<R>(g, pairs, ka, k, gr, g64, f32 ? g32.ptr : nullptr, beta, a_in,
                                 SBuf<R>{Ap, sN}, bb, sp, starts, 0, sc, true, s));
    }
    QFS_TRY(launch_apply_dist<R>(g, pairs[0], pairs[1], 0, true, gr,
                                 L == 1 ? SBuf<R>{F0, 0} : SBuf<R>{Ap, sN}, SBuf<R>{P0, 0}, sp,
                                 starts, 0, dpart.as<double>(),
                                 costs.as<double>(), s));
    return QFS_OK;
  };
  if (f32)
    QFS_TRY(run(float{}));
  else
    QFS_TRY(run(double{}));
  QFS_HIP(hipMemcpyAsync(c_train, costs.ptr, sizeof(double) * starts, hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

}  // extern "C"
