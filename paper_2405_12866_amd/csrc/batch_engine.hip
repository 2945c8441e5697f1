// Host side of the batched engine: problem setup, job queues grouped by size class,
// the work-group-size autotuner, and the per-problem decisions between launches
// (Sec. 3 success relations and double-and-restart; App. A plateau, min/max_iter,
// multistarts) for qfs_instantiate_batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.h"

namespace qfs {
namespace {

double bnow() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int to_reason(int st) {
  switch (st) {
    case BJ_SUCCESS: return QFS_SUCCESS;
    case BJ_PLATEAU: return QFS_PLATEAU;
    case BJ_NOT_GEN: return QFS_NOT_GENERALIZED;
    case BJ_TIMEOUT: return QFS_TIMEOUT;
    default: return QFS_MAX_ITER;
  }
}

bool terminal(int st) {
  return st == BJ_SUCCESS || st == BJ_PLATEAU || st == BJ_MAX_ITER || st == BJ_NOT_GEN ||
         st == BJ_TIMEOUT || st == BJ_SKIP;
}

// Autotuner cache: (precision, LDS bucket) -> work-group size. Process-wide.
std::mutex g_tune_mu;
std::map<std::pair<int, size_t>, int> g_tune;

struct ClassKey {
  int fp64;
  size_t bucket;  // bytes of the two state sets, rounded up to a power of two
  bool operator<(const ClassKey &o) const { return std::tie(fp64, bucket) < std::tie(o.fp64, o.bucket); }
};

size_t pow2_at_least(size_t x, size_t lo) {
  size_t b = lo;
  while (b < x) b <<= 1;
  return b;
}

constexpr size_t kLdsLimit = 128 * 1024;

// QFS_BATCH_TRACE=1 prints one line per persistent launch to stderr (tuning aid).
bool batch_trace() {
  static const bool on = [] {
    const char *e = std::getenv("QFS_BATCH_TRACE");
    return e && std::atoi(e) != 0;
  }();
  return on;
}
constexpr int kCUs = 256;
constexpr int kSideStreams = 8;

// Timing events of one call, released on every return path.
struct TimingEvents {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int create() {
    QFS_HIP(hipEventCreate(&e0));
    QFS_HIP(hipEventCreate(&e1));
    return QFS_OK;
  }
  ~TimingEvents() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Pooled streams and per-call join events for concurrent launches.
struct StreamSet {
  hipStream_t s[kSideStreams] = {};
  hipEvent_t ev[kSideStreams] = {};
  int create() {
    for (int i = 0; i < kSideStreams; ++i) {
      QFS_TRY(pool_stream(8 + i, &s[i]));
      QFS_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    }
    return QFS_OK;
  }
  ~StreamSet() {
    for (int i = 0; i < kSideStreams; ++i)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
  }
};

int default_threads(size_t bucket, int fp64) {
  const size_t amps = bucket / (fp64 ? 16 : 8) / 2;  // per state set
  if (amps <= 1024) return 64;
  if (amps <= 8192) return 128;
  return 256;
}

int grid_for(size_t lds, int threads, int njobs) {
  int wpc = 2048 / threads;
  if (lds > 0) wpc = std::min<int>(wpc, (int)((160 * 1024) / (lds + 8192)));  // + static LDS
  wpc = std::max(1, wpc);
  return std::max(1, std::min(njobs, kCUs * wpc));
}

}  // namespace
}  // namespace qfs

using namespace qfs;

int qfs::batch_instantiate(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                           const qfs_params *params, qfs_c128 *const *gates_out, qfs_result *res,
                           const BatchOpts &opts) {
  const double t0 = bnow();
  if (P < 1 || !tmpl || !targets || !params || !gates_out || !res) {
    set_error_detail("batch: null argument or P < 1");
    return QFS_EINVAL;
  }
  const qfs_params &p = *params;
  if (p.multistarts < 1 || p.m_init < 1 || p.max_iter < 1 || p.plateau_window < 1 || !(p.beta >= 0) ||
      !(p.beta <= 1) || (p.precision != QFS_PREC_FP64 && p.precision != QFS_PREC_MIXED) || p.m_val < 0 ||
      p.batch_sweeps < 0 || (p.batch_threads != 0 && p.batch_threads != 64 && p.batch_threads != 128 &&
                             p.batch_threads != 256)) {
    set_error_detail("batch: params out of range");
    return QFS_EINVAL;
  }
  if (p.full_unitary) {
    set_error_detail("batch: full_unitary is a qfs_instantiate mode");
    return QFS_EUNSUPPORTED;
  }
  const int S = p.multistarts;
  if (opts.independent && !p.fixed_m) {
    set_error_detail("batch: independent starts need fixed_m");
    return QFS_EINVAL;
  }
  // sweeps per launch: fixed when given; otherwise 8, raised as the set of running jobs
  // thins out (a long tail of slowly converging problems then costs few round trips)
  const bool adaptive_k = p.batch_sweeps == 0;
  const int K0 = p.batch_sweeps > 0 ? p.batch_sweeps : 8;
  hipStream_t st = static_cast<hipStream_t>(p.hip_stream);

  // ---------------------------------------------------------------- validation + sizes
  std::vector<BProb> hp(P);
  std::vector<size_t> off_psi(P), off_psiv(P), off_coef(P), off_g(P), off_pairs(P), off_tpairs(P),
      off_kinds(P);
  size_t c128s = 0, ints = 0;
  for (int i = 0; i < P; ++i) {
    const qfs_template &t = tmpl[i];
    const qfs_target &g = targets[i];
    if (t.n_qubits < 2 || t.n_qubits > 10 || t.n_gates < 1 || !t.pairs) {
      set_error_detail("batch: problem " + std::to_string(i) + ": need 2 <= n_qubits <= 10, n_gates >= 1");
      return t.n_qubits > 10 ? QFS_EUNSUPPORTED : QFS_EINVAL;
    }
    for (int k = 0; k < t.n_gates; ++k) {
      const int a = t.pairs[2 * k], b = t.pairs[2 * k + 1];
      if (a < 0 || b < 0 || a >= t.n_qubits || b >= t.n_qubits || a == b) {
        set_error_detail("batch: problem " + std::to_string(i) + ": invalid qubit pair");
        return QFS_EINVAL;
      }
      if (t.kinds) {
        const int kind = t.kinds[k];
        if (kind != QFS_GATE_2Q && kind != QFS_GATE_1Q && kind != QFS_GATE_FIXED) {
          set_error_detail("batch: problem " + std::to_string(i) + ": unknown gate kind");
          return QFS_EINVAL;
        }
        if (kind == QFS_GATE_FIXED && !t.fixed_gates) {
          set_error_detail("batch: problem " + std::to_string(i) + ": constant gates need fixed_gates");
          return QFS_EINVAL;
        }
      }
    }
    const int N = 1 << t.n_qubits;
    BProb &d = hp[i];
    std::memset(&d, 0, sizeof(d));
    d.n = t.n_qubits;
    d.L = t.n_gates;
    d.kind = g.kind;
    d.seed = opts.seeds ? opts.seeds[i] : p.seed + (uint64_t)i;
    d.done_sweep = kNoSweep;
    d.over_sweep = kNoSweep;
    int mcap = (p.m_max > 0 && p.m_max < N) ? p.m_max : N;
    int mvcap = 0;
    if (g.kind == QFS_TARGET_SAMPLES) {
      if (!g.psi || !g.phi || g.n_val < 0 || g.n_samples - g.n_val < 1 || g.n_samples - g.n_val > N) {
        set_error_detail("batch: problem " + std::to_string(i) + ": bad SAMPLES target");
        return QFS_EINVAL;
      }
      d.n_train = g.n_samples - g.n_val;
      mcap = std::min(mcap, d.n_train);
      d.s_psi = reinterpret_cast<const c128 *>(g.psi);
      d.s_phi = reinterpret_cast<const c128 *>(g.phi);
    } else if (g.kind == QFS_TARGET_DENSE) {
      if (!g.U) return set_error_detail("batch: DENSE target needs U"), QFS_EINVAL;
      d.U = reinterpret_cast<const c128 *>(g.U);
    } else if (g.kind == QFS_TARGET_CIRCUIT) {
      if (!g.circuit || g.circuit->n_qubits != t.n_qubits || g.circuit->n_gates < 0 || !g.circuit_gates ||
          (g.circuit->n_gates > 0 && !g.circuit->pairs))
        return set_error_detail("batch: bad CIRCUIT target"), QFS_EINVAL;
      d.Lt = g.circuit->n_gates;
      d.tgates = reinterpret_cast<const c128 *>(g.circuit_gates);
    } else {
      return set_error_detail("batch: unknown target kind"), QFS_EINVAL;
    }
    const int m_init = opts.m_init ? opts.m_init[i] : p.m_init;
    const int s_lo = opts.start_lo ? opts.start_lo[i] : 0;
    const int s_hi = opts.starts ? opts.starts[i] : S;
    if (m_init < 1 || s_lo < 0 || s_hi > S || s_lo >= s_hi) {
      set_error_detail("batch: problem " + std::to_string(i) + ": need m_init >= 1 and 0 <= first start < starts <= multistarts");
      return QFS_EINVAL;
    }
    d.M = std::max(1, std::min(m_init, mcap));
    if (p.fixed_m) mcap = d.M;
    d.mcap = mcap;
    d.full = d.M == N;
    if (g.kind == QFS_TARGET_SAMPLES) {
      d.Mv = g.n_val;
      mvcap = g.n_val;
    } else {
      d.Mv = p.m_val > 0 ? std::min(p.m_val, N) : d.M;
      mvcap = p.m_val > 0 ? std::min(p.m_val, N) : mcap;
    }
    off_psi[i] = c128s;
    c128s += 2 * (size_t)mcap * N;
    off_psiv[i] = c128s;
    c128s += 2 * (size_t)std::max(mvcap, 1) * N;
    off_coef[i] = c128s;
    c128s += (size_t)std::max(mcap, mvcap) + 1;
    off_g[i] = c128s;
    c128s += 2 * (size_t)S * t.n_gates * 16;
    off_pairs[i] = ints;
    ints += 2 * (size_t)t.n_gates;
    off_tpairs[i] = ints;
    ints += 2 * (size_t)d.Lt;
    off_kinds[i] = ints;
    if (t.kinds) ints += (size_t)t.n_gates;
  }
  for (int i = 0; i < P; ++i) {
    bool any_fixed = false;
    for (int k = 0; tmpl[i].kinds && k < tmpl[i].n_gates; ++k) any_fixed |= tmpl[i].kinds[k] == QFS_GATE_FIXED;
    if (any_fixed)
      QFS_TRY(check_gates_unitary(tmpl[i].fixed_gates, (size_t)tmpl[i].n_gates, tmpl[i].n_gates, tmpl[i].kinds,
                                  true, "fixed_gates", st));
  }
  // ---------------------------------------------------------------- device memory
  size_t fr = 0, tot = 0;
  int dev = 0;
  QFS_HIP(hipMemGetInfo(&fr, &tot));
  QFS_HIP(hipGetDevice(&dev));
  // (blocks the single-problem engine caches are freed on demand by DevBuf::alloc)
  const size_t budget =
      p.device_mem_budget ? p.device_mem_budget : (size_t)(0.9 * (double)(fr + device_cache_held(dev)));
  const size_t njobs_all = (size_t)P * S;
  const size_t need = c128s * sizeof(c128) + ints * 4 + njobs_all * (sizeof(BJob) + 8) + P * sizeof(BProb);
  if (need > budget) {
    set_error_detail("batch: problem data needs " + std::to_string(need) + " bytes of device memory");
    return QFS_ENOMEM;
  }
  DevBuf dmem, dints, dprobs, djobs, dqueue, dhead, dtodo, dm0, dprob_of, dfirst;
  QFS_TRY(dmem.alloc(c128s * sizeof(c128)));
  QFS_TRY(dints.alloc(std::max<size_t>(ints, 1) * 4));
  c128 *base = dmem.as<c128>();
  int32_t *ibase = dints.as<int32_t>();
  std::vector<int32_t> hints(std::max<size_t>(ints, 1));
  for (int i = 0; i < P; ++i) {
    BProb &d = hp[i];
    const int N = 1 << d.n;
    const int mvcap = (int)((off_coef[i] - off_psiv[i]) / (2 * (size_t)N));
    d.psi = base + off_psi[i];
    d.phi = d.psi + (size_t)d.mcap * N;
    d.psiv = base + off_psiv[i];
    d.phiv = d.psiv + (size_t)mvcap * N;
    d.coef = base + off_coef[i];
    d.g64 = base + off_g[i];
    d.vst = d.g64 + (size_t)S * d.L * 16;
    std::memcpy(hints.data() + off_pairs[i], tmpl[i].pairs, sizeof(int32_t) * 2 * d.L);
    d.pairs = ibase + off_pairs[i];
    if (tmpl[i].kinds) {
      std::memcpy(hints.data() + off_kinds[i], tmpl[i].kinds, sizeof(int32_t) * d.L);
      d.kinds = ibase + off_kinds[i];
      d.fixed = reinterpret_cast<const c128 *>(tmpl[i].fixed_gates);
    }
    if (d.kind == QFS_TARGET_CIRCUIT && d.Lt > 0) {
      std::memcpy(hints.data() + off_tpairs[i], targets[i].circuit->pairs, sizeof(int32_t) * 2 * d.Lt);
      d.tpairs = ibase + off_tpairs[i];
    }
  }
  QFS_HIP(hipMemcpyAsync(dints.ptr, hints.data(), sizeof(int32_t) * hints.size(), hipMemcpyHostToDevice, st));
  QFS_TRY(dprobs.alloc(sizeof(BProb) * P));
  QFS_HIP(hipMemcpyAsync(dprobs.ptr, hp.data(), sizeof(BProb) * P, hipMemcpyHostToDevice, st));
  std::vector<BJob> jobs(njobs_all);
  for (int i = 0; i < P; ++i)
    for (int s = 0; s < S; ++s) {
      BJob &j = jobs[(size_t)i * S + s];
      std::memset(&j, 0, sizeof(j));
      j.prob = i;
      j.start = s;
      const bool run = (!opts.starts || s < opts.starts[i]) && (!opts.start_lo || s >= opts.start_lo[i]);
      const bool park = !run && opts.park_rest && opts.starts && s >= opts.starts[i] &&
                        (!opts.start_lo || s >= opts.start_lo[i]);
      j.status = run ? BJ_RUN : (park ? BJ_PARKED : BJ_SKIP);
      j.c_train = j.c_val = HUGE_VAL;
      j.need_c0 = 1;
      j.fp64 = p.precision == QFS_PREC_FP64 ? 1 : 0;
    }
  QFS_TRY(djobs.alloc(sizeof(BJob) * njobs_all));
  QFS_HIP(hipMemcpyAsync(djobs.ptr, jobs.data(), sizeof(BJob) * njobs_all, hipMemcpyHostToDevice, st));

  // ---------------------------------------------------------------- setup + gates
  {
    std::vector<int32_t> todo(P), m0(P, 0), prob_of, first(P);
    for (int i = 0; i < P; ++i) todo[i] = i;
    int total = 0;
    for (int i = 0; i < P; ++i) {
      first[i] = total;
      total += S * hp[i].L;
    }
    prob_of.resize(total);
    for (int i = 0; i < P; ++i)
      for (int e = 0; e < S * hp[i].L; ++e) prob_of[first[i] + e] = i;
    QFS_TRY(dtodo.alloc(sizeof(int32_t) * P));
    QFS_TRY(dm0.alloc(sizeof(int32_t) * P));
    QFS_TRY(dprob_of.alloc(sizeof(int32_t) * total));
    QFS_TRY(dfirst.alloc(sizeof(int32_t) * P));
    QFS_HIP(hipMemcpyAsync(dtodo.ptr, todo.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, st));
    QFS_HIP(hipMemcpyAsync(dm0.ptr, m0.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, st));
    QFS_HIP(hipMemcpyAsync(dprob_of.ptr, prob_of.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice, st));
    QFS_HIP(hipMemcpyAsync(dfirst.ptr, first.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, st));
    QFS_TRY(launch_batch_setup(dprobs.as<BProb>(), dtodo.as<int32_t>(), P, dm0.as<int32_t>(), st));
    QFS_TRY(launch_batch_gates(dprobs.as<BProb>(), dprob_of.as<int32_t>(), dfirst.as<int32_t>(), total, st));
    QFS_HIP(hipStreamSynchronize(st));
  }

  BParams bp;
  bp.dist_tol = p.dist_tol;
  bp.diff_tol_r = p.diff_tol_r;
  bp.overtrain_ratio = p.overtrain_ratio;
  bp.beta = p.beta;
  bp.beta_normalized = p.beta_normalized != 0;
  bp.refine_below = p.refine_below;
  bp.plateau_window = p.plateau_window;
  bp.min_iter = p.min_iter;
  bp.max_iter = p.max_iter;
  bp.mixed = p.precision == QFS_PREC_MIXED ? 1 : 0;
  bp.independent = opts.independent ? 1 : 0;

  QFS_TRY(dqueue.alloc(sizeof(int32_t) * njobs_all));
  QFS_TRY(dhead.alloc(256));
  DevBuf scratch;
  std::vector<int> finished(P, 0), restarts(P, 0), m_total(P, 0), winner(P, -1);
  for (int i = 0; i < P; ++i) m_total[i] = hp[i].M;
  int remaining = P;
  double kernel_seconds = 0.0;
  TimingEvents tev;
  QFS_TRY(tev.create());
  hipEvent_t e0 = tev.e0, e1 = tev.e1;
  // side streams for concurrent class launches (default priority)
  StreamSet streams;
  QFS_TRY(streams.create());
  hipStream_t *side = streams.s;
  hipEvent_t *side_done = streams.ev;
  std::vector<int32_t> queue;

  while (remaining > 0) {
    // group runnable jobs by (precision, LDS bucket); longest first inside a class
    std::map<ClassKey, std::vector<int32_t>> classes;
    for (size_t j = 0; j < njobs_all; ++j) {
      const BJob &J = jobs[j];
      if (finished[J.prob] || J.status != BJ_RUN) continue;
      const BProb &d = hp[J.prob];
      const size_t cb = J.fp64 ? sizeof(c128) : sizeof(c64);
      const size_t bytes = ((size_t)std::max(d.M, d.Mv) + d.M) * ((size_t)1 << d.n) * cb;
      classes[ClassKey{J.fp64, pow2_at_least(bytes, 4096)}].push_back((int32_t)j);
    }
    if (classes.empty()) break;
    int K = K0;
    if (adaptive_k) {
      size_t runnable = 0;
      for (auto &kv : classes) runnable += kv.second.size();
      while (K < 256 && runnable * (size_t)(K / K0) * 4 <= njobs_all) K *= 2;
    }
    // Size classes are launched concurrently on side streams (each with its own queue
    // segment, queue head and scratch region); a class whose work-group size is not
    // known yet is first autotuned on the call's stream: its jobs are dealt to three
    // parts run with 64, 128 and 256 threads, one after the other.
    struct Launch {
      ClassKey key;
      int threads, grid, nj;
      size_t qoff, soff;
    };
    std::vector<Launch> plan;
    size_t qfill = 0, sfill = 0;
    std::vector<int32_t> qhost;
    qhost.reserve(njobs_all);
    for (auto &kv : classes) {
      std::vector<int32_t> &ids = kv.second;
      std::sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
        const BProb &pa = hp[jobs[a].prob], &pb = hp[jobs[b].prob];
        const double ca = (double)pa.L * ((double)pa.M + pa.Mv) * (1 << pa.n);
        const double cb2 = (double)pb.L * ((double)pb.M + pb.Mv) * (1 << pb.n);
        return ca > cb2;
      });
      const ClassKey key = kv.first;
      const bool use_lds = key.bucket <= kLdsLimit;
      const size_t lds = use_lds ? key.bucket : 0;
      int chosen = p.batch_threads;
      if (!chosen && !use_lds) chosen = 512;  // global-scratch states: wider groups
      if (!chosen) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find({key.fp64, key.bucket});
        if (it != g_tune.end()) chosen = it->second;
      }
      if (!chosen && ids.size() >= 3 * 64) {
        // autotune on the call's stream: the class's jobs (longest first) dealt round robin
        // to three parts of like size mix, run with 64, 128 and 256 threads one after the
        // other; a part's rate is the work its jobs did in the launch (their own work
        // counters, so jobs that stop early count what they ran) per millisecond
        const int cands[3] = {64, 128, 256};
        std::vector<int32_t> part_ids[3];
        for (size_t q = 0; q < ids.size(); ++q) part_ids[q % 3].push_back(ids[q]);
        float part_ms[3] = {0.f, 0.f, 0.f};
        for (int part = 0; part < 3; ++part) {
          const int nj = (int)part_ids[part].size();
          const int threads = cands[part];
          QFS_HIP(hipMemcpyAsync(dqueue.ptr, part_ids[part].data(), sizeof(int32_t) * nj, hipMemcpyHostToDevice, st));
          QFS_TRY(launch_zero(dhead.ptr, 16, st));
          const int grid = grid_for(lds, threads, nj);
          BatchArgs a;
          a.jobs = djobs.as<BJob>();
          a.probs = dprobs.as<BProb>();
          a.queue = dqueue.as<int32_t>();
          a.njobs = nj;
          a.queue_head = dhead.as<int32_t>();
          a.sweeps_per_launch = K;
          a.hp = bp;
          a.scratch = nullptr;
          a.scratch_slot_bytes = 0;
          QFS_HIP(hipEventRecord(e0, st));
          QFS_TRY(launch_batch_sweep(a, key.fp64 != 0, threads, grid, lds, st));
          QFS_HIP(hipEventRecord(e1, st));
          QFS_HIP(hipEventSynchronize(e1));
          QFS_HIP(hipEventElapsedTime(&part_ms[part], e0, e1));
          kernel_seconds += 1e-3 * part_ms[part];
          if (batch_trace())
            std::fprintf(stderr, "qfs batch: tune fp64=%d state_bytes<=%zu threads=%d jobs=%d grid=%d %.3f ms\n",
                         key.fp64, key.bucket, threads, nj, grid, part_ms[part]);
        }
        std::vector<BJob> after(njobs_all);
        QFS_HIP(hipMemcpyAsync(after.data(), djobs.ptr, sizeof(BJob) * njobs_all, hipMemcpyDeviceToHost, st));
        QFS_HIP(hipStreamSynchronize(st));
        double best_rate = -1.0;
        int best_threads = 64;
        for (int part = 0; part < 3; ++part) {
          double work = 0.0;
          for (int32_t j : part_ids[part]) work += after[j].work - jobs[j].work;
          const double rate = work / std::max(1e-6, (double)part_ms[part]);
          if (rate > best_rate) {
            best_rate = rate;
            best_threads = cands[part];
          }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[{key.fp64, key.bucket}] = best_threads;
        continue;
      }
      if (!chosen) chosen = default_threads(key.bucket, key.fp64);
      Launch l;
      l.key = key;
      l.threads = chosen;
      l.nj = (int)ids.size();
      l.grid = grid_for(lds, chosen, l.nj);
      l.qoff = qfill;
      qhost.insert(qhost.end(), ids.begin(), ids.end());
      qfill += ids.size();
      l.soff = sfill;
      if (!use_lds) sfill += (size_t)l.grid * key.bucket;
      plan.push_back(l);
    }
    if (!plan.empty()) {
      const int nl = (int)plan.size();
      if ((size_t)nl * 16 * sizeof(int32_t) > dhead.bytes) QFS_TRY(dhead.alloc((size_t)nl * 16 * sizeof(int32_t)));
      if (sfill > scratch.bytes) QFS_TRY(scratch.alloc(sfill));
      QFS_HIP(hipMemcpyAsync(dqueue.ptr, qhost.data(), sizeof(int32_t) * qfill, hipMemcpyHostToDevice, st));
      QFS_TRY(launch_zero(dhead.ptr, (size_t)nl * 16 * sizeof(int32_t), st));
      QFS_HIP(hipEventRecord(e0, st));
      const int ns = std::min(nl, kSideStreams);
      for (int c = 0; c < ns; ++c) QFS_HIP(hipStreamWaitEvent(side[c], e0, 0));
      for (int c = 0; c < nl; ++c) {
        const Launch &l = plan[c];
        BatchArgs a;
        a.jobs = djobs.as<BJob>();
        a.probs = dprobs.as<BProb>();
        a.queue = dqueue.as<int32_t>() + l.qoff;
        a.njobs = l.nj;
        a.queue_head = dhead.as<int32_t>() + 16 * c;
        a.sweeps_per_launch = K;
        a.hp = bp;
        const bool use_lds = l.key.bucket <= kLdsLimit;
        a.scratch = use_lds ? nullptr : scratch.as<char>() + l.soff;
        a.scratch_slot_bytes = use_lds ? 0 : l.key.bucket;
        QFS_TRY(launch_batch_sweep(a, l.key.fp64 != 0, l.threads, l.grid, use_lds ? l.key.bucket : 0,
                                   side[c % ns]));
        if (batch_trace())
          std::fprintf(stderr, "qfs batch: K=%d fp64=%d state_bytes<=%zu threads=%d jobs=%d grid=%d\n", K,
                       l.key.fp64, l.key.bucket, l.threads, l.nj, l.grid);
      }
      for (int c = 0; c < ns; ++c) {
        QFS_HIP(hipEventRecord(side_done[c], side[c]));
        QFS_HIP(hipStreamWaitEvent(st, side_done[c], 0));
      }
      QFS_HIP(hipEventRecord(e1, st));
      QFS_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      QFS_HIP(hipEventElapsedTime(&ms, e0, e1));
      kernel_seconds += 1e-3 * ms;
      if (batch_trace()) std::fprintf(stderr, "qfs batch: round of %d launches %.3f ms\n", nl, ms);
    }
    QFS_HIP(hipMemcpyAsync(jobs.data(), djobs.ptr, sizeof(BJob) * njobs_all, hipMemcpyDeviceToHost, st));
    QFS_HIP(hipMemcpyAsync(hp.data(), dprobs.ptr, sizeof(BProb) * P, hipMemcpyDeviceToHost, st));
    QFS_HIP(hipStreamSynchronize(st));
    const bool timed_out = p.time_budget_s > 0 && bnow() - t0 > p.time_budget_s;

    // ------------------------------------------------------------ per-problem decisions
    std::vector<int32_t> todo, m0s;
    bool probs_dirty = false;
    for (int i = 0; i < P; ++i) {
      if (finished[i]) continue;
      BProb &d = hp[i];
      BJob *js = jobs.data() + (size_t)i * S;
      const int ds = d.done_sweep, os = d.over_sweep;
      const int first = std::min(ds, os);
      bool behind = false, any_run = false;
      for (int s = 0; s < S; ++s) {
        if (js[s].status == BJ_RUN) {
          any_run = true;
          if (js[s].total < first) behind = true;
        }
      }
      auto finish = [&](int w, int reason_override) {
        finished[i] = 1;
        --remaining;
        winner[i] = w;
        if (reason_override >= 0) js[w].status = reason_override;
      };
      if (opts.independent) {
        // every start runs to its own stop; the problem ends when none is running
        for (int s = 0; s < S; ++s) {
          if (js[s].status == BJ_REFINE) {
            js[s].status = BJ_RUN;
            js[s].fp64 = 1;
            any_run = true;
          }
          if (timed_out && js[s].status == BJ_RUN) js[s].status = BJ_TIMEOUT;
        }
        if (timed_out) any_run = false;
        if (!any_run) {
          int w = -1;
          for (int s = 0; s < S; ++s)
            if (js[s].status == BJ_SUCCESS && (w < 0 || js[s].c_train < js[w].c_train)) w = s;
          if (w < 0)
            for (int s = 0; s < S; ++s)
              if (js[s].status != BJ_SKIP && (w < 0 || js[s].c_train < js[w].c_train)) w = s;
          finish(w, -1);
        }
        continue;
      }
      if (first < kNoSweep && behind && !timed_out) continue;
      if (ds < kNoSweep && ds <= os) {
        int w = -1;
        for (int s = 0; s < S; ++s)
          if (js[s].status == BJ_SUCCESS && js[s].total == ds && (w < 0 || js[s].c_train < js[w].c_train)) w = s;
        if (w < 0)  // the success at ds is the only reference; take the best success
          for (int s = 0; s < S; ++s)
            if (js[s].status == BJ_SUCCESS && (w < 0 || js[s].c_train < js[w].c_train)) w = s;
        finish(w, -1);
        continue;
      }
      if (os < kNoSweep && !timed_out) {
        // double-and-restart: extend the training set, keep every gate (App. A)
        const int N = 1 << d.n;
        const int m_old = d.M;
        d.M = std::min(2 * d.M, d.mcap);
        d.full = d.M == N;
        d.generation += 1;
        if (d.kind != QFS_TARGET_SAMPLES) d.Mv = p.m_val > 0 ? std::min(p.m_val, N) : d.M;
        d.over_sweep = kNoSweep;
        restarts[i] += 1;
        m_total[i] += d.M;
        todo.push_back(i);
        m0s.push_back(m_old);
        for (int s = 0; s < S; ++s)
          if (!terminal(js[s].status) && js[s].status != BJ_PARKED) {
            js[s].status = BJ_RUN;
            js[s].iter = 0;
            js[s].z = 0;
            js[s].need_c0 = 1;
          }
        probs_dirty = true;
        continue;
      }
      for (int s = 0; s < S; ++s) {
        if (js[s].status == BJ_REFINE) {
          js[s].status = BJ_RUN;
          js[s].fp64 = 1;
          any_run = true;
        } else if (js[s].status == BJ_PAUSED) {
          js[s].status = BJ_RUN;
          any_run = true;
        }
        // out of time: every start not already stopped for a reason of its own stops
        // with TIMEOUT (running, waiting for a doubling, or paused)
        if (timed_out && !terminal(js[s].status) && js[s].status != BJ_PARKED) js[s].status = BJ_TIMEOUT;
      }
      if (timed_out) any_run = false;
      if (!any_run && !timed_out) {
        // every running start stopped without success: wake the parked starts, which
        // continue from the problem's current training set
        bool woke = false;
        for (int s = 0; s < S; ++s)
          if (js[s].status == BJ_PARKED) {
            js[s].status = BJ_RUN;
            js[s].iter = 0;
            js[s].z = 0;
            js[s].need_c0 = 1;
            js[s].fp64 = p.precision == QFS_PREC_FP64 ? 1 : 0;
            woke = true;
          }
        if (woke) {
          if (opts.fallback_used) opts.fallback_used[i] = 1;
          continue;
        }
      }
      if (!any_run) {
        int w = -1;
        for (int s = 0; s < S; ++s)
          if (js[s].status != BJ_SKIP && js[s].status != BJ_PARKED &&
              (w < 0 || js[s].c_train < js[w].c_train))
            w = s;
        finish(w, -1);
      }
    }
    if (opts.park_rest) {
      // parked starts cost nothing once the device runs out of other work: when fewer
      // jobs than two per compute unit are left, wake every parked start at once (a
      // higher threshold trades the saved work for latency: at eight per compute unit
      // the learned runs of a 768-problem set did 0.98 of the plain method's work)
      size_t runnable = 0;
      for (size_t j = 0; j < njobs_all; ++j)
        runnable += !finished[jobs[j].prob] && jobs[j].status == BJ_RUN;
      if (runnable < 2 * (size_t)kCUs) {
        for (size_t j = 0; j < njobs_all; ++j) {
          BJob &J = jobs[j];
          if (finished[J.prob] || J.status != BJ_PARKED) continue;
          J.status = BJ_RUN;
          J.iter = 0;
          J.z = 0;
          J.need_c0 = 1;
          J.fp64 = p.precision == QFS_PREC_FP64 ? 1 : 0;
          if (opts.fallback_used) opts.fallback_used[J.prob] = 1;
        }
      }
    }
    if (probs_dirty) {
      QFS_HIP(hipMemcpyAsync(dprobs.ptr, hp.data(), sizeof(BProb) * P, hipMemcpyHostToDevice, st));
      QFS_HIP(hipMemcpyAsync(dtodo.ptr, todo.data(), sizeof(int32_t) * todo.size(), hipMemcpyHostToDevice, st));
      QFS_HIP(hipMemcpyAsync(dm0.ptr, m0s.data(), sizeof(int32_t) * m0s.size(), hipMemcpyHostToDevice, st));
      QFS_TRY(launch_batch_setup(dprobs.as<BProb>(), dtodo.as<int32_t>(), (int)todo.size(), dm0.as<int32_t>(), st));
    }
    QFS_HIP(hipMemcpyAsync(djobs.ptr, jobs.data(), sizeof(BJob) * njobs_all, hipMemcpyHostToDevice, st));
    QFS_HIP(hipStreamSynchronize(st));
  }

  // ---------------------------------------------------------------- results
  const double secs = bnow() - t0;
  for (int i = 0; i < P; ++i) {
    const BJob *js = jobs.data() + (size_t)i * S;
    int w = winner[i];
    for (int s = 0; w < 0 && s < S; ++s)
      if (js[s].status != BJ_SKIP) w = s;
    qfs_result &r = res[i];
    std::memset(&r, 0, sizeof(r));
    r.reason = to_reason(js[w].status);
    r.m_final = hp[i].M;
    r.sweeps = js[w].total;
    r.restarts = restarts[i];
    r.best_start = w;
    r.m_total = m_total[i];
    r.start_groups = 1;
    r.refined = (p.precision == QFS_PREC_MIXED && js[w].fp64) ? 1 : 0;
    r.c_train = js[w].c_train;
    r.c_val = js[w].c_val;
    r.seconds = secs;
    for (int s = 0; s < S; ++s) {
      r.start_sweeps += js[s].total;
      r.amp_updates += js[s].work;
    }
    if (opts.successes) {
      int c = 0;
      for (int s = 0; s < S; ++s) c += js[s].status == BJ_SUCCESS;
      opts.successes[i] = c;
    }
    r.sweep_seconds = kernel_seconds;
    if (gates_out[i])
      QFS_HIP(hipMemcpyAsync(gates_out[i], hp[i].g64 + (size_t)w * hp[i].L * 16,
                             sizeof(c128) * 16 * hp[i].L, hipMemcpyDeviceToDevice, st));
  }
  QFS_HIP(hipStreamSynchronize(st));
  return QFS_OK;
}

extern "C" int qfs_instantiate_batch(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                                     const qfs_params *params, qfs_c128 *const *gates_out,
                                     qfs_result *res) {
  return batch_instantiate(P, tmpl, targets, params, gates_out, res, BatchOpts{});
}

extern "C" int qfs_instantiate_batch_ex(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                                        const qfs_params *params, const int32_t *m_init,
                                        const int32_t *starts, qfs_c128 *const *gates_out,
                                        qfs_result *res) {
  BatchOpts o;
  o.m_init = m_init;
  o.starts = starts;
  return batch_instantiate(P, tmpl, targets, params, gates_out, res, o);
}

extern "C" int qfs_label_batch(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                               const qfs_params *params, int32_t *successes, qfs_result *res) {
  if (!params || !successes || P < 1) {
    set_error_detail("label: null argument or P < 1");
    return QFS_EINVAL;
  }
  qfs_params q = *params;
  q.fixed_m = 1;
  std::vector<qfs_c128 *> none((size_t)P, nullptr);
  BatchOpts o;
  o.independent = 1;
  o.successes = successes;
  return batch_instantiate(P, tmpl, targets, &q, none.data(), res, o);
}
