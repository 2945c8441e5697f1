// Learned initial sample count and start pruning (project extension). The paper leaves
// the choice of the initial number of training states open (Sec. 3, Sec. 5) and relates
// the number needed to the parameter count per amplitude (Sec. 4, the #U3 / 2^n study).
// Here a small network (mlp.hip) maps 64 structural features of the template to
//   y0 = log2 of the smallest power-of-two M at which a start succeeds and generalises,
//   y1 = logit of the probability that one random start succeeds at that M,
// and the instantiation runs with M0 = 2^round(y0) and the number of starts that
// minimises the expected start-runs under the predicted rate (see decide). A predicted M0
// that is too small is corrected by the method's own doubling on the held-out validation
// cost (Sec. 3); a start count that was too small is corrected by the fallback: when the
// learned run does not succeed, the pruned starts run with the plain method's control,
// from the M the learned run ended at, so no start of the plain method is lost.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "batch.h"
#include "mlp.h"

namespace qfs {
namespace {


double lnow() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool valid_template(const qfs_template *t) {
  if (!t || t->n_qubits < 2 || t->n_qubits > 30 || t->n_gates < 1 || !t->pairs) return false;
  for (int k = 0; k < t->n_gates; ++k) {
    const int a = t->pairs[2 * k], b = t->pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= t->n_qubits || b >= t->n_qubits || a == b) return false;
  }
  return true;
}

// The network was fitted on templates of two-qubit gates only.
bool two_qubit_only(const qfs_template *t) {
  if (t->kinds)
    for (int k = 0; k < t->n_gates; ++k)
      if (t->kinds[k] != QFS_GATE_2Q) return false;
  return true;
}

// Structural features, each scaled to O(1):
//   0 n/16, 1 L/128, 2 depth/64 (greedy layering), 3 log2(1 + 16L/2^n) (real parameters
//   per amplitude, the paper's explanatory variable up to the factor), 4 log2(16L)/16,
//   5 distinct pairs / L, 6 touched qubits / n, 7 max qubit degree / L, 8 std of qubit
//   degree / (L+1), 9 connected components / n, 10 depth / L, 11 log2(depth+1)/8,
//   12..27 histogram of qubit degrees (bins 0..15+, fraction of qubits),
//   28..43 histogram of |a - b| (bins 1..16+, fraction of gates),
//   44..59 histogram of gate layers over 16 equal depth bins (fraction of gates),
//   60 n/L, 61 min(1, 2^n / 16L), 62 1/n, 63 constant 1.
void template_features(const qfs_template &t, float *out) {
  const int n = t.n_qubits, L = t.n_gates;
  std::vector<int> layer(n, 0), deg(n, 0), gate_layer(L, 0);
  std::vector<char> adj((size_t)n * n, 0);
  int depth = 0, distinct = 0;
  for (int k = 0; k < L; ++k) {
    const int a = t.pairs[2 * k], b = t.pairs[2 * k + 1];
    const int l = std::max(layer[a], layer[b]) + 1;
    layer[a] = layer[b] = l;
    gate_layer[k] = l;
    depth = std::max(depth, l);
    ++deg[a];
    ++deg[b];
    if (!adj[(size_t)a * n + b]) ++distinct;
    adj[(size_t)a * n + b] = adj[(size_t)b * n + a] = 1;
  }
  std::vector<int> comp(n, -1), stack;
  int ncomp = 0;
  for (int q = 0; q < n; ++q) {
    if (comp[q] >= 0) continue;
    comp[q] = ncomp;
    stack.assign(1, q);
    while (!stack.empty()) {
      const int x = stack.back();
      stack.pop_back();
      for (int y = 0; y < n; ++y)
        if (adj[(size_t)x * n + y] && comp[y] < 0) {
          comp[y] = ncomp;
          stack.push_back(y);
        }
    }
    ++ncomp;
  }
  int touched = 0, maxdeg = 0;
  double mean = 0.0, var = 0.0;
  for (int q = 0; q < n; ++q) {
    touched += deg[q] > 0;
    maxdeg = std::max(maxdeg, deg[q]);
    mean += deg[q];
  }
  mean /= n;
  for (int q = 0; q < n; ++q) var += (deg[q] - mean) * (deg[q] - mean);
  var /= n;
  double f[kMlpF] = {0};
  const double N = std::ldexp(1.0, n);
  f[0] = n / 16.0;
  f[1] = L / 128.0;
  f[2] = depth / 64.0;
  f[3] = std::log2(1.0 + 16.0 * L / N);
  f[4] = std::log2(16.0 * L) / 16.0;
  f[5] = (double)distinct / L;
  f[6] = (double)touched / n;
  f[7] = (double)maxdeg / L;
  f[8] = std::sqrt(var) / (L + 1.0);
  f[9] = (double)ncomp / n;
  f[10] = (double)depth / L;
  f[11] = std::log2(depth + 1.0) / 8.0;
  for (int q = 0; q < n; ++q) f[12 + std::min(deg[q], 15)] += 1.0 / n;
  for (int k = 0; k < L; ++k) {
    const int d = std::abs(t.pairs[2 * k] - t.pairs[2 * k + 1]);
    f[28 + std::min(d, 16) - 1] += 1.0 / L;
  }
  for (int k = 0; k < L; ++k) f[44 + std::min(15, (int)((gate_layer[k] - 1) * 16.0 / depth))] += 1.0 / L;
  f[60] = (double)n / L;
  f[61] = std::min(1.0, N / (16.0 * L));
  f[62] = 1.0 / n;
  f[63] = 1.0;
  for (int i = 0; i < kMlpF; ++i) out[i] = (float)f[i];
}

// Network outputs -> (M0, kept starts). With a predicted per-start success rate p, k
// kept starts cost k start-runs and, with probability (1 - p)^k that none succeeds, the
// S - k pruned ones run afterwards; k minimises k + (1 - p)^k (S - k) (the batched run,
// where the device is kept full and time follows work).
void decide(const float *y, int n, int S, int32_t *m0, int32_t *starts, double *prob = nullptr) {
  const double lg = std::min<double>(n, std::max(1.0, std::nearbyint((double)y[0])));
  *m0 = (int32_t)std::ldexp(1.0, (int)lg);
  const double p = std::min(1.0, std::max(0.0, 1.0 / (1.0 + std::exp(-(double)y[1]))));
  if (prob) *prob = p;
  int best = S;
  double best_cost = (double)S;
  for (int k = 1; k < S; ++k) {
    const double cost = k + std::pow(1.0 - p, k) * (S - k);
    if (cost < best_cost) {
      best_cost = cost;
      best = k;
    }
  }
  *starts = best;
}

// One problem at a time the starts run together, so the time of a sweep is not
// proportional to the starts: about T0 + k b / BW for k starts of b bytes each (T0 the
// serial chain of the sweep, about 17.5 us per gate on the MI355X, BW about 3.7 TB/s of
// algorithmic bytes, b = (2 L + 1) M 2^n 8 bytes), i.e. proportional to
// 1 + k / k_sat with k_sat = T0 BW / b. The kept starts k then minimise the expected
// time (1 + k / k_sat) + (1 - p)^k (1 + (S - k) / k_sat) against 1 + S / k_sat for
// all S, and starts are pruned only when that saves at least a tenth of the time: small
// problems (k_sat >> S) keep every start, since pruning them saves no measurable time and
// risks the fallback's second run.
int decide_single(double p, int n, int L, int m0, int S) {
  const double b = (2.0 * L + 1.0) * (double)m0 * std::ldexp(1.0, n) * 8.0;
  const double k_sat = (17.5e-6 * L) * 3.7e12 / b;
  const double all = 1.0 + S / k_sat;
  int best = S;
  double best_cost = all;
  for (int k = 1; k < S; ++k) {
    const double cost = 1.0 + k / k_sat + std::pow(1.0 - p, k) * (1.0 + (S - k) / k_sat);
    if (cost < best_cost) {
      best_cost = cost;
      best = k;
    }
  }
  return best_cost < 0.9 * all ? best : S;
}

int predict_many(int P, const qfs_template *tmpl, const qfs_params &p, int32_t *m0, int32_t *starts,
                 hipStream_t s, double *prob = nullptr) {
  std::vector<float> feat((size_t)P * kMlpF), y((size_t)P * kMlpO);
  for (int i = 0; i < P; ++i) {
    if (!valid_template(&tmpl[i])) return set_error_detail("learned: invalid template"), QFS_EINVAL;
    if (!two_qubit_only(&tmpl[i]))
      return set_error_detail("learned: templates of two-qubit gates only"), QFS_EUNSUPPORTED;
    template_features(tmpl[i], feat.data() + (size_t)i * kMlpF);
  }
  DevBuf fd, yd;
  QFS_TRY(fd.alloc(sizeof(float) * feat.size()));
  QFS_TRY(yd.alloc(sizeof(float) * y.size()));
  QFS_HIP(hipMemcpyAsync(fd.ptr, feat.data(), sizeof(float) * feat.size(), hipMemcpyHostToDevice, s));
  QFS_TRY(mlp_predict(P, fd.as<float>(), yd.as<float>(), s));
  QFS_HIP(hipMemcpyAsync(y.data(), yd.ptr, sizeof(float) * y.size(), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  const int S = std::max(1, p.multistarts);
  for (int i = 0; i < P; ++i)
    decide(y.data() + (size_t)i * kMlpO, tmpl[i].n_qubits, S, m0 + i, starts + i, prob ? prob + i : nullptr);
  return QFS_OK;
}

}  // namespace
}  // namespace qfs

using namespace qfs;

extern "C" {

int qfs_features(const qfs_template *t, float *out) {
  if (!valid_template(t) || !out) return set_error_detail("features: invalid template"), QFS_EINVAL;
  if (!two_qubit_only(t)) return set_error_detail("features: templates of two-qubit gates only"), QFS_EUNSUPPORTED;
  template_features(*t, out);
  return QFS_OK;
}

int qfs_predict_m(const qfs_template *t, const qfs_params *params, int32_t *m0, uint32_t *keep_mask) {
  if (!t || !params || !m0) return QFS_EINVAL;
  int32_t k = 0;
  QFS_TRY(predict_many(1, t, *params, m0, &k, static_cast<hipStream_t>(params->hip_stream)));
  if (keep_mask) *keep_mask = k >= 32 ? 0xffffffffu : ((1u << k) - 1u);
  return QFS_OK;
}

int qfs_predict_batch(int32_t P, const qfs_template *tmpl, const qfs_params *params, int32_t *m0,
                      int32_t *starts) {
  if (P < 1 || !tmpl || !params || !m0 || !starts) return QFS_EINVAL;
  return predict_many(P, tmpl, *params, m0, starts, static_cast<hipStream_t>(params->hip_stream));
}

int qfs_instantiate_learned(const qfs_template *tmpl, const qfs_target *target, const qfs_params *params,
                            qfs_c128 *gates_out, qfs_result *res) {
  if (!tmpl || !target || !params || !res) return QFS_EINVAL;
  const double t0 = lnow();
  hipStream_t st = static_cast<hipStream_t>(params->hip_stream);
  int32_t m0 = 0, k = 0;
  double prob = 0.0;
  QFS_TRY(predict_many(1, tmpl, *params, &m0, &k, st, &prob));
  const int S = params->multistarts;
  k = decide_single(prob, tmpl->n_qubits, tmpl->n_gates, std::max(params->m_init, m0), S);
  qfs_params q = *params;
  q.m_init = std::max(params->m_init, m0);
  q.multistarts = k;
  qfs_result r1;
  QFS_TRY(qfs_instantiate(tmpl, target, &q, nullptr, gates_out, &r1));
  r1.m_predicted = m0;
  r1.starts_run = k;
  r1.fallback = 0;
  if (r1.reason == QFS_SUCCESS || k >= S) {
    *res = r1;
    res->seconds = lnow() - t0;
    return QFS_OK;
  }
  // fallback: the pruned starts k..S-1 (their own initial gates), plain doubling from m_init
  const int L = tmpl->n_gates;
  DevBuf all, best;
  QFS_TRY(all.alloc(sizeof(c128) * 16 * (size_t)S * L));
  QFS_TRY(best.alloc(sizeof(c128) * 16 * (size_t)L));
  QFS_TRY(qfs_haar_gates(params->seed, S, L, all.as<qfs_c128>(), st));
  if (gates_out)
    QFS_HIP(hipMemcpyAsync(best.ptr, gates_out, sizeof(c128) * 16 * L, hipMemcpyDeviceToDevice, st));
  qfs_params q2 = *params;
  q2.multistarts = S - k;
  q2.m_init = std::max(params->m_init, r1.m_final);
  qfs_result r2;
  QFS_TRY(qfs_instantiate(tmpl, target, &q2, all.as<qfs_c128>() + (size_t)k * L * 16, gates_out, &r2));
  const bool take2 = r2.reason == QFS_SUCCESS || r2.c_train < r1.c_train;
  if (!take2 && gates_out)
    QFS_HIP(hipMemcpyAsync(gates_out, best.ptr, sizeof(c128) * 16 * L, hipMemcpyDeviceToDevice, st));
  QFS_HIP(hipStreamSynchronize(st));
  *res = take2 ? r2 : r1;
  if (take2) res->best_start += k;
  res->m_predicted = m0;
  res->starts_run = S;
  res->fallback = 1;
  res->start_sweeps = r1.start_sweeps + r2.start_sweeps;
  res->amp_updates = r1.amp_updates + r2.amp_updates;
  res->sweep_seconds = r1.sweep_seconds + r2.sweep_seconds;
  res->m_total = r1.m_total + r2.m_total;
  res->seconds = lnow() - t0;
  return QFS_OK;
}

int qfs_instantiate_batch_learned(int32_t P, const qfs_template *tmpl, const qfs_target *targets,
                                  const qfs_params *params, qfs_c128 *const *gates_out, qfs_result *res) {
  if (P < 1 || !tmpl || !targets || !params || !gates_out || !res) return QFS_EINVAL;
  const double t0 = lnow();
  hipStream_t st = static_cast<hipStream_t>(params->hip_stream);
  const int S = params->multistarts;
  std::vector<int32_t> m0(P), k(P), fb(P, 0);
  QFS_TRY(predict_many(P, tmpl, *params, m0.data(), k.data(), st));
  std::vector<int32_t> m_run(P);
  for (int i = 0; i < P; ++i) m_run[i] = std::max(params->m_init, m0[i]);
  // one batched run: the kept starts first; a problem's pruned starts are parked and
  // woken inside the same run when all its kept starts stop without success
  BatchOpts o;
  o.m_init = m_run.data();
  o.starts = k.data();
  o.park_rest = 1;
  o.fallback_used = fb.data();
  QFS_TRY(batch_instantiate(P, tmpl, targets, params, gates_out, res, o));
  const double secs = lnow() - t0;
  for (int i = 0; i < P; ++i) {
    res[i].m_predicted = m0[i];
    res[i].starts_run = fb[i] ? S : k[i];
    res[i].fallback = fb[i];
    res[i].seconds = secs;
  }
  return QFS_OK;
}

}  // extern "C"
