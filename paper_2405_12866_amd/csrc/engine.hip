// Host runtime and C ABI of the HIP implementation: the instantiation control loop
// (Sec. 3 on-the-fly generalisation check and double-and-restart, Eq. 12 success
// relations; App. A plateau test, min_iter/max_iter, multistarts and the recursive
// half-multistart retry on device out-of-memory), device memory management and the
// per-step entry points declared in include/qfs.h.
#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>
#include <type_traits>

#include "qfs_internal.h"

namespace qfs {

static thread_local std::string g_detail;
void set_error_detail(const std::string &s) { g_detail = s; }

int pool_stream(int index, hipStream_t *out) {
  constexpr int kPool = 16, kDevices = 64;
  static std::mutex mu;
  static hipStream_t pool[kDevices][kPool] = {};
  if (index < 0 || index >= kPool) return QFS_EINVAL;
  int dev = 0;
  QFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kDevices) return QFS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(mu);
  if (!pool[dev][index]) QFS_HIP(hipStreamCreateWithFlags(&pool[dev][index], hipStreamNonBlocking));
  *out = pool[dev][index];
  return QFS_OK;
}

int ensure_dynamic_lds(const void *fn, size_t bytes, size_t *have) {
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (bytes > 64 * 1024 && bytes > *have) {
    QFS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    *have = bytes;
  }
  return QFS_OK;
}

// Device blocks kept between calls of the engine, by device and exact size. hipMalloc of
// the large working sets and hipFree (which drains the device) otherwise cost several
// hundred microseconds each in every call, during which the device idles. The cache holds
// at most an eighth of the device's memory; blocks beyond that are freed.
namespace {
struct BlockCache {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void *> blocks;
  std::map<int, size_t> held;
};
BlockCache &block_cache() {
  static BlockCache *c = new BlockCache;  // never destroyed: no HIP calls at process exit
  return *c;
}
bool cache_poison() {
  // debugging aid: cached blocks are filled with 0xff bytes (NaN for every float type), so
  // that code reading a block before writing it shows up
  static const bool on = [] {
    const char *e = std::getenv("QFS_CACHE_POISON");
    return e && std::atoi(e) != 0;
  }();
  return on;
}
}  // namespace

void *device_cache_take(int dev, size_t bytes) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.blocks.find({dev, bytes});
  if (it == c.blocks.end()) return nullptr;
  void *p = it->second;
  c.blocks.erase(it);
  c.held[dev] -= bytes;
  return p;
}

size_t device_cache_held(int dev) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.held.find(dev);
  return it == c.held.end() ? 0 : it->second;
}

size_t device_cache_trim(int dev) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  size_t freed = 0;
  for (auto it = c.blocks.lower_bound({dev, 0}); it != c.blocks.end() && it->first.first == dev;) {
    (void)hipFree(it->second);
    freed += it->first.second;
    it = c.blocks.erase(it);
  }
  c.held[dev] -= freed;
  return freed;
}

// Pinned host buffers for the per-sweep costs, kept for later calls (hipHostMalloc and
// hipHostFree cost tens to hundreds of microseconds each). Never freed: the pool holds at
// most one buffer per call that ran at the same time.
namespace {
std::mutex g_pin_mu;
std::multimap<size_t, void *> g_pins;
}  // namespace

static void *pinned_take(size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pins.lower_bound(bytes);
    if (it != g_pins.end()) {
      void *p = it->second;
      g_pins.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  if (hipHostMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

// (only once no copy into the buffer is pending)
static void pinned_put(void *p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pins.emplace(bytes, p);
}

// Takes idle blocks (the device has drained since their last use) of device dev.
static void device_cache_put(int dev, std::vector<std::pair<void *, size_t>> &blks) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    tot = 0;
  }
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto &b : blks) {
    if (c.held[dev] + b.second > tot / 8) {
      (void)hipFree(b.first);
      continue;
    }
    if (cache_poison() && hipMemset(b.first, 0xff, b.second) != hipSuccess) (void)hipGetLastError();
    c.blocks.emplace(std::make_pair(dev, b.second), b.first);
    c.held[dev] += b.second;
  }
  blks.clear();
}

namespace {

enum { kClsStep = 0, kClsForward = 1, kClsDist = 2, kClsPolar = 3, kClasses = 4 };

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

hipStream_t as_stream(void *p) { return static_cast<hipStream_t>(p); }

int ceil_log2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// Row-major N x ld masters (states as columns) use ld = 2^ceil(log2 max(M, 2)), so
// that the same buffer is also a one-chunk set of the chunked layout.
int master_ld(int M) { return 1 << std::max(1, ceil_log2(std::max(M, 2))); }

size_t lds_max_bytes() {
  static const size_t cached = [] {  // (initialised once, thread-safe)
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      return (size_t)v;
    return (size_t)64 * 1024;
  }();
  return cached;
}

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
    if (t->kinds) {
      const int kind = t->kinds[k];
      if (kind != QFS_GATE_2Q && kind != QFS_GATE_1Q && kind != QFS_GATE_FIXED) {
        set_error_detail("template: gate " + std::to_string(k) + " has an unknown kind");
        return QFS_EINVAL;
      }
      if (kind == QFS_GATE_FIXED && !t->fixed_gates) {
        set_error_detail("template: constant gates need fixed_gates");
        return QFS_EINVAL;
      }
    }
  }
  return QFS_OK;
}

bool has_kinds(const qfs_template *t) {
  if (!t->kinds) return false;
  for (int k = 0; k < t->n_gates; ++k)
    if (t->kinds[k] != QFS_GATE_2Q) return true;
  return false;
}

// Memory accounting for one call: every allocation goes through here so that the
// budget (device_mem_budget or the free memory) is enforced before hipMalloc. Blocks come
// from the cache of earlier calls when one of the exact size is there. A block the call
// gives back (a buffer freed or resized, or the call's end) is kept, not freed and not
// reused within the call; when the call ends, the device is drained once and its blocks go
// to the cache. On a device out-of-memory the kept blocks and the cache are freed and the
// allocation is tried once more.
struct Arena {
  size_t budget = 0, used = 0;
  int dev = 0;
  std::vector<std::pair<void *, size_t>> kept;
  Arena() {
    if (hipGetDevice(&dev) != hipSuccess) (void)hipGetLastError();
  }
  Arena(const Arena &) = delete;
  Arena &operator=(const Arena &) = delete;
  ~Arena() {
    if (kept.empty()) return;
    if (hipDeviceSynchronize() == hipSuccess) {
      device_cache_put(dev, kept);
    } else {
      (void)hipGetLastError();
      for (auto &b : kept) (void)hipFree(b.first);
      kept.clear();
    }
  }
  static void give_back(void *self, void *p, size_t bytes) {
    static_cast<Arena *>(self)->kept.emplace_back(p, bytes);
  }
  int alloc(DevBuf &b, size_t bytes) {
    const size_t old = b.bytes;
    if (used - old + bytes > budget) {
      set_error_detail("device memory budget exceeded: need " + std::to_string(used - old + bytes) +
                       " of " + std::to_string(budget) + " bytes");
      return QFS_ENOMEM;
    }
    used -= old;
    b.release();
    if (bytes == 0) return QFS_OK;
    void *p = device_cache_take(dev, bytes);
    if (!p) {
      hipError_t e = hipMalloc(&p, bytes);
      if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        // the blocks this call gave back are idle once the device has drained
        QFS_HIP(hipDeviceSynchronize());
        for (auto &k : kept) (void)hipFree(k.first);
        kept.clear();
        (void)device_cache_trim(dev);
        e = hipMalloc(&p, bytes);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error_detail(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? QFS_ENOMEM : QFS_EDEVICE;
      }
    }
    b.ptr = p;
    b.bytes = bytes;
    b.give_back = &Arena::give_back;
    b.owner = this;
    used += bytes;
    return QFS_OK;
  }
  void free(DevBuf &b) {
    used -= b.bytes;
    b.release();
  }
};

struct Counters {
  int64_t kl[kClasses] = {0, 0, 0, 0};
  double ks[kClasses] = {0, 0, 0, 0}, kb[kClasses] = {0, 0, 0, 0};
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
    QFS_TRY(reserve());
    QFS_HIP(hipEventRecord(ev_[2 * used_], s));
    return QFS_OK;
  }
  int end(hipStream_t s, int cls, double bytes) {
    if (!on) return QFS_OK;
    QFS_HIP(hipEventRecord(ev_[2 * used_ + 1], s));
    return count(cls, bytes);
  }
  // The next pair of events for a launch that records them itself (LaunchEvents, null
  // when timing is off); ext_end books it like end().
  int ext_begin(LaunchEvents *le) {
    *le = LaunchEvents{};
    if (!on) return QFS_OK;
    QFS_TRY(reserve());
    le->start = ev_[2 * used_];
    le->stop = ev_[2 * used_ + 1];
    return QFS_OK;
  }
  int ext_end(int cls, double bytes) { return on ? count(cls, bytes) : QFS_OK; }
  // Call only after the stream has been synchronised.
  int flush(Counters &r) {
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
  int reserve() {
    if (ev_.size() < 2 * (used_ + 1)) {
      hipEvent_t a, b;
      QFS_HIP(hipEventCreate(&a));
      QFS_HIP(hipEventCreate(&b));
      ev_.push_back(a);
      ev_.push_back(b);
    }
    return QFS_OK;
  }
  int count(int cls, double bytes) {
    if (cls_.size() <= used_) {
      cls_.resize(used_ + 1);
      bytes_.resize(used_ + 1);
    }
    cls_[used_] = cls;
    bytes_[used_] = bytes;
    ++used_;
    return QFS_OK;
  }
  std::vector<hipEvent_t> ev_;
  std::vector<int> cls_;
  std::vector<double> bytes_;
  size_t used_ = 0;
};

// ------------------------------------------------------------------ one sweep
// Everything one forward pass or one right-to-left update needs, for a set of starts
// sharing a training set. Used by the control loop and by qfs_sweep.
struct SweepCtx {
  int n = 0, L = 0;
  const int32_t *pairs_host = nullptr;
  const int32_t *pairs_dev = nullptr;
  const int32_t *kinds = nullptr;  // host [L] gate kinds, or nullptr: all two-qubit
  const int32_t *kinds_dev = nullptr;  // the same on the device
  Geometry g{}, gv{};  // training / validation sets (gv.M == 0: no validation)
  bool fused = false;
  const int32_t *slots = nullptr;
  int nslots = 0;
  c128 *g64 = nullptr;
  c64 *g32 = nullptr;
  c128 *vstore = nullptr;  // [S][L][16] Jacobi warm start (nullable)
  double beta = 0.0;
  void *psi = nullptr, *phi = nullptr, *psiv = nullptr, *phiv = nullptr;  // working sets
  void *blist = nullptr, *astate = nullptr, *vstate = nullptr;
  c128 *partials = nullptr;  // [S][kPcap][16]
  double *dpart0 = nullptr, *dpart1 = nullptr;  // [S][kPcap] each
  double *costs = nullptr;   // [3 S]: c_train, c_val, c_0
  int S = 0;
  KernelTimer *timer = nullptr;
  hipStream_t stream = nullptr;
  // Second stream and join events: without kernel timing, the backward pass runs the
  // two halves of the starts on two streams, so one half's environment reduction and
  // polar update overlap the other half's backward step.
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // Grouped backward pass (group.hip): groups from the last gate down, the device mask
  // of the B list entries they read, and the second-moment partials [S][kGPcap][256].
  bool grouped = false;
  const std::vector<GateGroup> *groups = nullptr;
  const int32_t *bneed_dev = nullptr;
  c128 *gpartials = nullptr;
  int gpstride = 0;
  c128 *vop = nullptr;  // [S][256]: the last finalized group's operator
  // forward pass by groups (complex64, fused): device plan, per-gate slots, group count
  const int32_t *fplan = nullptr, *fgslot = nullptr;
  int fngroups = 0;
  bool fforms = false;  // the forward plan holds one-qubit or CNOT gate forms
  // Grouped sweeps run the starts in up to nparts parts (2 by default: on MI355X more
  // parts measured no faster, their kernels slowing each other down), part p on
  // pstream[p] (pstream[0] is the call's stream), each part's forward pass right after its
  // own backward pass.
  static constexpr int kParts = 4;
  int nparts = 1;
  hipStream_t pstream[kParts] = {};
  hipEvent_t pfork = nullptr, pjoin[kParts] = {};
};

template <typename R>
GateRef gate_ref(const SweepCtx &c) {
  const bool f32 = sizeof(R) == 4;
  return GateRef{c.g64, f32 ? static_cast<const void *>(c.g32) : static_cast<const void *>(c.g64),
                 c.L * 16};
}

template <typename R>
double set_bytes(const SweepCtx &c, const Geometry &g) {
  return (double)g.elems() * sizeof(cx<R>) * (double)c.nslots;
}

// Forward pass (Fig. pre-comp): B_k = u_{k-1} B_{k-1}, k = 1 .. L-1, from the gates as
// they are before the sweep; the validation states go through every gate and their
// Eq. 9 cost against U psi_val is c_val of the current gates. with_c0 also takes the
// training cost of the current gates (needed once per training set).
template <typename R>
int sweep_forward(SweepCtx &c, bool with_c0) {
  const GateRef gr = gate_ref<R>(c);
  cx<R> *psi = static_cast<cx<R> *>(c.psi), *phi = static_cast<cx<R> *>(c.phi);
  cx<R> *psiv = static_cast<cx<R> *>(c.psiv), *phiv = static_cast<cx<R> *>(c.phiv);
  cx<R> *B = static_cast<cx<R> *>(c.blist);
  const int64_t sN = c.g.elems();
  const int64_t bstride = sN * std::max(c.L - 1, 1);
  const bool val = c.gv.M > 0;
  KernelTimer &T = *c.timer;
  if (c.fused) {
    QFS_TRY(T.begin(c.stream));
    if constexpr (std::is_same<R, float>::value) {
      if (c.grouped && c.fplan) {
        QFS_TRY(launch_forward_groups<float>(c.g, val ? &c.gv : nullptr, c.L, gr, psi, B, bstride,
                                             with_c0 ? phi : nullptr, c.dpart0, psiv, phiv, c.dpart1, c.slots,
                                             c.nslots, c.fplan, c.fngroups, c.fgslot, c.fforms, c.stream));
      } else {
        QFS_TRY(launch_forward_fused<R>(c.g, val ? &c.gv : nullptr, c.pairs_dev, c.L, gr, psi, B, bstride,
                                        with_c0 ? phi : nullptr, c.dpart0, psiv, phiv, c.dpart1, c.slots,
                                        c.nslots, c.kinds_dev, c.stream, c.grouped ? c.bneed_dev : nullptr));
      }
    } else {
      QFS_TRY(launch_forward_fused<R>(c.g, val ? &c.gv : nullptr, c.pairs_dev, c.L, gr, psi, B, bstride,
                                      with_c0 ? phi : nullptr, c.dpart0, psiv, phiv, c.dpart1, c.slots,
                                      c.nslots, c.kinds_dev, c.stream, c.grouped ? c.bneed_dev : nullptr));
    }
    // load Psi, store the B list entries the backward pass reads, read U Psi for c_0
    int stored = 0;
    if (c.grouped) {
      for (const GateGroup &gg : *c.groups) stored += gg.k_lo >= 1 && gg.nvar > 0;
    } else {
      stored = c.L - 1;
      for (int k = 1; c.kinds && k < c.L; ++k) stored -= c.kinds[k] == QFS_GATE_FIXED;
    }
    const double bytes = set_bytes<R>(c, c.g) * (1 + stored + (with_c0 ? 1 : 0)) +
                         (val ? 2.0 * set_bytes<R>(c, c.gv) : 0.0);
    QFS_TRY(T.end(c.stream, kClsForward, bytes));
    if (val) QFS_TRY(launch_dist_finalize(c.gv.nch, c.dpart1, c.slots, c.nslots, c.gv.M, c.costs + c.S, c.stream));
    if (with_c0)
      QFS_TRY(launch_dist_finalize(c.g.nch, c.dpart0, c.slots, c.nslots, c.g.M, c.costs + 2 * c.S, c.stream));
    return QFS_OK;
  }
  cx<R> *Vs = static_cast<cx<R> *>(c.vstate);
  const int64_t vstride = c.gv.elems();
  for (int k = 1; k < c.L; ++k) {
    const int qa = c.pairs_host[2 * (k - 1)], qb = c.pairs_host[2 * (k - 1) + 1];
    SBuf<R> src = k == 1 ? SBuf<R>{psi, 0} : SBuf<R>{B + (k - 2) * sN, bstride};
    QFS_TRY(T.begin(c.stream));
    QFS_TRY(launch_apply<R>(c.g, qa, qb, k - 1, false, gr, src, SBuf<R>{B + (k - 1) * sN, bstride},
                            c.slots, c.nslots, c.stream));
    QFS_TRY(T.end(c.stream, kClsForward, 2.0 * set_bytes<R>(c, c.g)));
    if (val) {
      QFS_TRY(T.begin(c.stream));
      QFS_TRY(launch_apply<R>(c.gv, qa, qb, k - 1, false, gr,
                              k == 1 ? SBuf<R>{psiv, 0} : SBuf<R>{Vs, vstride}, SBuf<R>{Vs, vstride},
                              c.slots, c.nslots, c.stream));
      QFS_TRY(T.end(c.stream, kClsForward, 2.0 * set_bytes<R>(c, c.gv)));
    }
  }
  const int qa = c.pairs_host[2 * (c.L - 1)], qb = c.pairs_host[2 * (c.L - 1) + 1];
  int P = 0;
  if (val) {
    QFS_TRY(T.begin(c.stream));
    QFS_TRY(launch_apply_dist<R>(c.gv, qa, qb, c.L - 1, false, gr,
                                 c.L == 1 ? SBuf<R>{psiv, 0} : SBuf<R>{Vs, vstride}, SBuf<R>{phiv, 0},
                                 c.slots, c.nslots, c.dpart1, &P, c.stream));
    QFS_TRY(T.end(c.stream, kClsDist, 2.0 * set_bytes<R>(c, c.gv)));
    QFS_TRY(launch_dist_finalize(P, c.dpart1, c.slots, c.nslots, c.gv.M, c.costs + c.S, c.stream));
  }
  if (with_c0) {
    QFS_TRY(T.begin(c.stream));
    QFS_TRY(launch_apply_dist<R>(c.g, qa, qb, c.L - 1, false, gr,
                                 c.L == 1 ? SBuf<R>{psi, 0} : SBuf<R>{B + (c.L - 2) * sN, bstride},
                                 SBuf<R>{phi, 0}, c.slots, c.nslots, c.dpart0, &P, c.stream));
    QFS_TRY(T.end(c.stream, kClsDist, 2.0 * set_bytes<R>(c, c.g)));
    QFS_TRY(launch_dist_finalize(P, c.dpart0, c.slots, c.nslots, c.g.M, c.costs + 2 * c.S, c.stream));
  }
  return QFS_OK;
}

// Right-to-left update with gate groups (Sec. 3; Fig. env_calc_tensor), issued group by
// group for the starts slots[0 .. n) on stream st. Item gi < ng: one pass moves the backward
// state through the previous group's just-updated gates and reduces group gi's
// second-moment matrix against the B entry before the group, then the finalize updates the
// group's gates in order. Item ng: the Eq. 9 cost of the updated gates from
// a_0 = C^dagger U psi (the last group's operator applied on the way). Item ng + 1: the
// forward pass of the updated gates and their validation cost.
template <typename R>
int grouped_item(SweepCtx &c, const int32_t *slots, int n, hipStream_t st, int item) {
  cx<R> *psi = static_cast<cx<R> *>(c.psi), *phi = static_cast<cx<R> *>(c.phi);
  cx<R> *B = static_cast<cx<R> *>(c.blist), *A = static_cast<cx<R> *>(c.astate);
  const int64_t sN = c.g.elems();
  const int64_t bstride = sN * std::max(c.L - 1, 1);
  KernelTimer &T = *c.timer;
  const std::vector<GateGroup> &G = *c.groups;
  const int ng = (int)G.size();
  const double set = set_bytes<R>(c, c.g) * n / c.nslots;
  LaunchEvents le;
  if (item < ng) {
    const GateGroup &cur = G[item];
    const GateGroup *prev = item ? &G[item - 1] : nullptr;
    int P = 0;
    if (prev || cur.nvar > 0) {
      // the state entering group item: U psi through groups 0 .. item-1 (written from 1 on)
      const SBuf<R> a_in = item <= 1 ? SBuf<R>{phi, 0} : SBuf<R>{A, sN};
      const SBuf<R> a_out = prev ? SBuf<R>{A, sN} : SBuf<R>{nullptr, 0};
      const SBuf<R> b = cur.k_lo == 0 ? SBuf<R>{psi, 0} : SBuf<R>{B + (cur.k_lo - 1) * sN, bstride};
      QFS_TRY(T.ext_begin(&le));
      QFS_TRY(launch_group_pass<R>(c.g, c.pairs_host, prev, &cur, false, c.vop, a_in, a_out, b, slots, n,
                                   group_blocks_per_start(c.nslots), c.gpartials, c.gpstride, nullptr, &P,
                                   st, le));
      QFS_TRY(T.ext_end(kClsStep, set * ((prev ? 2.0 : 1.0) + (cur.nvar > 0 ? 1.0 : 0.0))));
    }
    // (a group with nothing to reduce still forms its operator for the next pass)
    QFS_TRY(T.ext_begin(&le));
    QFS_TRY(launch_group_finalize(cur.nvar > 0 ? P : 0, c.gpartials, c.gpstride, slots, n, cur, c.pairs_host,
                                  c.kinds, c.beta, c.g64, sizeof(R) == 4 ? c.g32 : nullptr, c.L * 16,
                                  c.vstore, c.vop, st, le));
    QFS_TRY(T.ext_end(kClsPolar, (double)P * 4096.0 * n));
    return QFS_OK;
  }
  if (item == ng) {
    int P = 0;
    QFS_TRY(T.ext_begin(&le));
    QFS_TRY(launch_group_pass<R>(c.g, c.pairs_host, &G.back(), nullptr, true, c.vop,
                                 ng <= 1 ? SBuf<R>{phi, 0} : SBuf<R>{A, sN}, SBuf<R>{nullptr, 0},
                                 SBuf<R>{psi, 0}, slots, n, group_blocks_per_start(c.nslots), nullptr, kGPcap,
                                 c.dpart0, &P, st, le));
    QFS_TRY(T.ext_end(kClsDist, 2.0 * set));
    return launch_dist_finalize(P, c.dpart0, slots, n, c.g.M, c.costs, st, kGPcap);
  }
  SweepCtx sub = c;
  sub.slots = slots;
  sub.nslots = n;
  sub.stream = st;
  return sweep_forward<R>(sub, false);
}

// The parts a grouped sweep of the running starts runs in: without timing, and while every
// part still streams at least 2^20 amplitudes per pass, up to nparts consecutive ranges of
// the slot list, part p on pstream[p] (part 0 on the call's stream). off[p] is the part's
// first slot; returns the number of parts.
int sweep_parts(const SweepCtx &c, int off[], int pn[], hipStream_t pst[]) {
  int parts = c.timer->on ? 1 : std::min(c.nparts, c.nslots);
  while (parts > 1 && (int64_t)(c.nslots / parts) * c.g.elems() < (int64_t(1) << 20)) --parts;
  parts = std::max(parts, 1);
  const int base = c.nslots / parts, extra = c.nslots % parts;
  for (int p = 0, o = 0; p < parts; ++p) {
    pn[p] = base + (p < extra ? 1 : 0);
    off[p] = o;
    o += pn[p];
    pst[p] = p == 0 ? c.stream : c.pstream[p];
  }
  return parts;
}

// One grouped sweep of the running starts: backward pass and cost, then (with_forward)
// the forward pass of the updated gates, which also gives their validation cost, in the
// parts of sweep_parts. The host issues the parts' items round robin, part p `lag` items
// behind part p - 1, so the parts' chains of dependent launches advance together and the
// arithmetic-bound forward pass of one part runs beside the bandwidth-bound passes of the
// others. The part streams are forked from and joined to the call's stream around the
// sweep, unless `ordered` says the caller already ordered them (the control loop keeps
// them running from one sweep into the next).
template <typename R>
int sweep_grouped(SweepCtx &c, bool with_forward, bool ordered = false) {
  const int ng = (int)c.groups->size();
  const int items = ng + 1 + (with_forward ? 1 : 0);
  int off[SweepCtx::kParts], pn[SweepCtx::kParts];
  hipStream_t pst[SweepCtx::kParts];
  const int parts = sweep_parts(c, off, pn, pst);
  if (parts <= 1) {
    for (int i = 0; i < items; ++i) QFS_TRY(grouped_item<R>(c, c.slots, c.nslots, c.stream, i));
    return QFS_OK;
  }
  static const int lag_env = [] {
    const char *e = std::getenv("QFS_PART_LAG");  // tuning aid: items between part starts
    return e ? std::atoi(e) : -1;
  }();
  const int lag = lag_env >= 0 ? std::min(lag_env, items) : std::max(1, ng / (2 * parts));
  if (!ordered) {
    QFS_HIP(hipEventRecord(c.pfork, c.stream));
    for (int p = 1; p < parts; ++p) QFS_HIP(hipStreamWaitEvent(pst[p], c.pfork, 0));
  }
  for (int t = 0; t < items + lag * (parts - 1); ++t)
    for (int p = 0; p < parts; ++p) {
      const int i = t - p * lag;
      if (i >= 0 && i < items) QFS_TRY(grouped_item<R>(c, c.slots + off[p], pn[p], pst[p], i));
    }
  if (!ordered)
    for (int p = 1; p < parts; ++p) {
      QFS_HIP(hipEventRecord(c.pjoin[p], pst[p]));
      QFS_HIP(hipStreamWaitEvent(c.stream, c.pjoin[p], 0));
    }
  return QFS_OK;
}

// Right-to-left update (Sec. 3; Fig. env_calc_tensor): for k = L-1 .. 0 the backward
// state is moved through the just-updated gate k+1, the environment of gate k is
// reduced against B_k, and gate k is replaced by its polar factor. Then the Eq. 9
// cost of the updated gates from a_0 = C^dagger U psi.
template <typename R>
int sweep_backward(SweepCtx &c) {
  if (c.grouped) return sweep_grouped<R>(c, false);
  const GateRef gr = gate_ref<R>(c);
  cx<R> *psi = static_cast<cx<R> *>(c.psi), *phi = static_cast<cx<R> *>(c.phi);
  cx<R> *B = static_cast<cx<R> *>(c.blist), *A = static_cast<cx<R> *>(c.astate);
  const int64_t sN = c.g.elems();
  const int64_t bstride = sN * std::max(c.L - 1, 1);
  KernelTimer &T = *c.timer;
  // halves of the active starts, each on its own stream (one half when timing or when
  // a single start runs)
  // (only worth it when each half still streams at least 2^20 amplitudes per step;
  // small problems are launch-bound and would pay twice the launches)
  const bool split = !T.on && c.side && c.nslots >= 2 &&
                     (int64_t)(c.nslots / 2) * c.g.elems() >= (int64_t(1) << 20);
  const int halves = split ? 2 : 1;
  const int h0 = split ? c.nslots / 2 : c.nslots;
  const int32_t *hslots[2] = {c.slots, c.slots + h0};
  const int hn[2] = {h0, c.nslots - h0};
  hipStream_t hs[2] = {c.stream, c.side};
  if (split) {
    QFS_HIP(hipEventRecord(c.fork, c.stream));
    QFS_HIP(hipStreamWaitEvent(c.side, c.fork, 0));
  }
  auto kind_of = [&](int k) { return c.kinds ? c.kinds[k] : QFS_GATE_2Q; };
  auto same_qubits = [&](int i, int j) {
    const int32_t *p = c.pairs_host;
    return (p[2 * i] == p[2 * j] && p[2 * i + 1] == p[2 * j + 1]) ||
           (p[2 * i] == p[2 * j + 1] && p[2 * i + 1] == p[2 * j]);
  };
  bool a_written = false;  // A holds the backward state (else it is still phi)
  int fold = -1;           // gate whose u^dag the next step applies first (folded step)
  for (int k = c.L - 1; k >= 0; --k) {
    const int k_apply = (k == c.L - 1) ? -1 : k + 1;
    const int kind = kind_of(k);
    SBuf<R> a_in = a_written ? SBuf<R>{A, sN} : SBuf<R>{phi, 0};
    SBuf<R> b = k == 0 ? SBuf<R>{psi, 0} : SBuf<R>{B + (k - 1) * sN, bstride};
    if (kind == QFS_GATE_FIXED) {
      // a constant gate has no environment: only move the backward state through the
      // gate after it (nothing to do for the last gate). When the gate before it has an
      // environment and the gate after it acts on the same two qubits (a U3 + CNOT
      // block), that move is folded into the next step, which then applies
      // u_k^dag u_{k+1}^dag with one pass over the state instead of two.
      if (k_apply < 0) continue;
      if (k >= 1 && kind_of(k - 1) != QFS_GATE_FIXED && same_qubits(k, k + 1)) {
        fold = k + 1;
        continue;
      }
      for (int h = 0; h < halves; ++h) {
        QFS_TRY(T.begin(hs[h]));
        QFS_TRY(launch_apply<R>(c.g, c.pairs_host[2 * k_apply], c.pairs_host[2 * k_apply + 1], k_apply,
                                true, gr, a_in, SBuf<R>{A, sN}, hslots[h], hn[h], hs[h]));
        QFS_TRY(T.end(hs[h], kClsStep, 2.0 * set_bytes<R>(c, c.g) * hn[h] / c.nslots));
      }
      a_written = true;
      continue;
    }
    const int k_apply2 = fold;
    fold = -1;
    for (int h = 0; h < halves; ++h) {
      int P = 0;
      QFS_TRY(T.begin(hs[h]));
      QFS_TRY(launch_bwd_step<R>(c.g, c.pairs_host, k_apply, k, gr, a_in, SBuf<R>{A, sN}, b, hslots[h],
                                 hn[h], c.partials, &P, hs[h], k_apply2));
      QFS_TRY(T.end(hs[h], kClsStep, (k_apply < 0 ? 2.0 : 3.0) * set_bytes<R>(c, c.g) * hn[h] / c.nslots));
      QFS_TRY(T.begin(hs[h]));
      QFS_TRY(launch_env_finalize(P, c.partials, hslots[h], hn[h], nullptr, true, c.beta, c.g64,
                                  sizeof(R) == 4 ? c.g32 : nullptr, c.L * 16, k, c.vstore, kind, hs[h]));
      QFS_TRY(T.end(hs[h], kClsPolar, (double)P * 256.0 * hn[h]));
    }
    if (k_apply >= 0) a_written = true;
  }
  if (split) {
    QFS_HIP(hipEventRecord(c.join, c.side));
    QFS_HIP(hipStreamWaitEvent(c.stream, c.join, 0));
  }
  int P = 0;
  QFS_TRY(T.begin(c.stream));
  QFS_TRY(launch_apply_dist<R>(c.g, c.pairs_host[0], c.pairs_host[1], 0, true, gr,
                               a_written ? SBuf<R>{A, sN} : SBuf<R>{phi, 0}, SBuf<R>{psi, 0}, c.slots,
                               c.nslots, c.dpart0, &P, c.stream));
  QFS_TRY(T.end(c.stream, kClsDist, 2.0 * set_bytes<R>(c, c.g)));
  QFS_TRY(launch_dist_finalize(P, c.dpart0, c.slots, c.nslots, c.g.M, c.costs, c.stream));
  return QFS_OK;
}

// ------------------------------------------------------------------ control loop
struct GroupResult {
  int rc = QFS_OK;
  int reason = QFS_MAX_ITER;
  int best = -1;  // absolute start index
  double c_train = INFINITY, c_val = INFINITY;
  int m_final = 0, sweeps = 0, restarts = 0, m_total = 0;
  int64_t success_round = -1;  // sweep round at which the success was found
  int refined = 0;
  int64_t start_sweeps = 0;
  double amp_updates = 0.0;
  double sweep_seconds = 0.0;
  Counters k;
  std::vector<qfs_c128> gates;  // [L][16] of the chosen start (host copy)
};


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
    if (has_kinds(t)) {
      kinds_.assign(t->kinds, t->kinds + L_);
      fixed_ = reinterpret_cast<const c128 *>(t->fixed_gates);
    }
    stream_ = as_stream(p.hip_stream);
  }
  ~Group() {
    if (h_costs_) {
      // a run-ahead sweep's cost copies may still be in flight
      if (hipDeviceSynchronize() == hipSuccess)
        pinned_put(h_costs_, h_costs_bytes_);
      else
        (void)hipGetLastError();
    }
    if (seg0_) (void)hipEventDestroy(seg0_);
    for (auto &d : done_)
      for (hipEvent_t e : d)
        if (e) (void)hipEventDestroy(e);
    if (fork_) (void)hipEventDestroy(fork_);
    if (join_) (void)hipEventDestroy(join_);
    if (ctx_.pfork) (void)hipEventDestroy(ctx_.pfork);
    for (int p = 0; p < SweepCtx::kParts; ++p)
      if (ctx_.pjoin[p]) (void)hipEventDestroy(ctx_.pjoin[p]);

    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    if (gfork_) (void)hipEventDestroy(gfork_);
    if (vfork_) (void)hipEventDestroy(vfork_);
    if (vjoin_) (void)hipEventDestroy(vjoin_);
    if (gjoin_) (void)hipEventDestroy(gjoin_);

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
  std::vector<int32_t> kinds_;  // empty: every gate two-qubit
  const c128 *fixed_ = nullptr;
  std::vector<int32_t> fmode_;  // per gate: how the grouped forward pass applies it
  hipStream_t stream_ = nullptr;
  hipStream_t side_ = nullptr;  // second stream of the backward pass (default priority)
  hipEvent_t fork_ = nullptr, join_ = nullptr;
  // One sweep (backward pass, then the forward pass of the updated gates) captured as a
  // HIP graph on the internal stream cap_, replayed while nothing it depends on changes
  // (running starts, M, precision: each of those marks it dirty).
  hipStream_t cap_ = nullptr;
  hipEvent_t gfork_ = nullptr, gjoin_ = nullptr;
  hipEvent_t vfork_ = nullptr, vjoin_ = nullptr;  // validation set-up stream
  hipGraphExec_t gexec_ = nullptr;
  bool gdirty_ = true;
  int sweep_once();

  int M_ = 0, ldm_ = 0, Mv_ = 0, ldmv_ = 0, m_cap_ = 0, n_train_ = 0, generation_ = 0;
  bool fp64_ = true;
  DevBuf psi64_, phi64_, psiv64_, phiv64_;  // complex128 masters, row-major N x ldm
  DevBuf psiw_, phiw_, psivw_, phivw_;      // working sets in the sweep precision
  DevBuf blist_, astate_, vstate_;
  DevBuf g64_, g32_, vstore_, pairs_dev_, kinds_dev_;
  DevBuf partials_, dpart_, costs_, slots_, work_;
  DevBuf zslot_;  // one slot entry 0 (target simulation)
  DevBuf workv_;  // orthonormalisation work of the validation set
  DevBuf oflag_;  // set by the orthonormalisations on a non-positive pivot
  std::vector<GateGroup> groups_;  // grouped backward pass (backward_mode GROUPED)
  DevBuf bneed_dev_, gpartials_, vop_, fplan_dev_, fgslot_dev_;
  std::vector<int32_t> bneed_h_, fplan_h_, fgslot_h_;
  int gpstride_ = 0;
  // pinned [1 + 2 kParts][3 S] (c_train, c_val, c_0): read_costs's copy, then one copy per
  // sweep parity and part, written on the part's stream right after its sweep
  double *h_costs_ = nullptr;
  size_t h_costs_bytes_ = 0;
  double *cost_buf(int par, int part) { return h_costs_ + (size_t)(1 + par * SweepCtx::kParts + part) * 3 * S_; }
  // The control loop's sweeps: run-ahead (spec_), per sweep parity the starts and parts it
  // was issued with and an event per part at its end (timing reference seg0_), and the
  // snapshot of every start's gates after the sweep ([2][S][g64, g32, vstore]).
  struct Issued {
    std::vector<int> starts;
    int parts = 1;
    int off[SweepCtx::kParts] = {}, pn[SweepCtx::kParts] = {};
  };
  bool spec_ = false;
  Issued issued_[2];
  hipEvent_t done_[2][SweepCtx::kParts] = {};
  hipEvent_t seg0_ = nullptr;
  double seg_prev_ms_ = 0.0;
  DevBuf snap_, rslots_;
  size_t snap_bytes_per_start() const { return (size_t)L_ * 16 * (2 * sizeof(c128) + sizeof(c64)); }
  SlotCopy snap_copy(int par, bool restore);
  int begin_segment(bool new_ref);
  int end_segment();
  int issue_sweep(int par, const std::vector<int> &active);
  int wait_sweep(int par, std::vector<double> &ct, std::vector<double> &cv, double &seconds);
  int restore_gates(const std::vector<int> &starts, int par);
  KernelTimer timer_;
  SweepCtx ctx_;
  GroupResult *res_ = nullptr;

  int draw_training(int c0, int c1);
  int make_targets(DevBuf &psi, DevBuf &phi, int M, int ld, hipStream_t s);
  int draw_validation(hipStream_t s, bool targets = true);
  int setup_working();
  int set_slots(const std::vector<int> &active);
  int forward_any(bool with_c0) {
    return fp64_ ? sweep_forward<double>(ctx_, with_c0) : sweep_forward<float>(ctx_, with_c0);
  }
  int backward_any() { return fp64_ ? sweep_backward<double>(ctx_) : sweep_backward<float>(ctx_); }
  int read_costs(std::vector<double> &ct, std::vector<double> &cv, std::vector<double> *c0);
  int check_orth();
};

int Group::draw_training(int c0, int c1) {
  QFS_TRY(launch_ginibre(N_, c0, c1, ldm_, p_.seed, kRoleTrain, 0, psi64_.as<c128>(), stream_));
  QFS_TRY(arena_.alloc(work_, work_bytes_orth(N_, c1)));
  QFS_TRY(orthonormalize_columns(N_, ldm_, c0, c1, psi64_.as<c128>(), work_.ptr, stream_, oflag_.as<int>()));
  arena_.free(work_);
  return QFS_OK;
}

// phi = U psi (dense product, or simulation of the target circuit), FP64.
int Group::make_targets(DevBuf &psi, DevBuf &phi, int M, int ld, hipStream_t s) {
  if (tgt_->kind == QFS_TARGET_DENSE) {
    QFS_TRY(launch_zgemm(false, (int)N_, M, (int)N_, cmake(1.0, 0.0),
                         reinterpret_cast<const c128 *>(tgt_->U), (int)N_, psi.as<c128>(), ld,
                         cmake(0.0, 0.0), phi.as<c128>(), ld, s));
    return QFS_OK;
  }
  QFS_HIP(hipMemcpyAsync(phi.ptr, psi.ptr, sizeof(c128) * (size_t)N_ * ld, hipMemcpyDeviceToDevice, s));
  const qfs_template *ct = tgt_->circuit;
  const Geometry g{n_, (int32_t)N_, ceil_log2(ld), 1, M};  // the master is one chunk
  GateRef gr{reinterpret_cast<const c128 *>(tgt_->circuit_gates),
             reinterpret_cast<const c128 *>(tgt_->circuit_gates), 0};
  for (int k = 0; k < ct->n_gates; ++k) {
    QFS_TRY(launch_apply<double>(g, ct->pairs[2 * k], ct->pairs[2 * k + 1], k, false, gr,
                                 SBuf<double>{phi.as<c128>(), 0}, SBuf<double>{phi.as<c128>(), 0},
                                 zslot_.as<int32_t>(), 1, s));
  }
  return QFS_OK;
}

// The validation set (Sec. 3: held-out samples, drawn apart from the training set), on
// stream s; targets false leaves its target states to a make_targets call.
int Group::draw_validation(hipStream_t s, bool targets) {
  if (tgt_->kind == QFS_TARGET_SAMPLES) {
    Mv_ = tgt_->n_val;
    ldmv_ = master_ld(std::max(Mv_, 1));
    if (Mv_ == 0) return QFS_OK;
    QFS_TRY(arena_.alloc(psiv64_, sizeof(c128) * N_ * ldmv_));
    QFS_TRY(arena_.alloc(phiv64_, sizeof(c128) * N_ * ldmv_));
    const c128 *ps = reinterpret_cast<const c128 *>(tgt_->psi) + (size_t)n_train_ * N_;
    const c128 *ph = reinterpret_cast<const c128 *>(tgt_->phi) + (size_t)n_train_ * N_;
    QFS_TRY(launch_to_internal<double>(n_, Mv_, ceil_log2(ldmv_), 1, ps, psiv64_.as<c128>(), s));
    QFS_TRY(launch_to_internal<double>(n_, Mv_, ceil_log2(ldmv_), 1, ph, phiv64_.as<c128>(), s));
    return QFS_OK;
  }
  Mv_ = p_.m_val > 0 ? p_.m_val : M_;
  if (Mv_ > N_) Mv_ = (int)N_;
  ldmv_ = master_ld(Mv_);
  QFS_TRY(arena_.alloc(psiv64_, sizeof(c128) * N_ * ldmv_));
  QFS_TRY(arena_.alloc(phiv64_, sizeof(c128) * N_ * ldmv_));
  QFS_TRY(launch_zero(psiv64_.ptr, psiv64_.bytes, s));
  QFS_TRY(launch_ginibre(N_, 0, Mv_, ldmv_, p_.seed, kRoleVal, (uint32_t)generation_,
                         psiv64_.as<c128>(), s));
  QFS_TRY(arena_.alloc(workv_, work_bytes_orth(N_, Mv_)));
  QFS_TRY(orthonormalize_columns(N_, ldmv_, 0, Mv_, psiv64_.as<c128>(), workv_.ptr, s, oflag_.as<int>()));
  arena_.free(workv_);
  return targets ? make_targets(psiv64_, phiv64_, Mv_, ldmv_, s) : QFS_OK;
}

// Working sets in the sweep precision (chunk width chosen for the fused forward pass
// when a chunk of whole samples fits in LDS), and the per-start state buffers.
int Group::setup_working() {
  gdirty_ = true;
  const size_t rb = fp64_ ? sizeof(double) : sizeof(float);
  const size_t cb = 2 * rb;
  const size_t lds = lds_max_bytes();
  const bool fused = forward_fusable(n_, rb, lds);
  static const int logc_cap = [] {
    // tuning aid: cap the chunk width 2^logC (at least two samples: a complex64 packet
    // holds two samples of one amplitude)
    const char *e = std::getenv("QFS_LOGC_MAX");
    return e ? std::max(1, std::atoi(e)) : 30;
  }();
  const int logC = std::min(logc_cap, choose_log_chunk(n_, M_, rb, fused, S_, lds));
  const int C = 1 << logC;
  SweepCtx &c = ctx_;
  c.n = n_;
  c.L = L_;
  c.pairs_host = pairs_.data();
  c.pairs_dev = pairs_dev_.as<int32_t>();
  c.g = Geometry{n_, (int32_t)N_, logC, (M_ + C - 1) / C, M_};
  c.gv = Geometry{n_, (int32_t)N_, logC, std::max(1, (Mv_ + C - 1) / C), Mv_};
  c.fused = fused;
  c.grouped = p_.backward_mode == QFS_BWD_GROUPED && group_path_supported(c.g, rb);
  if (c.grouped) {
    // the partials grow with the chunk count (M); reallocated only when a larger stride is needed
    const int stride = group_partials_stride(c.g, rb);
    if (stride > gpstride_) {
      QFS_TRY(arena_.alloc(gpartials_, sizeof(c128) * 256 * (size_t)stride * S_));
      gpstride_ = stride;
    }
    if (!vop_.ptr) QFS_TRY(arena_.alloc(vop_, sizeof(c128) * 256 * (size_t)S_));
    if (!bneed_dev_.ptr) {
      bneed_h_.assign(L_, 0);
      for (const GateGroup &gg : groups_)
        if (gg.k_lo >= 1 && gg.nvar > 0) bneed_h_[gg.k_lo] = 1;
      QFS_TRY(arena_.alloc(bneed_dev_, sizeof(int32_t) * (size_t)L_));
      QFS_HIP(hipMemcpyAsync(bneed_dev_.ptr, bneed_h_.data(), sizeof(int32_t) * L_, hipMemcpyHostToDevice,
                             stream_));
    }
  }
  // the forward pass by groups (complex64 states, whole chunks in LDS); the plan follows the
  // chunk width
  c.fplan = c.fgslot = nullptr;
  c.fngroups = 0;
  if (c.grouped && fused && !fp64_ && build_forward_plan(c.g, L_, pairs_.data(), groups_, bneed_h_.data(),
                                                         fmode_.data(), fplan_h_, fgslot_h_) == QFS_OK) {
    if (!fplan_dev_.ptr) QFS_TRY(arena_.alloc(fplan_dev_, sizeof(int32_t) * fplan_h_.size()));
    if (!fgslot_dev_.ptr) QFS_TRY(arena_.alloc(fgslot_dev_, sizeof(int32_t) * fgslot_h_.size()));
    QFS_HIP(hipMemcpyAsync(fplan_dev_.ptr, fplan_h_.data(), sizeof(int32_t) * fplan_h_.size(),
                           hipMemcpyHostToDevice, stream_));
    QFS_HIP(hipMemcpyAsync(fgslot_dev_.ptr, fgslot_h_.data(), sizeof(int32_t) * fgslot_h_.size(),
                           hipMemcpyHostToDevice, stream_));
    c.fplan = fplan_dev_.as<int32_t>();
    c.fgslot = fgslot_dev_.as<int32_t>();
    c.fngroups = (int)groups_.size();
    c.fforms = std::any_of(fmode_.begin(), fmode_.end(), [](int32_t m) { return m != kFwdDense; });
  }
  if (!c.grouped && !partials_.ptr) {  // environment partials of the per-gate pass
    QFS_TRY(arena_.alloc(partials_, sizeof(c128) * 16 * (size_t)kPcap * S_));
    c.partials = partials_.as<c128>();
  }
  c.gpstride = gpstride_;
  c.vop = vop_.as<c128>();
  c.groups = &groups_;
  c.bneed_dev = bneed_dev_.as<int32_t>();
  c.gpartials = gpartials_.as<c128>();
  const size_t set = (size_t)c.g.elems() * cb, vset = (size_t)c.gv.elems() * cb;
  QFS_TRY(arena_.alloc(psiw_, set));
  QFS_TRY(arena_.alloc(phiw_, set));
  QFS_TRY(arena_.alloc(blist_, set * (size_t)S_ * (size_t)std::max(L_ - 1, 1)));
  QFS_TRY(arena_.alloc(astate_, set * (size_t)S_));
  if (Mv_ > 0) {
    QFS_TRY(arena_.alloc(psivw_, vset));
    QFS_TRY(arena_.alloc(phivw_, vset));
    if (!fused) QFS_TRY(arena_.alloc(vstate_, vset * (size_t)S_));
  }
  if (fp64_) {
    QFS_TRY(launch_pack<double>(c.g, ldm_, psi64_.as<c128>(), psiw_.as<c128>(), stream_));
    QFS_TRY(launch_pack<double>(c.g, ldm_, phi64_.as<c128>(), phiw_.as<c128>(), stream_));
    if (Mv_ > 0) {
      QFS_TRY(launch_pack<double>(c.gv, ldmv_, psiv64_.as<c128>(), psivw_.as<c128>(), stream_));
      QFS_TRY(launch_pack<double>(c.gv, ldmv_, phiv64_.as<c128>(), phivw_.as<c128>(), stream_));
    }
  } else {
    QFS_TRY(launch_pack<float>(c.g, ldm_, psi64_.as<c128>(), psiw_.as<c64>(), stream_));
    QFS_TRY(launch_pack<float>(c.g, ldm_, phi64_.as<c128>(), phiw_.as<c64>(), stream_));
    if (Mv_ > 0) {
      QFS_TRY(launch_pack<float>(c.gv, ldmv_, psiv64_.as<c128>(), psivw_.as<c64>(), stream_));
      QFS_TRY(launch_pack<float>(c.gv, ldmv_, phiv64_.as<c128>(), phivw_.as<c64>(), stream_));
    }
  }
  c.psi = psiw_.ptr;
  c.phi = phiw_.ptr;
  c.psiv = psivw_.ptr;
  c.phiv = phivw_.ptr;
  c.blist = blist_.ptr;
  c.astate = astate_.ptr;
  c.vstate = vstate_.ptr;
  return QFS_OK;
}

int Group::sweep_once() {
  if (!p_.graphs || timer_.on) {
    if (ctx_.grouped) return fp64_ ? sweep_grouped<double>(ctx_, true) : sweep_grouped<float>(ctx_, true);
    QFS_TRY(backward_any());
    return forward_any(false);
  }
  if (!cap_) {
    QFS_TRY(pool_stream(1, &cap_));
    QFS_HIP(hipEventCreateWithFlags(&gfork_, hipEventDisableTiming));
    QFS_HIP(hipEventCreateWithFlags(&gjoin_, hipEventDisableTiming));
  }
  // order the internal stream after everything issued so far on the caller's stream
  QFS_HIP(hipEventRecord(gfork_, stream_));
  QFS_HIP(hipStreamWaitEvent(cap_, gfork_, 0));
  if (gdirty_ || !gexec_) {
    if (gexec_) {
      QFS_HIP(hipGraphExecDestroy(gexec_));
      gexec_ = nullptr;
    }
    ctx_.stream = cap_;
    hipGraph_t graph = nullptr;
    QFS_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
    int rc;
    if (ctx_.grouped) {
      rc = fp64_ ? sweep_grouped<double>(ctx_, true) : sweep_grouped<float>(ctx_, true);
    } else {
      rc = backward_any();
      if (rc == QFS_OK) rc = forward_any(false);
    }
    const hipError_t e = hipStreamEndCapture(cap_, &graph);
    ctx_.stream = stream_;
    if (rc != QFS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    QFS_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&gexec_, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    QFS_HIP(ei);
    gdirty_ = false;
  }
  QFS_HIP(hipGraphLaunch(gexec_, cap_));
  QFS_HIP(hipEventRecord(gjoin_, cap_));
  QFS_HIP(hipStreamWaitEvent(stream_, gjoin_, 0));
  return QFS_OK;
}

int Group::set_slots(const std::vector<int> &active) {
  gdirty_ = true;
  ctx_.nslots = (int)active.size();
  if (ctx_.nslots == 0) return QFS_OK;
  QFS_HIP(hipMemcpyAsync(slots_.ptr, active.data(), sizeof(int32_t) * active.size(),
                         hipMemcpyHostToDevice, stream_));
  return QFS_OK;
}

// Snapshot copies of every start's gates (both precisions) and Jacobi warm starts, to or
// from the buffers of sweep parity par.
SlotCopy Group::snap_copy(int par, bool restore) {
  SlotCopy sc;
  const size_t per = snap_bytes_per_start();
  unsigned char *base = static_cast<unsigned char *>(snap_.ptr) + (size_t)par * per * S_;
  const size_t b64 = sizeof(c128) * 16 * (size_t)L_ * S_, b32 = sizeof(c64) * 16 * (size_t)L_ * S_;
  const void *live[3] = {g64_.ptr, g32_.ptr, vstore_.ptr};
  const void *copy[3] = {base, base + b64, base + b64 + b32};
  const int64_t units[3] = {(int64_t)L_ * 16, (int64_t)L_ * 8, (int64_t)L_ * 16};
  for (int b = 0; b < 3; ++b) {
    sc.src[b] = static_cast<const uint4 *>(restore ? copy[b] : live[b]);
    sc.dst[b] = const_cast<uint4 *>(static_cast<const uint4 *>(restore ? live[b] : copy[b]));
    sc.units[b] = units[b];
  }
  return sc;
}

// Order the part streams after the call's stream (and, with new_ref, restart the clock of
// the sweeps that follow).
int Group::begin_segment(bool new_ref) {
  if (new_ref) {
    QFS_HIP(hipEventRecord(seg0_, stream_));
    seg_prev_ms_ = 0.0;
  }
  if (!ctx_.pfork) return QFS_OK;
  QFS_HIP(hipEventRecord(ctx_.pfork, stream_));
  for (int p = 1; p < SweepCtx::kParts; ++p)
    if (ctx_.pstream[p]) QFS_HIP(hipStreamWaitEvent(ctx_.pstream[p], ctx_.pfork, 0));
  return QFS_OK;
}

// Order the call's stream after everything issued on the part streams.
int Group::end_segment() {
  for (int p = 1; p < SweepCtx::kParts; ++p)
    if (ctx_.pstream[p] && ctx_.pjoin[p]) {
      QFS_HIP(hipEventRecord(ctx_.pjoin[p], ctx_.pstream[p]));
      QFS_HIP(hipStreamWaitEvent(stream_, ctx_.pjoin[p], 0));
    }
  return QFS_OK;
}

// One sweep of the running starts (parity par). A grouped sweep without timing or graphs
// runs its parts on their streams with no join, each part going on into its next sweep;
// after each part: the snapshot of its gates (run-ahead only), its costs to the host and
// its end event.
int Group::issue_sweep(int par, const std::vector<int> &active) {
  Issued &is = issued_[par];
  is.starts = active;
  hipStream_t pst[SweepCtx::kParts];
  if (ctx_.grouped && !p_.graphs && !timer_.on) {
    is.parts = sweep_parts(ctx_, is.off, is.pn, pst);
    QFS_TRY(fp64_ ? sweep_grouped<double>(ctx_, true, true) : sweep_grouped<float>(ctx_, true, true));
  } else {
    is.parts = 1;
    is.off[0] = 0;
    is.pn[0] = ctx_.nslots;
    pst[0] = stream_;
    QFS_TRY(sweep_once());
  }
  for (int p = 0; p < is.parts; ++p) {
    if (spec_) QFS_TRY(launch_copy_slots(ctx_.slots + is.off[p], is.pn[p], snap_copy(par, false), pst[p]));
    QFS_HIP(hipMemcpyAsync(cost_buf(par, p), costs_.ptr, sizeof(double) * 3 * S_, hipMemcpyDeviceToHost, pst[p]));
    QFS_HIP(hipEventRecord(done_[par][p], pst[p]));
  }
  return QFS_OK;
}

// Wait for sweep parity par and read its costs (each start from its part's copy); seconds
// grows by the device time since the previous sweep's end.
int Group::wait_sweep(int par, std::vector<double> &ct, std::vector<double> &cv, double &seconds) {
  const Issued &is = issued_[par];
  float end_ms = 0.f;
  for (int p = 0; p < is.parts; ++p) {
    QFS_HIP(hipEventSynchronize(done_[par][p]));
    float ms = 0.f;
    QFS_HIP(hipEventElapsedTime(&ms, seg0_, done_[par][p]));
    end_ms = std::max(end_ms, ms);
  }
  seconds += 1e-3 * std::max(0.0, (double)end_ms - seg_prev_ms_);
  seg_prev_ms_ = std::max(seg_prev_ms_, (double)end_ms);
  if (res_ && timer_.on) {
    QFS_HIP(hipStreamSynchronize(stream_));
    QFS_TRY(timer_.flush(res_->k));
  }
  for (int p = 0; p < is.parts; ++p) {
    const double *h = cost_buf(par, p);
    for (int i = is.off[p]; i < is.off[p] + is.pn[p]; ++i) {
      const int s = is.starts[i];
      ct[s] = h[s];
      cv[s] = h[S_ + s];
    }
  }
  return QFS_OK;
}

// Gates and warm starts of the given starts back to the snapshot of sweep parity par, on
// the call's stream (after end_segment).
int Group::restore_gates(const std::vector<int> &starts, int par) {
  if (starts.empty()) return QFS_OK;
  QFS_HIP(hipMemcpyAsync(rslots_.ptr, starts.data(), sizeof(int32_t) * starts.size(), hipMemcpyHostToDevice,
                         stream_));
  return launch_copy_slots(rslots_.as<int32_t>(), (int)starts.size(), snap_copy(par, true), stream_);
}

// The orthonormalisations queued since the last check (after a stream synchronisation).
int Group::check_orth() {
  int h = 0;
  QFS_HIP(hipMemcpyAsync(&h, oflag_.ptr, sizeof(int), hipMemcpyDeviceToHost, stream_));
  QFS_HIP(hipStreamSynchronize(stream_));
  if (h) {
    set_error_detail("orthonormalisation: non-positive Cholesky pivot (dependent columns)");
    return QFS_ENUMERIC;
  }
  return QFS_OK;
}

int Group::read_costs(std::vector<double> &ct, std::vector<double> &cv, std::vector<double> *c0) {
  QFS_HIP(hipMemcpyAsync(h_costs_, costs_.ptr, sizeof(double) * 3 * S_, hipMemcpyDeviceToHost, stream_));
  QFS_HIP(hipStreamSynchronize(stream_));
  if (res_) QFS_TRY(timer_.flush(res_->k));
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
  const bool full_unitary = p_.full_unitary != 0;
  if (full_unitary) M_ = m_cap_ = (int)N_;
  ldm_ = master_ld(M_);
  fp64_ = p_.precision != QFS_PREC_MIXED;
  timer_.on = p_.timing != 0;
  res_ = &out;

  h_costs_bytes_ = sizeof(double) * 3 * S_ * (1 + 2 * SweepCtx::kParts);
  h_costs_ = static_cast<double *>(pinned_take(h_costs_bytes_));
  if (!h_costs_) return set_error_detail("hipHostMalloc of the cost buffer failed"), QFS_EDEVICE;
  // how the grouped forward pass applies each gate (the constant gates are the template's
  // in every start), before any work is queued on the stream
  {
    std::vector<c128> fixed_h;
    if (!kinds_.empty() && fixed_) {
      fixed_h.resize((size_t)L_ * 16);
      QFS_HIP(hipMemcpyAsync(fixed_h.data(), fixed_, sizeof(c128) * fixed_h.size(), hipMemcpyDeviceToHost,
                             stream_));
      QFS_HIP(hipStreamSynchronize(stream_));
    }
    fmode_ = forward_gate_modes(L_, kinds_.empty() ? nullptr : kinds_.data(),
                                fixed_h.empty() ? nullptr : fixed_h.data(), 1);
  }
  QFS_HIP(hipEventCreate(&seg0_));
  for (auto &d : done_)
    for (hipEvent_t &e : d) QFS_HIP(hipEventCreate(&e));
  QFS_TRY(arena_.alloc(dpart_, sizeof(double) * 2 * (size_t)kPcap * S_));
  QFS_TRY(arena_.alloc(costs_, sizeof(double) * 3 * S_));
  QFS_TRY(arena_.alloc(slots_, sizeof(int32_t) * S_));
  QFS_TRY(arena_.alloc(pairs_dev_, sizeof(int32_t) * 2 * (size_t)L_));
  QFS_HIP(hipMemcpyAsync(pairs_dev_.ptr, pairs_.data(), sizeof(int32_t) * 2 * L_, hipMemcpyHostToDevice,
                         stream_));
  QFS_TRY(launch_zero(costs_.ptr, costs_.bytes, stream_));
  QFS_TRY(arena_.alloc(zslot_, 16));
  QFS_TRY(arena_.alloc(oflag_, 16));
  QFS_TRY(launch_zero(zslot_.ptr, zslot_.bytes, stream_));
  QFS_TRY(launch_zero(oflag_.ptr, oflag_.bytes, stream_));
  // the validation set is drawn beside the training set, on a stream of its own: both are
  // chains of small kernels that leave most of the device idle
  hipStream_t vs = stream_;
  if (!samples && !full_unitary) {
    QFS_TRY(pool_stream(5, &vs));
    QFS_HIP(hipEventCreateWithFlags(&vfork_, hipEventDisableTiming));
    QFS_HIP(hipEventCreateWithFlags(&vjoin_, hipEventDisableTiming));
    QFS_HIP(hipEventRecord(vfork_, stream_));
    QFS_HIP(hipStreamWaitEvent(vs, vfork_, 0));
  }

  // training set and A tensor (computed once per training set)
  QFS_TRY(arena_.alloc(psi64_, sizeof(c128) * N_ * ldm_));
  QFS_TRY(arena_.alloc(phi64_, sizeof(c128) * N_ * ldm_));
  QFS_TRY(launch_zero(psi64_.ptr, psi64_.bytes, stream_));
  if (samples) {
    QFS_TRY(launch_to_internal<double>(n_, M_, ceil_log2(ldm_), 1, reinterpret_cast<const c128 *>(tgt_->psi),
                                       psi64_.as<c128>(), stream_));
    QFS_TRY(launch_to_internal<double>(n_, M_, ceil_log2(ldm_), 1, reinterpret_cast<const c128 *>(tgt_->phi),
                                       phi64_.as<c128>(), stream_));
  } else if (full_unitary) {
    // full-unitary QFactor: the computational basis, so phi holds U's columns
    QFS_TRY(launch_unit_columns(N_, ldm_, psi64_.as<c128>(), stream_));
    QFS_TRY(make_targets(psi64_, phi64_, M_, ldm_, stream_));
  } else {
    // both orthonormalisations are queued before either target simulation, so that the
    // two chains start together
    QFS_TRY(draw_training(0, M_));
    QFS_TRY(draw_validation(vs, false));
    QFS_TRY(make_targets(psi64_, phi64_, M_, ldm_, stream_));
  }
  if (full_unitary)
    Mv_ = 0;
  else if (samples)
    QFS_TRY(draw_validation(vs));
  else
    QFS_TRY(make_targets(psiv64_, phiv64_, Mv_, ldmv_, vs));

  // initial gates (App. A: random per start from the seed, or given)
  QFS_TRY(arena_.alloc(g64_, sizeof(c128) * 16 * (size_t)L_ * S_));
  QFS_TRY(arena_.alloc(g32_, sizeof(c64) * 16 * (size_t)L_ * S_));
  if (gates_in_) {
    QFS_HIP(hipMemcpyAsync(g64_.ptr, gates_in_ + (size_t)start0_ * L_ * 16,
                           sizeof(c128) * 16 * (size_t)L_ * S_, hipMemcpyDeviceToDevice, stream_));
  } else {
    QFS_TRY(launch_haar_gates(p_.seed, start0_, S_, L_, g64_.as<c128>(), stream_));
  }
  if (!kinds_.empty()) {
    QFS_TRY(arena_.alloc(kinds_dev_, sizeof(int32_t) * (size_t)L_));
    QFS_HIP(hipMemcpyAsync(kinds_dev_.ptr, kinds_.data(), sizeof(int32_t) * L_, hipMemcpyHostToDevice,
                           stream_));
    QFS_TRY(launch_kind_gates(p_.seed, start0_, S_, L_, kinds_dev_.as<int32_t>(), fixed_, !gates_in_,
                              g64_.as<c128>(), stream_));
  }
  QFS_TRY(launch_narrow((int64_t)16 * L_ * S_, g64_.as<c128>(), g32_.as<c64>(), stream_));
  QFS_TRY(arena_.alloc(vstore_, sizeof(c128) * 16 * (size_t)L_ * S_));
  QFS_TRY(launch_identity4((int64_t)L_ * S_, vstore_.as<c128>(), stream_));
  if (vs != stream_) {
    QFS_HIP(hipEventRecord(vjoin_, vs));
    QFS_HIP(hipStreamWaitEvent(stream_, vjoin_, 0));
  }

  groups_ = plan_gate_groups(L_, pairs_.data(), kinds_.empty() ? nullptr : kinds_.data());
  SweepCtx &c = ctx_;
  c.kinds = kinds_.empty() ? nullptr : kinds_.data();
  c.kinds_dev = kinds_.empty() ? nullptr : kinds_dev_.as<int32_t>();
  c.slots = slots_.as<int32_t>();
  c.g64 = g64_.as<c128>();
  c.g32 = g32_.as<c64>();
  c.vstore = vstore_.as<c128>();
  c.beta = effective_beta(p_.beta, p_.beta_normalized != 0, M_);
  c.partials = partials_.as<c128>();
  c.dpart0 = dpart_.as<double>();
  c.dpart1 = dpart_.as<double>() + (size_t)kPcap * S_;
  c.costs = costs_.as<double>();
  c.S = S_;
  c.timer = &timer_;
  c.stream = stream_;
  static const bool split_ok = [] {
    const char *e = std::getenv("QFS_BWD_SPLIT");  // 0: one stream for the backward pass
    return !(e && std::atoi(e) == 0);
  }();
  if (S_ >= 2 && split_ok) {
    QFS_TRY(pool_stream(0, &side_));
    QFS_HIP(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
    QFS_HIP(hipEventCreateWithFlags(&join_, hipEventDisableTiming));
    c.side = side_;
    c.fork = fork_;
    c.join = join_;
    static const int parts_env = [] {
      const char *e = std::getenv("QFS_PARTS");  // tuning aid: most stream parts of a sweep
      return e ? std::max(1, std::min(SweepCtx::kParts, std::atoi(e))) : 2;
    }();
    c.nparts = parts_env;
    c.pstream[1] = side_;
    for (int p = 2; p < SweepCtx::kParts; ++p) QFS_TRY(pool_stream(p + 1, &c.pstream[p]));
    QFS_HIP(hipEventCreateWithFlags(&c.pfork, hipEventDisableTiming));
    for (int p = 0; p < SweepCtx::kParts; ++p) QFS_HIP(hipEventCreateWithFlags(&c.pjoin[p], hipEventDisableTiming));
  }
  QFS_TRY(setup_working());

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
  QFS_TRY(check_orth());
  for (int s = 0; s < S_; ++s) {
    c_prev[s] = c0[s];
    ct[s] = c0[s];
    if (Mv_ == 0) cv[s] = ct[s];
  }

  // Run-ahead: sweep t + 1 of the running starts is issued before the costs of sweep t are
  // read, so the device never waits for the host's decisions. Its results are kept when
  // every start continues (the usual case); a start that stops at sweep t gets the gates it
  // had after sweep t back from the snapshot taken then, and a decision for all starts
  // (success, over-training, the switch to complex128) undoes sweep t + 1 of every start
  // before it acts, so the trajectory is that of one sweep at a time.
  static const bool run_ahead_env = [] {
    const char *e = std::getenv("QFS_RUN_AHEAD");  // tuning aid: 0 decides after every sweep
    return !(e && std::atoi(e) == 0);
  }();
  spec_ = run_ahead_env && !timer_.on;
  if (spec_) QFS_TRY(arena_.alloc(snap_, 2 * snap_bytes_per_start() * (size_t)S_));
  QFS_TRY(arena_.alloc(rslots_, sizeof(int32_t) * S_));
  int chosen = -1;
  int par = 0;  // parity of the sweep decided next (its snapshot and cost buffers)
  QFS_TRY(begin_segment(true));
  QFS_TRY(issue_sweep(par, active));
  std::vector<double> nct(S_), ncv(S_);
  for (;;) {
    // (not past max_iter: when sweep t is the last every running start may make, nothing is
    // issued ahead of it)
    bool last = true;
    for (int s : active) last = last && total[s] + 1 >= p_.max_iter;
    const bool ahead = spec_ && !last;
    if (ahead) QFS_TRY(issue_sweep(par ^ 1, active));
    QFS_TRY(wait_sweep(par, nct, ncv, out.sweep_seconds));
    ++round;
    out.start_sweeps += (int64_t)active.size();
    out.amp_updates += (double)active.size() * (double)(M_ + Mv_) * (double)N_ * (double)L_;

    const bool full = (int64_t)M_ == N_;
    bool any_success = false, any_over = false;
    const bool timed_out = p_.time_budget_s > 0 && now_s() - t_start > p_.time_budget_s;
    for (int s : active) {
      ct[s] = nct[s];
      cv[s] = Mv_ > 0 ? ncv[s] : nct[s];
      status[s] = control_step(p_, ct[s], cv[s], full || Mv_ == 0, M_ < m_cap_, timed_out, iter[s], z[s],
                               total[s], c_prev[s], reason[s]);
      any_success |= status[s] == ST_STOP && reason[s] == QFS_SUCCESS;
      any_over |= status[s] == ST_OVER;
    }
    std::vector<int> next;
    for (int s : active)
      if (status[s] == ST_RUN) next.push_back(s);
    // precision policy: complex128 refinement once the best running start is close
    bool switch_now = false;
    if (!fp64_ && !any_success && !any_over && !next.empty()) {
      double best = INFINITY;
      for (int s : next) best = std::min(best, ct[s]);
      switch_now = best < p_.refine_below;
    }
    const bool all_continue = !any_success && !any_over && !switch_now && next.size() == active.size();
    if (all_continue) {
      if (!ahead) QFS_TRY(issue_sweep(par ^ 1, active));
      par ^= 1;
      continue;
    }
    // something changes: order the call's stream after every part, then undo sweep t + 1
    // where its result is not kept. The survivors' sweep t + 1 is kept when only some starts
    // stopped and the survivors' passes split their sums as they would have if issued now
    // (grouped passes, same blocks per start), so that the result does not depend on the
    // run-ahead, bit for bit.
    const bool keep = ahead && !any_success && !any_over && !switch_now && !next.empty() && ctx_.grouped &&
                      group_blocks_per_start((int)next.size()) == group_blocks_per_start((int)active.size());
    QFS_TRY(end_segment());
    if (ahead) {
      if (keep) {
        std::vector<int> stopped;
        for (int s : active)
          if (status[s] != ST_RUN) stopped.push_back(s);
        QFS_TRY(restore_gates(stopped, par));
      } else {
        QFS_TRY(restore_gates(active, par));
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
      QFS_HIP(hipStreamSynchronize(stream_));
      const int M_new = std::min(2 * M_, m_cap_);
      const int ld_new = master_ld(M_new);
      DevBuf npsi, nphi;
      QFS_TRY(arena_.alloc(npsi, sizeof(c128) * N_ * ld_new));
      QFS_TRY(arena_.alloc(nphi, sizeof(c128) * N_ * ld_new));
      QFS_TRY(launch_zero(npsi.ptr, npsi.bytes, stream_));
      QFS_HIP(hipMemcpy2DAsync(npsi.ptr, sizeof(c128) * ld_new, psi64_.ptr, sizeof(c128) * ldm_,
                               sizeof(c128) * M_, N_, hipMemcpyDeviceToDevice, stream_));
      arena_.free(psi64_);  // (kept until the call ends: the copy above may still read it)
      arena_.free(phi64_);
      psi64_.swap(npsi);
      phi64_.swap(nphi);
      const int M_old = M_;
      M_ = M_new;
      ldm_ = ld_new;
      if (samples) {
        QFS_TRY(launch_to_internal<double>(n_, M_, ceil_log2(ldm_), 1, reinterpret_cast<const c128 *>(tgt_->psi),
                                           psi64_.as<c128>(), stream_));
        QFS_TRY(launch_to_internal<double>(n_, M_, ceil_log2(ldm_), 1, reinterpret_cast<const c128 *>(tgt_->phi),
                                           phi64_.as<c128>(), stream_));
      } else {
        // the new validation generation on its own stream, as in the set-up
        hipStream_t vs = stream_;
        if (vfork_) {
          QFS_TRY(pool_stream(5, &vs));
          QFS_HIP(hipEventRecord(vfork_, stream_));
          QFS_HIP(hipStreamWaitEvent(vs, vfork_, 0));
        }
        QFS_TRY(draw_training(M_old, M_));
        ++generation_;
        arena_.free(psiv64_);
        arena_.free(phiv64_);
        QFS_TRY(draw_validation(vs, false));
        QFS_TRY(make_targets(psi64_, phi64_, M_, ldm_, stream_));
        QFS_TRY(make_targets(psiv64_, phiv64_, Mv_, ldmv_, vs));
        if (vs != stream_) {
          QFS_HIP(hipEventRecord(vjoin_, vs));
          QFS_HIP(hipStreamWaitEvent(stream_, vjoin_, 0));
        }
      }
      QFS_TRY(setup_working());
      ctx_.beta = effective_beta(p_.beta, p_.beta_normalized != 0, M_);
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
      QFS_TRY(check_orth());
      for (int s : active) c_prev[s] = c0[s];
      par = 0;
      QFS_TRY(begin_segment(true));
      QFS_TRY(issue_sweep(par, active));
      continue;
    }
    if (next.empty()) {
      double best = INFINITY;
      for (int s = 0; s < S_; ++s)
        if (ct[s] < best || chosen < 0) {
          best = ct[s];
          chosen = s;
        }
      break;
    }
    // the forward pass just run (in sweep t, or in sweep t + 1 when it is kept) holds valid
    // B lists for the survivors
    active = next;
    QFS_TRY(set_slots(active));
    if (switch_now) {
      QFS_HIP(hipStreamSynchronize(stream_));
      fp64_ = true;
      out.refined = 1;
      QFS_TRY(setup_working());
      QFS_TRY(forward_any(false));  // B lists again, in complex128, from the FP64 gates
      par = 0;
      QFS_TRY(begin_segment(true));
      QFS_TRY(issue_sweep(par, active));
      continue;
    }
    // some starts stopped, the others go on: sweep t + 1 of the survivors, when kept, is the
    // next to decide (in the old parts; later sweeps use the new ones); else it is issued
    // now, after a forward pass that rebuilds the B lists from the restored gates
    if (ahead && !keep) QFS_TRY(forward_any(false));
    QFS_TRY(begin_segment(false));
    if (!keep) QFS_TRY(issue_sweep(par ^ 1, active));
    par ^= 1;
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
    if (r.rc != QFS_OK) (void)hipStreamSynchronize(as_stream(p.hip_stream));
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

// A per-gate (unfused) chunked geometry for the step entry points.
Geometry api_geometry(int n, int M) {
  const int logC = choose_log_chunk(n, M, sizeof(double), false, 1, 0);
  const int C = 1 << logC;
  return Geometry{n, 1 << n, logC, (M + C - 1) / C, M};
}

int one_slot(DevBuf &slot, hipStream_t s) {
  int32_t zero = 0;
  QFS_TRY(slot.alloc(sizeof(int32_t)));
  QFS_HIP(hipMemcpyAsync(slot.ptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
  return QFS_OK;
}

}  // namespace

// Gate slots [count][4][4] (gate index gi % L of the template) must be unitary to 1e-10,
// and a one-qubit slot must have the form v (x) I_2. fixed_only: check the constant gates
// only (the template's fixed_gates); else every slot but the constant gates' (gates_in).
int check_gates_unitary(const qfs_c128 *gates_dev, size_t count, int L, const int32_t *kinds,
                        bool fixed_only, const char *what, hipStream_t s) {
  std::vector<qfs_c128> h(count * 16);
  QFS_HIP(hipMemcpyAsync(h.data(), gates_dev, sizeof(qfs_c128) * h.size(), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  for (size_t gi = 0; gi < count; ++gi) {
    const qfs_c128 *u = h.data() + gi * 16;
    const int kind = kinds ? kinds[gi % L] : QFS_GATE_2Q;
    if ((kind == QFS_GATE_FIXED) != fixed_only) continue;
    if (kind == QFS_GATE_1Q) {
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          const qfs_c128 want = ((r & 1) == (c & 1)) ? u[(r & 2) * 4 + (c & 2)] : qfs_c128{0.0, 0.0};
          if (std::fabs(u[r * 4 + c].re - want.re) > 1e-10 || std::fabs(u[r * 4 + c].im - want.im) > 1e-10) {
            set_error_detail(std::string(what) + ": one-qubit gate " + std::to_string(gi) +
                             " is not of the form v (x) I_2");
            return QFS_EINVAL;
          }
        }
    }
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
          set_error_detail(std::string(what) + ": gate " + std::to_string(gi) + " is not unitary to 1e-10");
          return QFS_EINVAL;
        }
      }
  }
  return QFS_OK;
}

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

const char *qfs_version(void) { return "qfs-hip 0.2 (gfx950)"; }

int qfs_release_device_cache(size_t *bytes_freed) {
  int dev = 0;
  QFS_HIP(hipGetDevice(&dev));
  const size_t b = qfs::device_cache_trim(dev);
  if (bytes_freed) *bytes_freed = b;
  return QFS_OK;
}

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
  p->timing = 0;
  p->batch_sweeps = 0;
  p->batch_threads = 0;
  p->graphs = 0;
  p->full_unitary = 0;
  p->beta_normalized = 0;
  p->backward_mode = QFS_BWD_GROUPED;
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
      p.m_val < 0 || p.m_val > N || (p.full_unitary != 0 && p.full_unitary != 1) ||
      (p.beta_normalized != 0 && p.beta_normalized != 1) ||
      (p.backward_mode != QFS_BWD_GROUPED && p.backward_mode != QFS_BWD_PER_GATE)) {
    set_error_detail("params out of range");
    return QFS_EINVAL;
  }
  if (p.full_unitary && target->kind == QFS_TARGET_SAMPLES) {
    set_error_detail("full_unitary needs a DENSE or CIRCUIT target");
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
  if (gates_in)
    QFS_TRY(check_gates_unitary(gates_in, (size_t)p.multistarts * tmpl->n_gates, tmpl->n_gates,
                                tmpl->kinds, false, "gates_in", s));
  if (has_kinds(tmpl) && tmpl->fixed_gates)
    QFS_TRY(check_gates_unitary(tmpl->fixed_gates, (size_t)tmpl->n_gates, tmpl->n_gates, tmpl->kinds,
                                true, "fixed_gates", s));
  size_t budget = p.device_mem_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    int dev = 0;
    QFS_HIP(hipMemGetInfo(&fr, &tot));
    QFS_HIP(hipGetDevice(&dev));
    // blocks cached from earlier calls are free for this one
    budget = (size_t)(0.92 * (double)(fr + device_cache_held(dev)));
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
    res->amp_updates += x.amp_updates;
    res->sweep_seconds += x.sweep_seconds;
    for (int c = 0; c < kClasses; ++c) {
      res->kernel_launches[c] += x.k.kl[c];
      res->kernel_seconds[c] += x.k.ks[c];
      res->kernel_bytes[c] += x.k.kb[c];
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
  const int64_t N = int64_t(1) << n, ld = master_ld(M);
  DevBuf A, W;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(launch_zero(A.ptr, A.bytes, s));
  QFS_TRY(launch_ginibre(N, 0, M, ld, seed, role, stream, A.as<c128>(), s));
  QFS_TRY(W.alloc(work_bytes_orth(N, M)));
  QFS_TRY(orthonormalize_columns(N, ld, 0, M, A.as<c128>(), W.ptr, s));
  QFS_TRY(launch_from_internal<double>(n, M, ceil_log2(ld), A.as<c128>(), reinterpret_cast<c128 *>(out), s));
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

int qfs_apply_gates(int32_t n, int32_t M, qfs_c128 *states, int32_t L, const int32_t *pairs,
                    const qfs_c128 *gates, int32_t dagger, void *hip_stream) {
  qfs_template t{n, L, pairs};
  QFS_TRY(validate_template(&t));
  if (M < 1 || !states || !gates) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const Geometry g = api_geometry(n, M);
  DevBuf A, slot;
  QFS_TRY(A.alloc(sizeof(c128) * g.elems()));
  QFS_TRY(one_slot(slot, s));
  QFS_TRY(launch_to_internal<double>(n, M, g.logC, g.nch, reinterpret_cast<const c128 *>(states), A.as<c128>(), s));
  GateRef gr{reinterpret_cast<const c128 *>(gates), gates, 0};
  for (int i = 0; i < L; ++i) {
    const int k = dagger ? L - 1 - i : i;
    QFS_TRY(launch_apply<double>(g, pairs[2 * k], pairs[2 * k + 1], k, dagger != 0, gr,
                                 SBuf<double>{A.as<c128>(), 0}, SBuf<double>{A.as<c128>(), 0},
                                 slot.as<int32_t>(), 1, s));
  }
  QFS_TRY(launch_from_internal<double>(n, M, g.logC, A.as<c128>(), reinterpret_cast<c128 *>(states), s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_dense_apply(int32_t n, int32_t M, const qfs_c128 *U, const qfs_c128 *psi, qfs_c128 *out,
                    void *hip_stream) {
  if (n < 1 || n > 16 || M < 1 || !U || !psi || !out) return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const int64_t N = int64_t(1) << n, ld = master_ld(M);
  DevBuf A, B;
  QFS_TRY(A.alloc(sizeof(c128) * N * ld));
  QFS_TRY(B.alloc(sizeof(c128) * N * ld));
  QFS_TRY(launch_to_internal<double>(n, M, ceil_log2(ld), 1, reinterpret_cast<const c128 *>(psi), A.as<c128>(), s));
  QFS_TRY(launch_zgemm(false, (int)N, (int)ld, (int)N, cmake(1.0, 0.0), reinterpret_cast<const c128 *>(U),
                       (int)N, A.as<c128>(), (int)ld, cmake(0.0, 0.0), B.as<c128>(), (int)ld, s));
  QFS_TRY(launch_from_internal<double>(n, M, ceil_log2(ld), B.as<c128>(), reinterpret_cast<c128 *>(out), s));
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
  const Geometry g = api_geometry(n, M);
  DevBuf A, B, slot, part;
  QFS_TRY(A.alloc(sizeof(c128) * g.elems()));
  QFS_TRY(B.alloc(sizeof(c128) * g.elems()));
  QFS_TRY(part.alloc(sizeof(c128) * 16 * kPcap));
  QFS_TRY(one_slot(slot, s));
  QFS_TRY(launch_to_internal<double>(n, M, g.logC, g.nch, reinterpret_cast<const c128 *>(a), A.as<c128>(), s));
  QFS_TRY(launch_to_internal<double>(n, M, g.logC, g.nch, reinterpret_cast<const c128 *>(b), B.as<c128>(), s));
  GateRef gr{nullptr, nullptr, 0};
  int P = 0;
  QFS_TRY(launch_bwd_step<double>(g, pr, -1, 0, gr, SBuf<double>{A.as<c128>(), 0},
                                  SBuf<double>{A.as<c128>(), 0}, SBuf<double>{B.as<c128>(), 0},
                                  slot.as<int32_t>(), 1, part.as<c128>(), &P, s));
  QFS_TRY(launch_env_finalize(P, part.as<c128>(), slot.as<int32_t>(), 1, reinterpret_cast<c128 *>(gamma),
                              false, 0.0, nullptr, nullptr, 0, 0, nullptr, QFS_GATE_2Q, s));
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
  const Geometry g = api_geometry(n, M);
  DevBuf A, B, slot, part, out;
  QFS_TRY(A.alloc(sizeof(c128) * g.elems()));
  QFS_TRY(B.alloc(sizeof(c128) * g.elems()));
  QFS_TRY(part.alloc(sizeof(double) * kPcap));
  QFS_TRY(out.alloc(16));
  QFS_TRY(one_slot(slot, s));
  QFS_TRY(launch_to_internal<double>(n, M, g.logC, g.nch, reinterpret_cast<const c128 *>(x), A.as<c128>(), s));
  QFS_TRY(launch_to_internal<double>(n, M, g.logC, g.nch, reinterpret_cast<const c128 *>(y), B.as<c128>(), s));
  GateRef gr{nullptr, nullptr, 0};
  int P = 0;
  QFS_TRY(launch_apply_dist<double>(g, 0, 1, -1, false, gr, SBuf<double>{A.as<c128>(), 0},
                                    SBuf<double>{B.as<c128>(), 0}, slot.as<int32_t>(), 1,
                                    part.as<double>(), &P, s));
  QFS_TRY(launch_dist_finalize(P, part.as<double>(), slot.as<int32_t>(), 1, M, out.as<double>(), s));
  QFS_HIP(hipMemcpyAsync(result, out.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

int qfs_sweep(int32_t n, int32_t L, const int32_t *pairs, const int32_t *kinds, int32_t M,
              const qfs_c128 *psi, const qfs_c128 *phi, int32_t starts, qfs_c128 *gates,
              int32_t precision, double beta, int32_t backward_mode, double *c_train,
              void *hip_stream) {
  // constant gates are the gates' own entries here: validate the kinds without them
  std::vector<int32_t> kv;
  if (kinds) {
    kv.assign(kinds, kinds + std::max(L, 0));
    for (int32_t &k : kv)
      if (k == QFS_GATE_FIXED) k = QFS_GATE_2Q;
  }
  qfs_template t{n, L, pairs, kinds ? kv.data() : nullptr, nullptr};
  QFS_TRY(validate_template(&t));
  if (M < 1 || (int64_t)M > (int64_t(1) << n) || starts < 1 || !psi || !phi || !gates || !c_train ||
      (precision != QFS_PREC_FP64 && precision != QFS_PREC_MIXED) || !(beta >= 0 && beta <= 1) ||
      (backward_mode != QFS_BWD_GROUPED && backward_mode != QFS_BWD_PER_GATE))
    return QFS_EINVAL;
  hipStream_t s = as_stream(hip_stream);
  const bool f32 = precision == QFS_PREC_MIXED;
  const size_t rb = f32 ? sizeof(float) : sizeof(double), cb = 2 * rb;
  const size_t lds = lds_max_bytes();
  const bool fused = forward_fusable(n, rb, lds);
  const int logC = choose_log_chunk(n, M, rb, fused, starts, lds);
  const int C = 1 << logC;
  SweepCtx c;
  c.n = n;
  c.L = L;
  c.pairs_host = pairs;
  c.kinds = kinds;
  DevBuf kdev;
  if (kinds) {
    QFS_TRY(kdev.alloc(sizeof(int32_t) * L));
    QFS_HIP(hipMemcpyAsync(kdev.ptr, kinds, sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
    c.kinds_dev = kdev.as<int32_t>();
  }
  c.g = Geometry{n, 1 << n, logC, (M + C - 1) / C, M};
  c.gv = Geometry{n, 1 << n, logC, 1, 0};
  c.fused = fused;
  c.beta = beta;
  c.S = starts;
  KernelTimer timer;
  c.timer = &timer;
  c.stream = s;
  const size_t set = (size_t)c.g.elems() * cb;
  DevBuf ps, ph, Bl, As, g32, slots, part, dpart, costs, pdev;
  QFS_TRY(ps.alloc(set));
  QFS_TRY(ph.alloc(set));
  QFS_TRY(Bl.alloc(set * (size_t)std::max(L - 1, 1) * starts));
  QFS_TRY(As.alloc(set * starts));
  QFS_TRY(g32.alloc(sizeof(c64) * 16 * (size_t)L * starts));
  QFS_TRY(slots.alloc(sizeof(int32_t) * starts));
  QFS_TRY(part.alloc(sizeof(c128) * 16 * kPcap * (size_t)starts));
  QFS_TRY(dpart.alloc(sizeof(double) * 2 * kPcap * (size_t)starts));
  QFS_TRY(costs.alloc(sizeof(double) * 3 * starts));
  QFS_TRY(pdev.alloc(sizeof(int32_t) * 2 * L));
  QFS_HIP(hipMemcpyAsync(pdev.ptr, pairs, sizeof(int32_t) * 2 * L, hipMemcpyHostToDevice, s));
  std::vector<int32_t> sl(starts);
  for (int i = 0; i < starts; ++i) sl[i] = i;
  QFS_HIP(hipMemcpyAsync(slots.ptr, sl.data(), sizeof(int32_t) * starts, hipMemcpyHostToDevice, s));
  if (f32) {
    QFS_TRY(launch_to_internal<float>(n, M, logC, c.g.nch, reinterpret_cast<const c128 *>(psi), ps.as<c64>(), s));
    QFS_TRY(launch_to_internal<float>(n, M, logC, c.g.nch, reinterpret_cast<const c128 *>(phi), ph.as<c64>(), s));
    QFS_TRY(launch_narrow((int64_t)16 * L * starts, reinterpret_cast<const c128 *>(gates), g32.as<c64>(), s));
  } else {
    QFS_TRY(launch_to_internal<double>(n, M, logC, c.g.nch, reinterpret_cast<const c128 *>(psi), ps.as<c128>(), s));
    QFS_TRY(launch_to_internal<double>(n, M, logC, c.g.nch, reinterpret_cast<const c128 *>(phi), ph.as<c128>(), s));
  }
  c.pairs_dev = pdev.as<int32_t>();
  c.slots = slots.as<int32_t>();
  c.nslots = starts;
  c.g64 = reinterpret_cast<c128 *>(gates);
  c.g32 = g32.as<c64>();
  c.psi = ps.ptr;
  c.phi = ph.ptr;
  c.blist = Bl.ptr;
  c.astate = As.ptr;
  c.partials = part.as<c128>();
  c.dpart0 = dpart.as<double>();
  c.dpart1 = dpart.as<double>() + (size_t)kPcap * starts;
  c.costs = costs.as<double>();
  std::vector<GateGroup> groups;
  std::vector<int32_t> need, fplan_h, fgslot_h;
  DevBuf gpart, bneed, vopb, fplan_d, fgslot_d;
  c.grouped = backward_mode == QFS_BWD_GROUPED && group_path_supported(c.g, rb);
  if (c.grouped) {
    groups = plan_gate_groups(L, pairs, kinds);
    need.assign(L, 0);
    for (const GateGroup &gg : groups)
      if (gg.k_lo >= 1 && gg.nvar > 0) need[gg.k_lo] = 1;
    c.gpstride = group_partials_stride(c.g, rb);
    QFS_TRY(gpart.alloc(sizeof(c128) * 256 * (size_t)c.gpstride * starts));
    QFS_TRY(vopb.alloc(sizeof(c128) * 256 * (size_t)starts));
    c.vop = vopb.as<c128>();
    QFS_TRY(bneed.alloc(sizeof(int32_t) * L));
    QFS_HIP(hipMemcpyAsync(bneed.ptr, need.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
    c.groups = &groups;
    c.bneed_dev = bneed.as<int32_t>();
    c.gpartials = gpart.as<c128>();
    // how the forward pass applies each gate; a constant gate counts as a CNOT only if it
    // is one in every start's gates
    std::vector<int32_t> fmode;
    if (f32 && fused) {
      std::vector<c128> gh;
      bool any_fixed = false;
      for (int k = 0; kinds && k < L; ++k) any_fixed |= kinds[k] == QFS_GATE_FIXED;
      if (any_fixed) {
        gh.resize((size_t)starts * L * 16);
        QFS_HIP(hipMemcpyAsync(gh.data(), gates, sizeof(c128) * gh.size(), hipMemcpyDeviceToHost, s));
        QFS_HIP(hipStreamSynchronize(s));
      }
      fmode = forward_gate_modes(L, kinds, gh.empty() ? nullptr : gh.data(), starts);
    }
    if (f32 && fused && build_forward_plan(c.g, L, pairs, groups, need.data(), fmode.data(), fplan_h, fgslot_h) == QFS_OK) {
      QFS_TRY(fplan_d.alloc(sizeof(int32_t) * fplan_h.size()));
      QFS_TRY(fgslot_d.alloc(sizeof(int32_t) * fgslot_h.size()));
      QFS_HIP(hipMemcpyAsync(fplan_d.ptr, fplan_h.data(), sizeof(int32_t) * fplan_h.size(), hipMemcpyHostToDevice, s));
      QFS_HIP(hipMemcpyAsync(fgslot_d.ptr, fgslot_h.data(), sizeof(int32_t) * fgslot_h.size(),
                             hipMemcpyHostToDevice, s));
      c.fplan = fplan_d.as<int32_t>();
      c.fgslot = fgslot_d.as<int32_t>();
      c.fngroups = (int)groups.size();
      c.fforms = std::any_of(fmode.begin(), fmode.end(), [](int32_t m) { return m != kFwdDense; });
    }
  }
  if (f32) {
    QFS_TRY(sweep_forward<float>(c, false));
    QFS_TRY(sweep_backward<float>(c));
  } else {
    QFS_TRY(sweep_forward<double>(c, false));
    QFS_TRY(sweep_backward<double>(c));
  }
  QFS_HIP(hipMemcpyAsync(c_train, costs.ptr, sizeof(double) * starts, hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

}  // extern "C"
