// Sweep kernels of QFactor-Sample (Sec. 3; Fig. pre-comp; Fig. env_calc_tensor).
//
// State sets use the chunked amplitude-major layout (see qfs_internal.h): element
// (amplitude i, sample j) of a set lives at (j / C) * N * C + i * C + (j % C), C a power
// of two. A "packet" is 16 bytes of consecutive samples of one amplitude (two complex64
// or one complex128), so every access is a 16-byte vector access and a wave covers
// contiguous memory whatever qubits a gate acts on.
//
// Forward pass: one block per (chunk of C samples, start) holds the whole chunk in LDS,
// applies the gates in order and streams each intermediate state B_k to HBM straight
// from registers; validation states go through every gate without leaving LDS.
// Backward pass: grid = (P blocks, active starts); each thread owns "super groups": the
// 2^t amplitudes closed under the t <= 4 bit positions of the gate it applies (u^dag)
// and of the gate whose environment it accumulates. Environments are reduced thread ->
// wave (cross-lane shuffles) -> block (LDS, FP64 partial); a one-wave-per-start kernel
// then sums the block partials in a fixed order and runs the FP64 polar update.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "polar2.h"
#include "polar4.h"
#include "stream_common.h"
#include "qfs_internal.h"

namespace qfs {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kFwdBlock = 512;

template <typename R>
__device__ __forceinline__ R wave_sum(R x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Wave sums of the 16 complex entries of a 4x4 environment (32 reals) by recursive
// halving: at the exchange with lane ^ m (m = 32 .. 2) each lane keeps half of its values
// (the upper half when its bit m is set) and adds its partner's copy of that half, so 31
// exchanges replace 6 per value; a last exchange with lane ^ 1 completes the sums. Lane l
// returns the wave sum of real value l >> 1 (entry (l >> 2), real part when bit 1 of l is
// clear).
template <int C, typename R>
__device__ __forceinline__ void halve_level(R (&v)[32], int lane) {
  const bool hi = (lane & (2 * C)) != 0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const R give = hi ? v[i] : v[C + i];
    const R keep = hi ? v[C + i] : v[i];
    v[i] = keep + __shfl_xor(give, 2 * C);
  }
}
template <typename R>
__device__ __forceinline__ R wave_sum_env(const cx<R> (&acc)[16]) {
  const int lane = threadIdx.x & 63;
  R v[32];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    v[2 * e] = acc[e].re;
    v[2 * e + 1] = acc[e].im;
  }
  halve_level<16>(v, lane);
  halve_level<8>(v, lane);
  halve_level<4>(v, lane);
  halve_level<2>(v, lane);
  halve_level<1>(v, lane);
  return v[0] + __shfl_xor(v[0], 1);
}

// Local index of the environment gate's (q, sigma) inside a super group, per variant
// (see host-side classify_step for how the canonical bit order is built).
template <int VAR>
__device__ __forceinline__ constexpr int env_index(int q, int sg) {
  return VAR == 0   ? q
         : VAR == 1 ? ((q & 1) << 1) | (q >> 1)
         : VAR == 2 ? ((q >> 1) << 2) | (sg << 1) | (q & 1)
         : VAR == 3 ? (sg << 2) | ((q >> 1) << 1) | (q & 1)
         : VAR == 4 ? ((q & 1) << 2) | (sg << 1) | (q >> 1)
         : VAR == 5 ? (sg << 2) | ((q & 1) << 1) | (q >> 1)
                    : (sg << 2) | ((q >> 1) << 1) | (q & 1);
}
template <int VAR>
__host__ __device__ __forceinline__ constexpr int var_bits() {
  return VAR <= 1 ? 2 : (VAR <= 5 ? 3 : 4);
}

// Chunked index decomposition shared by the streaming kernels: item ->
// (chunk q, super group r, packet jv), packets fastest.
struct ChunkGeom {
  int32_t logC;     // log2 chunk width
  int32_t logJ;     // log2 packets per chunk row (C / V)
  int32_t logG;     // log2 super groups per chunk (n - t)
  int32_t n;
  uint32_t items;   // nch << (logG + logJ)
};

__device__ __forceinline__ void split_item(uint32_t it, const ChunkGeom &cg, uint32_t &q,
                                           uint32_t &r, uint32_t &jv) {
  jv = it & ((1u << cg.logJ) - 1u);
  const uint32_t rest = it >> cg.logJ;
  r = rest & ((1u << cg.logG) - 1u);
  q = rest >> cg.logG;
}

// u^dag of gate k_apply, or u_{k_apply}^dag u_{k_apply2}^dag when a second gate on the same
// two qubits goes first (a constant gate's backward step folded into the next one); the
// second gate is taken into the first one's local basis (indices 1 and 2 exchanged when
// it names the qubits in the opposite order)
template <typename R>
__device__ __forceinline__ void load_step_gate(const cx<R> *g, int k_apply, int k_apply2, int swap2,
                                               cx<R> (&ud)[16]) {
  load_gate<R>(g + k_apply * 16, ud, true);
  if (k_apply2 < 0) return;
  cx<R> u2[16];
  load_gate<R>(g + k_apply2 * 16, u2, true);
  if (swap2) {
    constexpr int pm[4] = {0, 2, 1, 3};
    cx<R> t[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = u2[pm[e >> 2] * 4 + pm[e & 3]];
#pragma unroll
    for (int e = 0; e < 16; ++e) u2[e] = t[e];
  }
  cx<R> m[16];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      cx<R> acc = cmake<R>(0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) cfma(acc, ud[q * 4 + r], u2[r * 4 + p]);
      m[q * 4 + p] = acc;
    }
#pragma unroll
  for (int e = 0; e < 16; ++e) ud[e] = m[e];
}


// ------------------------------------------------------------------ per-gate apply
template <typename R>
struct ApplySeg {
  const cx<R> *src;
  int64_t src_stride;
  cx<R> *dst;
  int64_t dst_stride;
  ChunkGeom cg;
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_apply(ApplySeg<R> sg, int pa, int pb,
                                                  const cx<R> *gates, int32_t gstride, int k,
                                                  int dagger, const int32_t *slot_to_start) {
  const int s = slot_to_start[blockIdx.y];
  cx<R> u[16];
  load_gate<R>(gates + (int64_t)s * gstride + k * 16, u, dagger != 0);
  const cx<R> *src = sg.src + sg.src_stride * s;
  cx<R> *dst = sg.dst + sg.dst_stride * s;
  const int lo = min(pa, pb), hi = max(pa, pb);
  const int sorted[2] = {lo, hi};
  constexpr int V = Pk<R>::V;
  const int logC = sg.cg.logC, n = sg.cg.n;
  const uint32_t ma = 1u << pa, mb = 1u << pb;
  for (uint32_t it = blockIdx.x * kBlock + threadIdx.x; it < sg.cg.items; it += gridDim.x * kBlock) {
    uint32_t q, rr, jv;
    split_item(it, sg.cg, q, rr, jv);
    const uint32_t i0 = deposit(rr, sorted, 2);
    const int64_t base = ((int64_t)q << (n + logC)) + jv * V;
    int64_t o[4];
    o[0] = base + ((int64_t)i0 << logC);
    o[1] = base + ((int64_t)(i0 + mb) << logC);
    o[2] = base + ((int64_t)(i0 + ma) << logC);
    o[3] = base + ((int64_t)(i0 + ma + mb) << logC);
    Pk<R> x[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) x[p] = ld_pk(src + o[p]);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      Pk<R> y;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        cx<R> acc = cmake<R>(0, 0);
#pragma unroll
        for (int p = 0; p < 4; ++p) cfma(acc, u[qq * 4 + p], x[p].v[e]);
        y.v[e] = acc;
      }
      st_pk(dst + o[qq], y);
    }
  }
}

// ------------------------------------------------------------------ fused forward
template <typename R>
struct FwdSeg {
  const cx<R> *src;     // initial states (shared by all starts), chunked
  cx<R> *blist;         // B list (B_{k+1} at list index k) or nullptr
  int64_t bstride;      // per start
  int64_t sN;           // per list entry
  const cx<R> *ref;     // states to compare against after the last applied gate, or nullptr
  double *partials;     // [S][nch] distance partials
  int32_t nch;          // chunks
  int32_t kapply;       // gates applied: 0 .. kapply-1
  int32_t kstore;       // outputs stored for gates 0 .. kstore-1
};

// One LDS pass over gates k0 .. k0 + run - 1, all on the qubits of gate k0 (in either
// order). Each gate is taken into gate k0's local basis (indices 1 and 2 exchanged when
// it names the qubits the other way round); a one-qubit slot v (x) I_2 skips its zero
// products (on the first local bit in its own order, so on the second one when
// exchanged). B_{k+1} is stored from registers after gate k when some environment reads
// it (bit j of store_mask: after gate k0 + j; blist: this chunk's entry 0 of the start,
// entries sN apart).
template <typename R>
__device__ __forceinline__ void forward_run(cx<R> *lds, uint32_t groups, int logJ, int logC,
                                            const int (&sorted)[2], uint32_t ma, uint32_t mb,
                                            cptr<int32_t> pairs, cptr<cx<R>> g, cptr<int32_t> kinds,
                                            int k0, int run, uint32_t store_mask, cx<R> *blist,
                                            int64_t sN) {
  constexpr int V = Pk<R>::V;
  constexpr bool MF = std::is_same<R, float>::value;  // complex64: products on the matrix cores
  const int FB = blockDim.x;
  const uint32_t lane = threadIdx.x & 63u;
  // (wave-uniform trip count: every lane of a wave runs the matrix-core products)
  for (uint32_t gb = threadIdx.x - lane; gb < groups; gb += FB) {
    const uint32_t gi = gb + lane;
    const bool ok = gi < groups;
    const uint32_t jv = gi & ((1u << logJ) - 1u);
    const uint32_t i0 = deposit(gi >> logJ, sorted, 2);
    uint32_t o[4];
    o[0] = (i0 << logC) + jv * V;
    o[1] = ((i0 + mb) << logC) + jv * V;
    o[2] = ((i0 + ma) << logC) + jv * V;
    o[3] = ((i0 + ma + mb) << logC) + jv * V;
    Pk<R> x[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (ok) {
        x[p] = ld_pk(lds + o[p]);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) x[p].v[e] = cmake<R>(0, 0);
      }
    }
    for (int j = 0; j < run; ++j) {
      const int k = k0 + j;
      const bool swapped = pairs[2 * k] != pairs[2 * k0];
      if constexpr (MF) {
        const Gate4 G4 = gate4_row(g + k * 16, swapped);
        Pk<R> y[4];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          c64 xe[4], ye[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) xe[p] = x[p].v[e];
          gate4_apply(G4, xe, ye);
#pragma unroll
          for (int p = 0; p < 4; ++p) y[p].v[e] = ye[p];
        }
        if (ok && blist && ((store_mask >> j) & 1u)) {
          cx<R> *dst = blist + sN * k;
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) st_pk(dst + o[qq], y[qq]);
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) x[qq] = y[qq];
        continue;
      }
      cx<R> u[16];
      load_gate<R>(g + k * 16, u, false);
      if (swapped) {
        constexpr int pm[4] = {0, 2, 1, 3};
        cx<R> t[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) t[e] = u[pm[e >> 2] * 4 + pm[e & 3]];
#pragma unroll
        for (int e = 0; e < 16; ++e) u[e] = t[e];
      }
      const int mode = (kinds && kinds[k] == QFS_GATE_1Q) ? (swapped ? 2 : 1) : 0;
      Pk<R> y[4];
      auto product = [&](auto m) {
        constexpr int MODE = decltype(m)::value;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
          for (int e = 0; e < V; ++e) {
            cx<R> acc = cmake<R>(0, 0);
#pragma unroll
            for (int p = 0; p < 4; ++p)
              if (MODE == 0 || (MODE == 1 ? (p & 1) == (qq & 1) : (p >> 1) == (qq >> 1)))
                cfma(acc, u[qq * 4 + p], x[p].v[e]);
            y[qq].v[e] = acc;
          }
      };
      if (mode == 0)
        product(std::integral_constant<int, 0>{});
      else if (mode == 1)
        product(std::integral_constant<int, 1>{});
      else
        product(std::integral_constant<int, 2>{});
      if (ok && blist && ((store_mask >> j) & 1u)) {
        cx<R> *dst = blist + sN * k;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) st_pk(dst + o[qq], y[qq]);
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) x[qq] = y[qq];
    }
    if (ok) {
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) st_pk(lds + o[qq], x[qq]);
    }
  }
}

// A gate on the lowest amplitude bits makes a thread's four outputs rows 32 or 64 bytes
// apart; for such gates (when coalesce_b is set) B_k leaves LDS in a second, contiguous
// pass instead of straight from registers.
//
// With two segments (training and validation sets) blockIdx.x alternates between them
// (even: seg0 chunk x/2, odd: seg1 chunk x/2), so the store-bound training chunks and the
// arithmetic-bound validation chunks (which store nothing) are dispatched side by side
// and overlap, instead of one phase of the grid after the other.
template <typename R, int FB>
__global__ __launch_bounds__(FB) void k_forward_fused(FwdSeg<R> seg0, FwdSeg<R> seg1, int nseg, int n,
                                                             int logC, const int32_t *pairs_in,
                                                             const cx<R> *gates_in, int32_t gstride,
                                                             const int32_t *slot_to_start,
                                                             int coalesce_b, const int32_t *kinds_in,
                                                             const int32_t *bneed_in) {
  const cptr<int32_t> pairs = as_const(pairs_in);
  const cptr<int32_t> kinds = kinds_in ? as_const(kinds_in) : (cptr<int32_t>)nullptr;
  const cptr<int32_t> bneed = bneed_in ? as_const(bneed_in) : (cptr<int32_t>)nullptr;
  // B_j is read by the backward pass: the given mask, else every entry but those before a
  // constant gate
  auto needed = [&](int j) { return bneed ? bneed[j] != 0 : !(kinds && kinds[j] == QFS_GATE_FIXED); };
  const cptr<cx<R>> gates = as_const(gates_in);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cx<R> *lds = reinterpret_cast<cx<R> *>(lds_raw);
  __shared__ double red[FB / 64];
  const bool second = nseg == 2 && (blockIdx.x & 1);
  const FwdSeg<R> sg = second ? seg1 : seg0;
  const int q = nseg == 2 ? (int)(blockIdx.x >> 1) : (int)blockIdx.x;
  if (q >= sg.nch) return;
  const int s = slot_to_start[blockIdx.y];
  constexpr int V = Pk<R>::V, LOGV = Pk<R>::LOGV;
  const int logJ = logC - LOGV;
  const uint32_t chunk = 1u << (n + logC);                 // elements per chunk
  const int64_t cbase = (int64_t)q << (n + logC);
  const cx<R> *src = sg.src + cbase;
  for (uint32_t e = threadIdx.x * V; e < chunk; e += FB * V) st_pk(lds + e, ld_pk(src + e));
  __syncthreads();
  const uint32_t groups = 1u << (n - 2 + logJ);
  for (int k = 0; k < sg.kapply;) {
    const int pa = n - 1 - pairs[2 * k], pb = n - 1 - pairs[2 * k + 1];
    const int sorted[2] = {min(pa, pb), max(pa, pb)};
    const uint32_t ma = 1u << pa, mb = 1u << pb;
    // the gates after k on the same two qubits (a U3 + CNOT block) join this pass: each
    // group of four amplitudes goes through all of them in registers, with their B list
    // entries stored on the way, and LDS is read and written once. Not for gates on the
    // lowest amplitude bits when B entries are stored (those leave LDS in a second pass).
    int run = 1;
    if (sg.kstore == 0 || !(coalesce_b && ((sizeof(cx<R>) << (logC + min(pa, pb))) < 128))) {
      while (k + run < sg.kapply && run < 32) {
        const int c0 = pairs[2 * (k + run)], c1 = pairs[2 * (k + run) + 1];
        const int a0 = pairs[2 * k], a1 = pairs[2 * k + 1];
        if (!((c0 == a0 && c1 == a1) || (c0 == a1 && c1 == a0))) break;
        ++run;
      }
    }
    run = __builtin_amdgcn_readfirstlane(run);
    if (run > 1) {
      // which gates of the run are followed by a B entry some environment reads (none
      // before a constant gate); uniform, worked out before the per-thread loop
      uint32_t mask = 0;
      for (int j = 0; j < run; ++j)
        if (k + j < sg.kstore && needed(k + j + 1)) mask |= 1u << j;
      mask = __builtin_amdgcn_readfirstlane(mask);
      forward_run<R>(lds, groups, logJ, logC, sorted, ma, mb, pairs, gates + (int64_t)s * gstride, kinds, k,
                     run, mask, sg.blist ? sg.blist + sg.bstride * s + cbase : nullptr, sg.sN);
      __syncthreads();
      k += run;
      continue;
    }
    cx<R> u[16];
    load_gate<R>(gates + (int64_t)s * gstride + k * 16, u, false);
    // B_{k+1} serves only the environment of gate k+1: none for a constant gate
    const bool store = k < sg.kstore && needed(k + 1);
    cx<R> *dst = store ? sg.blist + sg.bstride * s + sg.sN * k + cbase : nullptr;
    const bool late = store && coalesce_b && ((sizeof(cx<R>) << (logC + min(pa, pb))) < 128);
    // a one-qubit slot is v (x) I_2: output 2i + j mixes inputs j and 2 + j only, so half
    // of the products (those with the slot's exact zeros) are skipped; the remaining ones
    // are accumulated in the same order, so the result is that of the full product
    if constexpr (std::is_same<R, float>::value) {
      // complex64: the products on the matrix cores (wave-uniform trip count)
      const Gate4 G4 = gate4_row(gates + (int64_t)s * gstride + k * 16, false);
      const uint32_t lane = threadIdx.x & 63u;
      for (uint32_t gb = threadIdx.x - lane; gb < groups; gb += FB) {
        const uint32_t g = gb + lane;
        const bool ok = g < groups;
        const uint32_t jv = g & ((1u << logJ) - 1u);
        const uint32_t i0 = deposit(g >> logJ, sorted, 2);
        uint32_t o[4];
        o[0] = (i0 << logC) + jv * V;
        o[1] = ((i0 + mb) << logC) + jv * V;
        o[2] = ((i0 + ma) << logC) + jv * V;
        o[3] = ((i0 + ma + mb) << logC) + jv * V;
        Pk<R> x[4], y[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          if (ok) {
            x[p] = ld_pk(lds + o[p]);
          } else {
#pragma unroll
            for (int e = 0; e < V; ++e) x[p].v[e] = cmake<R>(0, 0);
          }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          c64 xe[4], ye[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) xe[p] = x[p].v[e];
          gate4_apply(G4, xe, ye);
#pragma unroll
          for (int p = 0; p < 4; ++p) y[p].v[e] = ye[p];
        }
        if (ok) {
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            st_pk(lds + o[qq], y[qq]);
            if (store && !late) st_pk(dst + o[qq], y[qq]);
          }
        }
      }
    }
    auto apply = [&](auto one_qubit) {
      constexpr bool ONEQ = decltype(one_qubit)::value;
      for (uint32_t g = threadIdx.x; g < groups; g += FB) {
        const uint32_t jv = g & ((1u << logJ) - 1u);
        const uint32_t i0 = deposit(g >> logJ, sorted, 2);
        uint32_t o[4];
        o[0] = (i0 << logC) + jv * V;
        o[1] = ((i0 + mb) << logC) + jv * V;
        o[2] = ((i0 + ma) << logC) + jv * V;
        o[3] = ((i0 + ma + mb) << logC) + jv * V;
        Pk<R> x[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) x[p] = ld_pk(lds + o[p]);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          Pk<R> y;
#pragma unroll
          for (int e = 0; e < V; ++e) {
            cx<R> acc = cmake<R>(0, 0);
#pragma unroll
            for (int p = 0; p < 4; ++p)
              if (!ONEQ || (p & 1) == (qq & 1)) cfma(acc, u[qq * 4 + p], x[p].v[e]);
            y.v[e] = acc;
          }
          st_pk(lds + o[qq], y);
          if (store && !late) st_pk(dst + o[qq], y);
        }
      }
    };
    if constexpr (!std::is_same<R, float>::value) {
      if (kinds && kinds[k] == QFS_GATE_1Q)
        apply(std::true_type{});
      else
        apply(std::false_type{});
    }
    __syncthreads();
    if (late) {
      for (uint32_t e = threadIdx.x * V; e < chunk; e += FB * V) st_pk(dst + e, ld_pk(lds + e));
      __syncthreads();
    }
    ++k;
  }
  if (sg.ref) {
    const cx<R> *ref = sg.ref + cbase;
    double acc = 0.0;
    for (uint32_t e = threadIdx.x * V; e < chunk; e += FB * V) {
      const Pk<R> a = ld_pk(lds + e), b = ld_pk(ref + e);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const R dr = a.v[v].re - b.v[v].re, di = a.v[v].im - b.v[v].im;
        acc += (double)dr * (double)dr + (double)di * (double)di;
      }
    }
    acc = wave_sum<double>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int w = 0; w < FB / 64; ++w) tot += red[w];
      sg.partials[(int64_t)s * sg.nch + q] = tot;
    }
  }
}

// ------------------------------------------------------------------ backward step
struct StepGeom {
  ChunkGeom cg;
  int32_t t;
  int32_t sorted_pos[4];
  int32_t off[16];  // amplitude-index offset of each local index
};

template <typename R>
struct StepArgs {
  const cx<R> *a_in;
  int64_t a_in_stride;
  cx<R> *a_out;
  int64_t a_out_stride;
  const cx<R> *b;
  int64_t b_stride;
  const cx<R> *gR;      // gates in state precision
  int32_t gstride;
  int32_t k_apply;
  int32_t k_apply2;     // >= 0: apply u^dag of this gate first (same qubits as k_apply)
  int32_t swap2;        // k_apply2 names the two qubits in the opposite order
  c128 *partials;       // [S][kPcap][16], blocks 0 .. P-1 used
  const int32_t *slot_to_start;
  StepGeom geo;
};

// EXTRA: the step may fold a second gate into its apply (k_apply2); a separate
// instantiation, so the common step keeps its registers.
template <typename R, int VAR, bool APPLY, bool EXTRA>
__global__ __launch_bounds__(kBlock) void k_bwd_step(StepArgs<R> A) {
  constexpr int t = var_bits<VAR>();
  constexpr int NL = 1 << t;
  constexpr int NS = NL / 4;
  constexpr int V = Pk<R>::V;
  __shared__ double red[kWaves][32];

  const int s = A.slot_to_start[blockIdx.y];
  const int P = gridDim.x;
  cx<R> ud[16];
  if (APPLY) {
    if (EXTRA)
      load_step_gate<R>(A.gR + (int64_t)s * A.gstride, A.k_apply, A.k_apply2, A.swap2, ud);
    else
      load_gate<R>(A.gR + (int64_t)s * A.gstride + A.k_apply * 16, ud, true);
  }
  const cx<R> *a_in = A.a_in + A.a_in_stride * s;
  cx<R> *a_out = A.a_out + A.a_out_stride * s;
  const cx<R> *b = A.b + A.b_stride * s;
  const StepGeom &G = A.geo;
  const int logC = G.cg.logC, n = G.cg.n;

  cx<R> acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = cmake<R>(0, 0);

  for (uint32_t it = blockIdx.x * kBlock + threadIdx.x; it < G.cg.items; it += P * kBlock) {
    uint32_t q, rr, jv;
    split_item(it, G.cg, q, rr, jv);
    const int64_t base = ((int64_t)q << (n + logC)) + ((int64_t)deposit(rr, G.sorted_pos, t) << logC) + jv * V;
    Pk<R> a[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) a[l] = ld_pk(a_in + base + ((int64_t)G.off[l] << logC));
    // keep the NL loads of the super group together (one memory round trip per item): left
    // to itself the scheduler folds each packet into the product as it arrives and waits
    // for every load in turn
    __builtin_amdgcn_sched_barrier(0);
    if (APPLY) {
#pragma unroll
      for (int rho = 0; rho < NS; ++rho) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          cx<R> x[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) x[p] = a[p * NS + rho].v[e];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            cx<R> y = cmake<R>(0, 0);
#pragma unroll
            for (int p = 0; p < 4; ++p) cfma(y, ud[qq * 4 + p], x[p]);
            a[qq * NS + rho].v[e] = y;
          }
        }
      }
#pragma unroll
      for (int l = 0; l < NL; ++l) st_pk(a_out + base + ((int64_t)G.off[l] << logC), a[l]);
    }
    // the item's B_k packets, likewise in one batch (issued after the stores: loading them
    // together with the state costs an occupancy step and measured no faster)
    Pk<R> bl[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) bl[l] = ld_pk(b + base + ((int64_t)G.off[l] << logC));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const Pk<R> &aq = a[env_index<VAR>(qq, sg)];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int e = 0; e < V; ++e) cfma_conj(acc[qq * 4 + p], aq.v[e], bl[env_index<VAR>(p, sg)].v[e]);
      }
    }
  }

  // thread -> wave -> block partial (FP64 across waves)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const R ws = wave_sum_env<R>(acc);
  if ((lane & 1) == 0) red[wv][lane >> 1] = (double)ws;
  __syncthreads();
  if (threadIdx.x < 16) {
    const int e = threadIdx.x;
    c128 sum = cmake(red[0][2 * e], red[0][2 * e + 1]);
    for (int w = 1; w < kWaves; ++w) sum = sum + cmake(red[w][2 * e], red[w][2 * e + 1]);
    A.partials[((int64_t)s * kPcap + blockIdx.x) * 16 + threadIdx.x] = sum;
  }
}

// LDS-staged variant of the backward step for steps whose gates act on the lowest
// amplitude bits. There a thread's super-group members are rows 32 or 64 bytes apart,
// so in k_bwd_step each load instruction of a wave touches four times as many cache
// lines as it fills. Here a wave owns a "box": the rows spanned by the t gate bits and
// the W lowest other bits (64 packets per gate-bit combination). It reads the box with
// one fully contiguous 1 KB access per combination, stages it in its own LDS slice, and
// each lane then takes its super group out of LDS; updated states leave the same way.
// The arithmetic per super group is that of k_bwd_step.
constexpr int kLdsBlock = 128;
constexpr int kLdsWaves = kLdsBlock / 64;

struct LdsGeom {
  int32_t W;           // row bits inside a box besides the gate bits (6 - logJ)
  int32_t logJ;        // log2 packets per row
  int32_t nps;         // W + t
  int32_t logWin;      // n - t - W: other row bits above the box
  uint32_t witems;     // boxes per start: nch << logWin
  int32_t ps[12];      // ascending row-bit positions spanned by a box
  int32_t segoff[16];  // row offset of box segment l (box index l << W)
  int32_t ngslot[8];   // box bit of the w-th lowest non-gate position
  int32_t boxmem[16];  // box bits of super-group member l
};

__device__ __forceinline__ int lds_slot(uint32_t box, int jv, int logJ) {
  const int pk = (int)(box << logJ) + jv;
  return pk + ((pk >> 4) << 1);  // 32 bytes of padding per 256 bytes: fewer bank conflicts
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R>
__device__ __forceinline__ void lds_put(float4 *lds, int slot, const Pk<R> &v) {
  Pk<R> tmp = v;
  lds[slot] = *reinterpret_cast<const float4 *>(&tmp);
}
template <typename R>
__device__ __forceinline__ Pk<R> lds_get(const float4 *lds, int slot) {
  const float4 x = lds[slot];
  return *reinterpret_cast<const Pk<R> *>(&x);
}

template <typename R, int VAR, bool APPLY, bool EXTRA>
__global__ __launch_bounds__(kLdsBlock) void k_bwd_step_lds(StepArgs<R> A, LdsGeom Lg) {
  constexpr int t = var_bits<VAR>();
  constexpr int NL = 1 << t;
  constexpr int NS = NL / 4;
  constexpr int V = Pk<R>::V;
  constexpr int kSlots = NL * 72;  // 64 packets per segment + padding
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double red[kLdsWaves][32];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float4 *lds = reinterpret_cast<float4 *>(lds_raw) + wv * kSlots;

  const int s = A.slot_to_start[blockIdx.y];
  const int P = gridDim.x;
  cx<R> ud[16];
  if (APPLY) {
    if (EXTRA)
      load_step_gate<R>(A.gR + (int64_t)s * A.gstride, A.k_apply, A.k_apply2, A.swap2, ud);
    else
      load_gate<R>(A.gR + (int64_t)s * A.gstride + A.k_apply * 16, ud, true);
  }
  const cx<R> *a_in = A.a_in + A.a_in_stride * s;
  cx<R> *a_out = A.a_out + A.a_out_stride * s;
  const cx<R> *b = A.b + A.b_stride * s;
  const int logC = A.geo.cg.logC, n = A.geo.cg.n;
  const int jv = lane & ((1 << Lg.logJ) - 1), rlow = lane >> Lg.logJ;
  uint32_t box_i = 0;
  for (int w = 0; w < Lg.W; ++w) box_i |= (uint32_t)((rlow >> w) & 1) << Lg.ngslot[w];

  cx<R> acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = cmake<R>(0, 0);

  for (uint32_t wi = blockIdx.x * kLdsWaves + wv; wi < Lg.witems; wi += P * kLdsWaves) {
    const uint32_t q = wi >> Lg.logWin, hi = wi & ((1u << Lg.logWin) - 1u);
    const uint32_t base_row = deposit(hi, Lg.ps, Lg.nps);
    const int64_t gbase = ((int64_t)q << (n + logC)) + ((int64_t)(base_row + rlow) << logC) + jv * V;
    // the box of a: one contiguous 1 KB read per segment, into this wave's LDS slice
#pragma unroll
    for (int l = 0; l < NL; ++l)
      lds_put<R>(lds, lds_slot(((uint32_t)l << Lg.W) + rlow, jv, Lg.logJ),
                 ld_pk(a_in + gbase + ((int64_t)Lg.segoff[l] << logC)));
    wave_sync();
    Pk<R> a[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) a[l] = lds_get<R>(lds, lds_slot(box_i + Lg.boxmem[l], jv, Lg.logJ));
    if (APPLY) {
#pragma unroll
      for (int rho = 0; rho < NS; ++rho) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          cx<R> x[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) x[p] = a[p * NS + rho].v[e];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            cx<R> y = cmake<R>(0, 0);
#pragma unroll
            for (int p = 0; p < 4; ++p) cfma(y, ud[qq * 4 + p], x[p]);
            a[qq * NS + rho].v[e] = y;
          }
        }
      }
      wave_sync();
#pragma unroll
      for (int l = 0; l < NL; ++l) lds_put<R>(lds, lds_slot(box_i + Lg.boxmem[l], jv, Lg.logJ), a[l]);
      wave_sync();
#pragma unroll
      for (int l = 0; l < NL; ++l)
        st_pk(a_out + gbase + ((int64_t)Lg.segoff[l] << logC),
              lds_get<R>(lds, lds_slot(((uint32_t)l << Lg.W) + rlow, jv, Lg.logJ)));
    }
    wave_sync();
    // the box of B_k, same way (all NL loads issued before the first LDS write, so they
    // share one memory round trip)
    {
      Pk<R> bl[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) bl[l] = ld_pk(b + gbase + ((int64_t)Lg.segoff[l] << logC));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int l = 0; l < NL; ++l) lds_put<R>(lds, lds_slot(((uint32_t)l << Lg.W) + rlow, jv, Lg.logJ), bl[l]);
    }
    wave_sync();
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
      Pk<R> bb[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        bb[p] = lds_get<R>(lds, lds_slot(box_i + Lg.boxmem[env_index<VAR>(p, sg)], jv, Lg.logJ));
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const Pk<R> &aq = a[env_index<VAR>(qq, sg)];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int e = 0; e < V; ++e) cfma_conj(acc[qq * 4 + p], aq.v[e], bb[p].v[e]);
      }
    }
    wave_sync();
  }

  const R ws = wave_sum_env<R>(acc);
  if ((lane & 1) == 0) red[wv][lane >> 1] = (double)ws;
  __syncthreads();
  if (threadIdx.x < 16) {
    const int e = threadIdx.x;
    c128 sum = cmake(red[0][2 * e], red[0][2 * e + 1]);
    for (int w = 1; w < kLdsWaves; ++w) sum = sum + cmake(red[w][2 * e], red[w][2 * e + 1]);
    A.partials[((int64_t)s * kPcap + blockIdx.x) * 16 + threadIdx.x] = sum;
  }
}

// Per start: fixed-order FP64 sum of the P block partials of the environment (256
// threads: thread 16 g + e sums entry e over blocks g, g + 16, ... with four independent
// accumulators, so many loads are in flight; the 16 group sums are then added in group
// order), then the gate update u <- polar((1 - beta) Gamma + beta u) on the first wave
// (one-qubit gates: polar2_update on one thread).
constexpr int kFinBlock = 256;

__global__ __launch_bounds__(kFinBlock) void k_env_finalize(const c128 *partials, int P,
                                                            const int32_t *slot_to_start,
                                                            c128 *gamma_out, int do_update,
                                                            double beta, c128 *g64, c64 *g32,
                                                            int32_t gstride, int32_t k_env,
                                                            c128 *vstore, int kind) {
  __shared__ c128 gsum[kFinBlock / 16][16];
  __shared__ c128 gam[16];
  __shared__ c128 pg[16], pv[16];
  __shared__ double psig[4];
  const int s = slot_to_start[blockIdx.x];
  const int e = threadIdx.x & 15, grp = threadIdx.x >> 4;
  constexpr int G = kFinBlock / 16;
  const c128 *src = partials + (int64_t)s * kPcap * 16 + e;
  c128 acc[4] = {cmake(0.0, 0.0), cmake(0.0, 0.0), cmake(0.0, 0.0), cmake(0.0, 0.0)};
  int blk = grp;
  for (; blk + 3 * G < P; blk += 4 * G) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = acc[u] + src[(int64_t)(blk + u * G) * 16];
  }
  if (blk < P) acc[0] = acc[0] + src[(int64_t)blk * 16];
  if (blk + G < P) acc[1] = acc[1] + src[(int64_t)(blk + G) * 16];
  if (blk + 2 * G < P) acc[2] = acc[2] + src[(int64_t)(blk + 2 * G) * 16];
  gsum[grp][e] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (threadIdx.x < 16) {
    c128 tot = gsum[0][e];
    for (int g = 1; g < G; ++g) tot = tot + gsum[g][e];
    gam[e] = tot;
    if (gamma_out) gamma_out[(int64_t)s * 16 + e] = tot;
  }
  __syncthreads();
  if (do_update && threadIdx.x < 64) {
    c128 *u64 = g64 + (int64_t)s * gstride + k_env * 16;
    c64 *u32 = g32 ? g32 + (int64_t)s * gstride + k_env * 16 : nullptr;
    if (kind == QFS_GATE_1Q) {
      if (threadIdx.x == 0) polar2_update<float>(gam, beta, u64, u32);
      return;
    }
    c128 *vs = vstore ? vstore + (int64_t)s * gstride + k_env * 16 : nullptr;
    polar4_wave(gam, beta, u64, u64, u32, pg, pv, psig, vs);
  }
}

// ------------------------------------------------------------------ apply + distance
template <typename R>
struct DistArgs {
  const cx<R> *x;
  int64_t x_stride;
  const cx<R> *ref;
  int64_t ref_stride;
  const cx<R> *gR;
  int32_t gstride;
  int32_t k;        // gate to apply (< 0: none)
  int32_t dagger;
  int32_t pa, pb;
  ChunkGeom cg;
  double *partials;  // [S][P]
  const int32_t *slot_to_start;
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_apply_dist(DistArgs<R> A) {
  __shared__ double red[kWaves];
  const int s = A.slot_to_start[blockIdx.y];
  const int P = gridDim.x;
  cx<R> u[16];
  const bool has_gate = A.k >= 0;
  if (has_gate) load_gate<R>(A.gR + (int64_t)s * A.gstride + A.k * 16, u, A.dagger != 0);
  const cx<R> *x = A.x + A.x_stride * s;
  const cx<R> *ref = A.ref + A.ref_stride * s;
  const int lo = min(A.pa, A.pb), hi = max(A.pa, A.pb);
  const int sorted[2] = {lo, hi};
  const uint32_t ma = 1u << A.pa, mb = 1u << A.pb;
  constexpr int V = Pk<R>::V;
  const int logC = A.cg.logC, n = A.cg.n;
  double acc = 0.0;
  for (uint32_t it = blockIdx.x * kBlock + threadIdx.x; it < A.cg.items; it += P * kBlock) {
    uint32_t q, rr, jv;
    split_item(it, A.cg, q, rr, jv);
    const uint32_t i0 = deposit(rr, sorted, 2);
    const int64_t base = ((int64_t)q << (n + logC)) + jv * V;
    int64_t o[4];
    o[0] = base + ((int64_t)i0 << logC);
    o[1] = base + ((int64_t)(i0 + mb) << logC);
    o[2] = base + ((int64_t)(i0 + ma) << logC);
    o[3] = base + ((int64_t)(i0 + ma + mb) << logC);
    Pk<R> xv[4], rv[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      xv[p] = ld_pk(x + o[p]);
      rv[p] = ld_pk(ref + o[p]);
    }
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        cx<R> y;
        if (has_gate) {
          y = cmake<R>(0, 0);
#pragma unroll
          for (int p = 0; p < 4; ++p) cfma(y, u[qq * 4 + p], xv[p].v[e]);
        } else {
          y = xv[qq].v[e];
        }
        const R dr = y.re - rv[qq].v[e].re, di = y.im - rv[qq].v[e].im;
        acc += (double)dr * (double)dr + (double)di * (double)di;
      }
  }
  acc = wave_sum<double>(acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = red[0];
    for (int w = 1; w < kWaves; ++w) sum += red[w];
    A.partials[(int64_t)s * P + blockIdx.x] = sum;
  }
}

// Per start (one wave): fixed-order sum of the P block partials, divided by M.
__global__ __launch_bounds__(64) void k_dist_finalize(const double *partials, int P, int stride,
                                                      const int32_t *slot_to_start, double inv_m,
                                                      double *out) {
  const int s = slot_to_start[blockIdx.x];
  double sum = 0.0;
  for (int blk = threadIdx.x; blk < P; blk += 64) sum += partials[(int64_t)s * stride + blk];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_down(sum, o);
  if (threadIdx.x == 0) out[s] = sum * inv_m;
}

__global__ void k_polar_batch(int count, const c128 *gamma, double beta, c128 *u) {
  __shared__ c128 pg[16], pv[16];
  __shared__ double psig[4];
  const int i = blockIdx.x;
  if (i >= count) return;
  polar4_wave(gamma + (int64_t)i * 16, beta, u + (int64_t)i * 16, u + (int64_t)i * 16, nullptr,
              pg, pv, psig);
}

__global__ void k_identity4(int64_t count, c128 *v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count * 16;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(e & 15);
    v[e] = cmake(((q >> 2) == (q & 3)) ? 1.0 : 0.0, 0.0);
  }
}

// Pack FP64 masters [N][ld] (row-major, states as columns) into the chunked working
// layout in R, zero beyond column M.
template <typename R>
__global__ void k_pack(int n, int logC, int64_t ld, int M, int64_t total, const c128 *src,
                       cx<R> *dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e >> (n + logC);
    const int64_t rem = e & ((int64_t(1) << (n + logC)) - 1);
    const int64_t i = rem >> logC, j = (q << logC) + (rem & ((1 << logC) - 1));
    c128 v = cmake(0.0, 0.0);
    if (j < M) v = src[i * ld + j];
    dst[e] = cmake<R>((R)v.re, (R)v.im);
  }
}

}  // namespace

// ------------------------------------------------------------------ host launchers
static int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

bool forward_fusable(int n, size_t rbytes, size_t lds_max) {
  return forward_lds_bytes(n, 1, rbytes) <= std::min<size_t>(lds_max, 128 * 1024);
}

int choose_log_chunk(int n, int M, size_t rbytes, bool fused, int starts, size_t lds_max) {
  const int pm = std::max(1, ilog2(std::max(M, 2)));
  if (!fused) return std::min(pm, 5);
  const size_t lim = std::min<size_t>(lds_max, 128 * 1024);
  int logC = 1;
  while (logC + 1 <= pm && forward_lds_bytes(n, logC + 1, rbytes) <= lim) ++logC;
  // keep at least ~two blocks per compute unit in the forward pass
  while (logC > 1 && (int64_t)((M + (1 << logC) - 1) >> logC) * starts < 512) --logC;
  return logC;
}

static ChunkGeom chunk_geom(const Geometry &g, int t, size_t rbytes) {
  ChunkGeom cg;
  const int logV = rbytes == 4 ? 1 : 0;
  cg.n = g.n;
  cg.logC = g.logC;
  cg.logJ = g.logC - logV;
  cg.logG = g.n - t;
  cg.items = (uint32_t)((uint64_t)g.nch << (cg.logG + cg.logJ));
  return cg;
}

static int blocks_for(uint32_t items, int nslots) {
  const int64_t pmax = std::max<int64_t>(1, ((int64_t)items + kBlock - 1) / kBlock);
  return (int)std::min<int64_t>(pmax, std::max(1, 2048 / std::max(1, nslots)));
}

template <typename R>
int launch_apply(const Geometry &g, int qa, int qb, int k, bool dagger, GateRef gates,
                 SBuf<R> src, SBuf<R> dst, const int32_t *slot_to_start, int nslots,
                 hipStream_t s) {
  if (nslots <= 0) return QFS_OK;
  ApplySeg<R> seg;
  seg.src = src.base;
  seg.src_stride = src.stride;
  seg.dst = dst.base;
  seg.dst_stride = dst.stride;
  seg.cg = chunk_geom(g, 2, sizeof(R));
  const int P = blocks_for(seg.cg.items, nslots);
  const int pa = g.n - 1 - qa, pb = g.n - 1 - qb;
  hipLaunchKernelGGL(k_apply<R>, dim3(P, nslots, 1), dim3(kBlock), 0, s, seg, pa, pb,
                     static_cast<const cx<R> *>(gates.gR), gates.gstride, k, dagger ? 1 : 0,
                     slot_to_start);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

size_t forward_lds_bytes(int n, int logC, size_t rbytes) {
  return (size_t(1) << (n + logC)) * 2 * rbytes;
}

template <typename R>
int launch_forward_fused(const Geometry &g, const Geometry *gv, const int32_t *pairs_dev, int L,
                         GateRef gates, const cx<R> *psi, cx<R> *blist, int64_t bstride,
                         const cx<R> *phi_ref, double *c0_partials, const cx<R> *psiv,
                         const cx<R> *phiv, double *val_partials, const int32_t *slot_to_start,
                         int nslots, const int32_t *kinds_dev, hipStream_t s,
                         const int32_t *bneed_dev) {
  if (nslots <= 0) return QFS_OK;
  FwdSeg<R> a{}, b{};
  a.src = psi;
  a.blist = blist;
  a.bstride = bstride;
  a.sN = (int64_t)g.nch * ((int64_t)g.N << g.logC);
  a.ref = phi_ref;
  a.partials = c0_partials;
  a.nch = g.nch;
  a.kstore = L - 1;
  a.kapply = phi_ref ? L : L - 1;
  int nz = 1;
  if (gv) {
    if (gv->logC != g.logC) {
      set_error_detail("fused forward: training and validation chunk widths differ");
      return QFS_EINVAL;
    }
    b.src = psiv;
    b.blist = nullptr;
    b.bstride = 0;
    b.sN = 0;
    b.ref = phiv;
    b.partials = val_partials;
    b.nch = gv->nch;
    b.kstore = 0;
    b.kapply = L;
    nz = 2;
  }
  const int gx = std::max(a.nch, gv ? b.nch : 0);
  const size_t lds = forward_lds_bytes(g.n, g.logC, sizeof(R));
  static const int coalesce_b = [] {
    const char *e = std::getenv("QFS_FWD_COALESCE");  // 0: always store from registers
    return e ? std::atoi(e) : 1;
  }();
  static const int fwd_env = [] {
    const char *e = std::getenv("QFS_FWD_THREADS");  // work-group size: 512 or 1024 (0: by size)
    return e ? std::atoi(e) : 0;
  }();
  // 1024 threads once every thread has at least two gate groups per gate, else 512
  const int64_t groups = int64_t(1) << (g.n - 2 + g.logC - (sizeof(R) == 4 ? 1 : 0));
  const int fwd_threads = fwd_env == 512 || fwd_env == 1024 ? fwd_env : (groups >= 2048 ? 1024 : 512);
  auto go = [&](auto kernel, int threads) -> int {
    // dynamic LDS above 64 KB must be requested per kernel (one entry per block size:
    // both sizes share this lambda's instantiation)
    static size_t attr_bytes[2] = {0, 0};
    size_t &ab = attr_bytes[threads == 1024 ? 1 : 0];
    QFS_TRY(ensure_dynamic_lds(reinterpret_cast<const void *>(kernel), lds, &ab));
    hipLaunchKernelGGL(kernel, dim3(gx * nz, nslots, 1), dim3(threads), lds, s, a, b, nz, g.n, g.logC, pairs_dev,
                       static_cast<const cx<R> *>(gates.gR), gates.gstride, slot_to_start, coalesce_b,
                       kinds_dev, bneed_dev);
    QFS_HIP(hipGetLastError());
    return QFS_OK;
  };
  if (fwd_threads == 1024) return go(k_forward_fused<R, 1024>, 1024);
  return go(k_forward_fused<R, 512>, 512);
}

template <typename R>
int launch_pack(const Geometry &g, int64_t ld, const c128 *master, cx<R> *dst, hipStream_t s) {
  const int64_t total = (int64_t)g.nch * ((int64_t)g.N << g.logC);
  hipLaunchKernelGGL(k_pack<R>, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)),
                     dim3(256), 0, s, g.n, g.logC, ld, g.M, total, master, dst);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// Canonical bit order for a backward step and its variant id (see env_index).
static int classify_step(const int32_t *pairs, int k_apply, int k_env, int32_t tq[4], int *t) {
  const int a0 = pairs[2 * k_env], b0 = pairs[2 * k_env + 1];
  if (k_apply < 0) {
    tq[0] = a0;
    tq[1] = b0;
    *t = 2;
    return 0;
  }
  const int a1 = pairs[2 * k_apply], b1 = pairs[2 * k_apply + 1];
  tq[0] = a1;
  tq[1] = b1;
  if (a0 == a1 && b0 == b1) {
    *t = 2;
    return 0;
  }
  if (a0 == b1 && b0 == a1) {
    *t = 2;
    return 1;
  }
  *t = 3;
  if (a0 == a1) { tq[2] = b0; return 2; }
  if (a0 == b1) { tq[2] = b0; return 3; }
  if (b0 == a1) { tq[2] = a0; return 4; }
  if (b0 == b1) { tq[2] = a0; return 5; }
  *t = 4;
  tq[2] = a0;
  tq[3] = b0;
  return 6;
}

template <typename R, int VAR, bool APPLY, bool EXTRA>
static void launch_step_kernel(dim3 grid, const StepArgs<R> &a, const LdsGeom *lg, hipStream_t s) {
  if (lg) {
    const size_t lds = (size_t)kLdsWaves * (1 << var_bits<VAR>()) * 72 * 16;
    hipLaunchKernelGGL((k_bwd_step_lds<R, VAR, APPLY, EXTRA>), grid, dim3(kLdsBlock), lds, s, a, *lg);
  } else {
    hipLaunchKernelGGL((k_bwd_step<R, VAR, APPLY, EXTRA>), grid, dim3(kBlock), 0, s, a);
  }
}

template <typename R, bool EXTRA>
static void launch_step_var(int var, bool apply, dim3 grid, const StepArgs<R> &a, const LdsGeom *lg,
                            hipStream_t s) {
  if (!apply) {
    launch_step_kernel<R, 0, false, EXTRA>(grid, a, lg, s);
    return;
  }
  switch (var) {
    case 0: launch_step_kernel<R, 0, true, EXTRA>(grid, a, lg, s); break;
    case 1: launch_step_kernel<R, 1, true, EXTRA>(grid, a, lg, s); break;
    case 2: launch_step_kernel<R, 2, true, EXTRA>(grid, a, lg, s); break;
    case 3: launch_step_kernel<R, 3, true, EXTRA>(grid, a, lg, s); break;
    case 4: launch_step_kernel<R, 4, true, EXTRA>(grid, a, lg, s); break;
    case 5: launch_step_kernel<R, 5, true, EXTRA>(grid, a, lg, s); break;
    default: launch_step_kernel<R, 6, true, EXTRA>(grid, a, lg, s); break;
  }
}

// Box geometry of the LDS-staged step, or false when the plain step already reads whole
// cache lines (lowest gate bit high enough) or the state is too small for a box.
static bool lds_geometry(const Geometry &g, const StepGeom &G, const int32_t *pos, size_t rbytes,
                         LdsGeom *L) {
  static const int mode = [] {
    const char *e = std::getenv("QFS_BWD_LDS");  // 0: never, 1: auto (default), 2: always
    return e ? std::atoi(e) : 1;
  }();
  if (mode == 0) return false;
  const int t = G.t;
  const int logJ = G.cg.logJ;
  const int W = 6 - logJ;
  if (W < 1 || g.n - t < W) return false;
  const size_t row_bytes = (size_t(1) << g.logC) * rbytes * 2;
  if (mode == 1 && (row_bytes << G.sorted_pos[0]) >= 128) return false;
  std::memset(L, 0, sizeof(*L));
  L->W = W;
  L->logJ = logJ;
  L->nps = W + t;
  L->logWin = g.n - t - W;
  L->witems = (uint32_t)((uint64_t)g.nch << L->logWin);
  // box positions: the gate bits and the W lowest other bits, ascending
  int ng[32], nng = 0;
  for (int p = 0; p < g.n && nng < W; ++p) {
    bool gate = false;
    for (int m = 0; m < t; ++m) gate |= G.sorted_pos[m] == p;
    if (!gate) ng[nng++] = p;
  }
  int all[12], na = 0;
  for (int m = 0; m < t; ++m) all[na++] = G.sorted_pos[m];
  for (int w = 0; w < W; ++w) all[na++] = ng[w];
  std::sort(all, all + na);
  for (int i = 0; i < na; ++i) L->ps[i] = all[i];
  auto slot_of = [&](int pos) {
    for (int i = 0; i < na; ++i)
      if (all[i] == pos) return i;
    return -1;
  };
  for (int l = 0; l < (1 << t); ++l) {
    int32_t off = 0;
    for (int b = 0; b < t; ++b)
      if ((l >> b) & 1) off += 1 << all[W + b];
    L->segoff[l] = off;
  }
  for (int w = 0; w < W; ++w) L->ngslot[w] = slot_of(ng[w]);
  for (int l = 0; l < (1 << t); ++l) {
    int32_t bx = 0;
    for (int m = 0; m < t; ++m)
      if ((l >> (t - 1 - m)) & 1) bx |= 1 << slot_of(pos[m]);
    L->boxmem[l] = bx;
  }
  return true;
}

template <typename R>
int launch_bwd_step(const Geometry &g, const int32_t *pairs_host, int k_apply, int k_env,
                    GateRef gates, SBuf<R> a_in, SBuf<R> a_out, SBuf<R> b,
                    const int32_t *slot_to_start, int nslots, c128 *partials, int *P_out,
                    hipStream_t s, int k_apply2) {
  if (nslots <= 0) return QFS_OK;
  int swap2 = 0;
  if (k_apply2 >= 0) {
    const int a0 = pairs_host[2 * k_apply], a1 = pairs_host[2 * k_apply + 1];
    const int b0 = pairs_host[2 * k_apply2], b1 = pairs_host[2 * k_apply2 + 1];
    if (k_apply < 0 || !((a0 == b0 && a1 == b1) || (a0 == b1 && a1 == b0))) {
      set_error_detail("backward step: the folded gate must act on the same two qubits");
      return QFS_EINVAL;
    }
    swap2 = a0 == b1 ? 1 : 0;
  }
  int32_t tq[4];
  int t = 0;
  const int var = classify_step(pairs_host, k_apply, k_env, tq, &t);
  StepArgs<R> a;
  a.a_in = a_in.base;
  a.a_in_stride = a_in.stride;
  a.a_out = a_out.base;
  a.a_out_stride = a_out.stride;
  a.b = b.base;
  a.b_stride = b.stride;
  a.gR = static_cast<const cx<R> *>(gates.gR);
  a.gstride = gates.gstride;
  a.k_apply = k_apply;
  a.k_apply2 = k_apply2;
  a.swap2 = swap2;
  a.partials = partials;
  a.slot_to_start = slot_to_start;
  StepGeom &G = a.geo;
  G.cg = chunk_geom(g, t, sizeof(R));
  G.t = t;
  int32_t pos[4];
  for (int m = 0; m < t; ++m) pos[m] = g.n - 1 - tq[m];
  for (int m = 0; m < 4; ++m) G.sorted_pos[m] = 0;
  for (int m = 0; m < t; ++m) G.sorted_pos[m] = pos[m];
  std::sort(G.sorted_pos, G.sorted_pos + t);
  for (int l = 0; l < 16; ++l) {
    int32_t o = 0;
    if (l < (1 << t))
      for (int m = 0; m < t; ++m)
        if ((l >> (t - 1 - m)) & 1) o += 1 << pos[m];
    G.off[l] = o;
  }
  LdsGeom lg;
  const bool use_lds = lds_geometry(g, G, pos, sizeof(R), &lg);
  const LdsGeom *lgp = use_lds ? &lg : nullptr;
  int P;
  if (use_lds) {
    const int64_t pmax = std::max<int64_t>(1, ((int64_t)lg.witems + kLdsWaves - 1) / kLdsWaves);
    P = (int)std::min<int64_t>(pmax, std::max(1, 4096 / std::max(1, nslots)));
  } else {
    P = blocks_for(G.cg.items, nslots);
  }
  *P_out = P;
  dim3 grid(P, nslots);
  if (k_apply2 >= 0)
    launch_step_var<R, true>(var, k_apply >= 0, grid, a, lgp, s);
  else
    launch_step_var<R, false>(var, k_apply >= 0, grid, a, lgp, s);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_env_finalize(int P, const c128 *partials, const int32_t *slot_to_start, int nslots,
                        c128 *gamma_out, bool do_update, double beta, c128 *g64, c64 *g32,
                        int32_t gstride, int32_t k_env, c128 *vstore, int kind, hipStream_t s) {
  if (nslots <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_env_finalize, dim3(nslots), dim3(kFinBlock), 0, s, partials, P, slot_to_start,
                     gamma_out, do_update ? 1 : 0, beta, g64, g32, gstride, k_env, vstore, kind);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

template <typename R>
int launch_apply_dist(const Geometry &g, int qa, int qb, int k, bool dagger, GateRef gates,
                      SBuf<R> x, SBuf<R> ref, const int32_t *slot_to_start, int nslots,
                      double *partials, int *P_out, hipStream_t s) {
  if (nslots <= 0) return QFS_OK;
  DistArgs<R> a;
  a.x = x.base;
  a.x_stride = x.stride;
  a.ref = ref.base;
  a.ref_stride = ref.stride;
  a.gR = static_cast<const cx<R> *>(gates.gR);
  a.gstride = gates.gstride;
  a.k = k;
  a.dagger = dagger ? 1 : 0;
  a.pa = g.n - 1 - qa;
  a.pb = g.n - 1 - qb;
  a.cg = chunk_geom(g, 2, sizeof(R));
  a.partials = partials;
  a.slot_to_start = slot_to_start;
  const int P = blocks_for(a.cg.items, nslots);
  *P_out = P;
  hipLaunchKernelGGL(k_apply_dist<R>, dim3(P, nslots), dim3(kBlock), 0, s, a);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_dist_finalize(int P, const double *partials, const int32_t *slot_to_start, int nslots,
                         int M, double *out, hipStream_t s, int stride) {
  if (nslots <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_dist_finalize, dim3(nslots), dim3(64), 0, s, partials, P, stride > 0 ? stride : P,
                     slot_to_start, 1.0 / (double)M, out);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_identity4(int64_t count, c128 *v, hipStream_t s) {
  if (count <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_identity4, dim3((unsigned)std::min<int64_t>((count * 16 + 255) / 256, 65536)),
                     dim3(256), 0, s, count, v);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int launch_polar_batch(int count, const c128 *gamma, double beta, c128 *u, hipStream_t s) {
  if (count <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_polar_batch, dim3(count), dim3(64), 0, s, count, gamma, beta, u);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

#define QFS_INST(R)                                                                          \
  template int launch_apply<R>(const Geometry &, int, int, int, bool, GateRef, SBuf<R>,       \
                               SBuf<R>, const int32_t *, int, hipStream_t);                   \
  template int launch_bwd_step<R>(const Geometry &, const int32_t *, int, int, GateRef,       \
                                  SBuf<R>, SBuf<R>, SBuf<R>, const int32_t *, int, c128 *,    \
                                  int *, hipStream_t, int);                                  \
  template int launch_apply_dist<R>(const Geometry &, int, int, int, bool, GateRef, SBuf<R>,  \
                                    SBuf<R>, const int32_t *, int, double *, int *,           \
                                    hipStream_t);                                            \
  template int launch_forward_fused<R>(const Geometry &, const Geometry *, const int32_t *,   \
                                       int, GateRef, const cx<R> *, cx<R> *, int64_t,         \
                                       const cx<R> *, double *, const cx<R> *, const cx<R> *, \
                                       double *, const int32_t *, int, const int32_t *,       \
                                       hipStream_t, const int32_t *);                         \
  template int launch_pack<R>(const Geometry &, int64_t, const c128 *, cx<R> *, hipStream_t);
QFS_INST(float)
QFS_INST(double)
#undef QFS_INST

}  // namespace qfs
