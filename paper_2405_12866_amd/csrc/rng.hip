// The method's own random draws on the device (training and validation states,
// initial gates), from the generator in philox.h.
#include "philox.h"

namespace qfs {

// Ginibre columns [col0, col1) of a rows-row matrix into the amplitude-major layout:
// A[i * ld + j] = z(index j * rows + i).
__global__ void k_ginibre(int64_t rows, int64_t col0, int64_t ncols, int64_t ld, uint64_t seed,
                          uint32_t role, uint32_t stream, c128 *A) {
  const int64_t total = rows * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ncols;
    const int64_t j = col0 + (e - i * ncols);
    A[i * ld + j] = complex_normal(seed, role, stream, (uint64_t)(j * rows + i));
  }
}

int launch_ginibre(int64_t rows, int64_t col0, int64_t col1, int64_t ld, uint64_t seed,
                   uint32_t role, uint32_t stream, c128 *A, hipStream_t s) {
  const int64_t total = rows * (col1 - col0);
  if (total <= 0) return QFS_OK;
  const int threads = 256;
  const int64_t blocks = std::min<int64_t>((total + threads - 1) / threads, 65536);
  hipLaunchKernelGGL(k_ginibre, dim3((unsigned)blocks), dim3(threads), 0, s, rows, col0,
                     col1 - col0, ld, seed, role, stream, A);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// Haar 4x4 per (start, gate): 4x4 Ginibre block (index 16*gate + 4*col + row, role 3,
// stream = start), orthonormalised column by column with positive diag(R); one thread
// per gate, written row-major u[q][p] = Q[q][p].
__global__ void k_haar_gates(uint64_t seed, int32_t start0, int32_t starts, int32_t L,
                             c128 *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)starts * L) return;
  const int32_t s = (int32_t)(t / L), k = (int32_t)(t - (int64_t)s * L);
  c128 q[4][4];  // [col][row]
  for (int c = 0; c < 4; ++c)
    for (int r = 0; r < 4; ++r)
      q[c][r] = complex_normal(seed, 3u, (uint32_t)(start0 + s), (uint64_t)k * 16u + 4u * c + r);
  for (int c = 0; c < 4; ++c) {
    for (int rep = 0; rep < 2; ++rep)
      for (int o = 0; o < c; ++o) {
        c128 d = cmake(0.0, 0.0);
        for (int r = 0; r < 4; ++r) cfma(d, cconj(q[o][r]), q[c][r]);
        for (int r = 0; r < 4; ++r) q[c][r] = q[c][r] - d * q[o][r];
      }
    double nrm = 0.0;
    for (int r = 0; r < 4; ++r) nrm += cabs2(q[c][r]);
    const double inv = 1.0 / sqrt(nrm);
    for (int r = 0; r < 4; ++r) q[c][r] = cscale(q[c][r], inv);
  }
  c128 *u = out + (int64_t)t * 16;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) u[r * 4 + c] = q[c][r];
}

int launch_haar_gates(uint64_t seed, int32_t start0, int32_t starts, int32_t L, c128 *out,
                      hipStream_t s) {
  const int64_t total = (int64_t)starts * L;
  if (total <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_haar_gates, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s,
                     seed, start0, starts, L, out);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// Gate kinds after the 4x4 draw (or copy) of every slot: a one-qubit gate of a drawn
// start becomes v (x) I_2 with v Haar on U(2) from the 2x2 Ginibre block at indices
// 16*gate + 2*col + row of the same stream (a copied one is projected onto that form);
// a constant gate is copied from fixed[gate].
// One thread per (start, gate).
__global__ void k_kind_gates(uint64_t seed, int32_t start0, int32_t starts, int32_t L,
                             const int32_t *kinds, const c128 *fixed, int32_t drawn, c128 *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)starts * L) return;
  const int32_t s = (int32_t)(t / L), k = (int32_t)(t - (int64_t)s * L);
  const int kind = kinds[k];
  c128 *u = out + t * 16;
  if (kind == QFS_GATE_FIXED) {
    for (int e = 0; e < 16; ++e) u[e] = fixed[(int64_t)k * 16 + e];
    return;
  }
  if (kind != QFS_GATE_1Q) return;
  if (!drawn) {
    // a supplied one-qubit slot (checked to be within 1e-10 of v (x) I_2) is made exactly
    // v (x) I_2, v from its entries (2i, 2j), so every kernel may rely on that form
    c128 v[4];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) v[i * 2 + j] = u[(2 * i) * 4 + 2 * j];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) u[r * 4 + c] = ((r & 1) == (c & 1)) ? v[(r >> 1) * 2 + (c >> 1)] : cmake(0.0, 0.0);
    return;
  }
  c128 q[2][2];  // [col][row]
  for (int c = 0; c < 2; ++c)
    for (int r = 0; r < 2; ++r)
      q[c][r] = complex_normal(seed, 3u, (uint32_t)(start0 + s), (uint64_t)k * 16u + 2u * c + r);
  for (int c = 0; c < 2; ++c) {
    for (int rep = 0; rep < 2; ++rep)
      for (int o = 0; o < c; ++o) {
        const c128 d = cconj(q[o][0]) * q[c][0] + cconj(q[o][1]) * q[c][1];
        for (int r = 0; r < 2; ++r) q[c][r] = q[c][r] - d * q[o][r];
      }
    const double inv = 1.0 / sqrt(cabs2(q[c][0]) + cabs2(q[c][1]));
    for (int r = 0; r < 2; ++r) q[c][r] = cscale(q[c][r], inv);
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      u[r * 4 + c] = ((r & 1) == (c & 1)) ? q[c >> 1][r >> 1] : cmake(0.0, 0.0);
}

int launch_kind_gates(uint64_t seed, int32_t start0, int32_t starts, int32_t L,
                      const int32_t *kinds, const c128 *fixed, bool drawn, c128 *out,
                      hipStream_t s) {
  const int64_t total = (int64_t)starts * L;
  if (total <= 0 || !kinds) return QFS_OK;
  hipLaunchKernelGGL(k_kind_gates, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s,
                     seed, start0, starts, L, kinds, fixed, drawn ? 1 : 0, out);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

}  // namespace qfs
