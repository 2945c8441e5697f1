// Complex FP64 dense linear algebra for the sample draw (CholeskyQR2 with block
// Gram-Schmidt projection) and the dense-target product, plus layout conversions.
#include <algorithm>

#include "qfs_internal.h"

namespace qfs {

// ------------------------------------------------------------------ ZGEMM
// 32x32 output tile per 256-thread block, K tiles of 16 staged in LDS; each thread
// owns a 2x2 sub-tile at rows ty, ty+16 and columns tx, tx+16.
template <bool CT>
__global__ __launch_bounds__(256) void k_zgemm(int m, int n, int k, c128 alpha, const c128 *A,
                                               int lda, const c128 *B, int ldb, c128 beta,
                                               c128 *C, int ldc) {
  __shared__ c128 As[16][33];
  __shared__ c128 Bs[16][33];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  c128 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = cmake(0.0, 0.0);
  for (int kb = 0; kb < k; kb += 16) {
    for (int e = tid; e < 512; e += 256) {
      int ii, kk;
      if (CT) {
        ii = e & 31;
        kk = e >> 5;
      } else {
        kk = e & 15;
        ii = e >> 4;
      }
      const int gi = i0 + ii, gk = kb + kk;
      c128 v = cmake(0.0, 0.0);
      if (gi < m && gk < k) v = CT ? cconj(A[(int64_t)gk * lda + gi]) : A[(int64_t)gi * lda + gk];
      As[kk][ii] = v;
    }
    for (int e = tid; e < 512; e += 256) {
      const int jj = e & 31, kk = e >> 5;
      const int gj = j0 + jj, gk = kb + kk;
      Bs[kk][jj] = (gk < k && gj < n) ? B[(int64_t)gk * ldb + gj] : cmake(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const c128 a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const c128 b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      cfma(acc[0][0], a0, b0);
      cfma(acc[0][1], a0, b1);
      cfma(acc[1][0], a1, b0);
      cfma(acc[1][1], a1, b1);
    }
    __syncthreads();
  }
  const bool read_c = !(beta.re == 0.0 && beta.im == 0.0);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int gi = i0 + ty + 16 * a, gj = j0 + tx + 16 * b;
      if (gi < m && gj < n) {
        c128 v = alpha * acc[a][b];
        if (read_c) v = v + beta * C[(int64_t)gi * ldc + gj];
        C[(int64_t)gi * ldc + gj] = v;
      }
    }
}

int launch_zgemm(bool conjtrans_a, int m, int n, int k, c128 alpha, const c128 *A, int lda,
                 const c128 *B, int ldb, c128 beta, c128 *C, int ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return QFS_OK;
  dim3 grid((n + 31) / 32, (m + 31) / 32);
  if (conjtrans_a)
    hipLaunchKernelGGL(k_zgemm<true>, grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  else
    hipLaunchKernelGGL(k_zgemm<false>, grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// C = A^H B for a short, wide product (m x n output, k >> m, n; the Gram matrices of
// the sample draw): the k range is split over up to kGramParts work-groups per output
// tile, each writing a partial tile to `work` [parts][m][n]; k_sum_parts adds them in
// part order.
__global__ __launch_bounds__(256) void k_zgemm_ct_part(int m, int n, int k, int kchunk,
                                                       const c128 *A, int lda, const c128 *B,
                                                       int ldb, c128 *work) {
  __shared__ c128 As[16][33];
  __shared__ c128 Bs[16][33];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32, part = blockIdx.z;
  const int k0 = part * kchunk, k1 = min(k, k0 + kchunk);
  c128 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = cmake(0.0, 0.0);
  for (int kb = k0; kb < k1; kb += 16) {
    for (int e = tid; e < 512; e += 256) {
      const int ii = e & 31, kk = e >> 5;
      const int gi = i0 + ii, gk = kb + kk;
      As[kk][ii] = (gi < m && gk < k1) ? cconj(A[(int64_t)gk * lda + gi]) : cmake(0.0, 0.0);
      const int gj = j0 + ii;
      Bs[kk][ii] = (gk < k1 && gj < n) ? B[(int64_t)gk * ldb + gj] : cmake(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const c128 a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const c128 b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      cfma(acc[0][0], a0, b0);
      cfma(acc[0][1], a0, b1);
      cfma(acc[1][0], a1, b0);
      cfma(acc[1][1], a1, b1);
    }
    __syncthreads();
  }
  c128 *W = work + (int64_t)part * m * n;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int gi = i0 + ty + 16 * a, gj = j0 + tx + 16 * b;
      if (gi < m && gj < n) W[(int64_t)gi * n + gj] = acc[a][b];
    }
}

__global__ void k_sum_parts(int64_t mn, int parts, const c128 *work, c128 *C) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= mn) return;
  c128 s = work[e];
  for (int p = 1; p < parts; ++p) s = s + work[(int64_t)p * mn + e];
  C[e] = s;
}

// k splits: enough work-groups to cover the chip (about 2048 with the m x m tiles),
// at most 16
static int gram_parts(int64_t m) {
  const int64_t tiles = ((m + 31) / 32) * ((m + 31) / 32);
  return (int)std::max<int64_t>(1, std::min<int64_t>(16, 2048 / std::max<int64_t>(1, tiles)));
}

static int gram_splitk(int m, int n, int k, const c128 *A, int lda, const c128 *B, int ldb, c128 *C,
                       c128 *work, hipStream_t s) {
  const int nparts = gram_parts(std::max(m, n));
  const int kchunk = ((k + nparts - 1) / nparts + 15) / 16 * 16;
  const int parts = (k + kchunk - 1) / kchunk;
  dim3 grid((n + 31) / 32, (m + 31) / 32, parts);
  hipLaunchKernelGGL(k_zgemm_ct_part, grid, dim3(256), 0, s, m, n, k, kchunk, A, lda, B, ldb, work);
  QFS_HIP(hipGetLastError());
  const int64_t mn = (int64_t)m * n;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, mn, parts, work, C);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// ------------------------------------------------------------------ Cholesky, R^-1
// In-place upper Cholesky G = R^H R of an m x m Hermitian positive-definite matrix
// (row-major, ld m), right-looking: R[j][j] = sqrt(G[j][j]), R[j][c] = G[j][c] / R[j][j],
// G[i][c] -= conj(R[j][i]) R[j][c] for i, c > j. flag[0] is set on a non-positive pivot.
// Blocked: rows [j, j + b) of the trailing matrix (the
// "row panel", b x w with w = m - j, in LDS) are factored by one work-group with the
// column steps above restricted to the panel; the rest of the trailing matrix is then
// updated with one GEMM, G[j+b:, j+b:] -= R[J, j+b:]^H R[J, j+b:]. Only the upper
// triangle is ever read; the strictly lower part is cleared at the end.
__global__ __launch_bounds__(1024) void k_chol_panel(int m, int j, int b, c128 *G, int *flag) {
  extern __shared__ c128 pan[];  // [b][w]
  __shared__ double inv_pivot;
  const int tid = threadIdx.x, nt = blockDim.x, w = m - j;
  for (int e = tid; e < b * w; e += nt) {
    const int r = e / w, c = e % w;
    pan[e] = G[(int64_t)(j + r) * m + j + c];
  }
  __syncthreads();
  for (int jj = 0; jj < b; ++jj) {
    if (tid == 0) {
      const double d = pan[jj * w + jj].re;
      if (!(d > 0.0)) {
        flag[0] = 1;
        inv_pivot = 0.0;
        pan[jj * w + jj] = cmake(1.0, 0.0);
      } else {
        const double r = sqrt(d);
        pan[jj * w + jj] = cmake(r, 0.0);
        inv_pivot = 1.0 / r;
      }
    }
    __syncthreads();
    const double ip = inv_pivot;
    for (int c = jj + 1 + tid; c < w; c += nt) pan[jj * w + c] = cscale(pan[jj * w + c], ip);
    __syncthreads();
    // rows jj+1 .. b-1 of the panel, columns from the row's diagonal on
    const int rows = b - jj - 1;
    for (int e = tid; e < rows * w; e += nt) {
      const int ii = jj + 1 + e / w, c = e % w;
      if (c < ii) continue;
      c128 v = pan[ii * w + c];
      cfma(v, cscale(cconj(pan[jj * w + ii]), -1.0), pan[jj * w + c]);
      pan[ii * w + c] = v;
    }
    __syncthreads();
  }
  for (int e = tid; e < b * w; e += nt) {
    const int r = e / w, c = e % w;
    G[(int64_t)(j + r) * m + j + c] = pan[e];
  }
}

__global__ void k_zero_lower(int m, c128 *G) {
  const int64_t total = (int64_t)m * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / m), c = (int)(e % m);
    if (c < i) G[e] = cmake(0.0, 0.0);
  }
}

static int cholesky_upper_blocked(int m, c128 *G, int *flag, hipStream_t s) {
  constexpr size_t kPanelLds = 144 * 1024;
  static size_t attr = 0;
  QFS_TRY(ensure_dynamic_lds(reinterpret_cast<const void *>(&k_chol_panel), kPanelLds, &attr));
  const c128 one = cmake(1.0, 0.0), mone = cmake(-1.0, 0.0);
  for (int j = 0; j < m;) {
    const int w = m - j;
    int b = (int)std::min<size_t>(32, kPanelLds / ((size_t)w * sizeof(c128)));
    b = std::max(1, std::min(b, w));
    hipLaunchKernelGGL(k_chol_panel, dim3(1), dim3(1024), sizeof(c128) * (size_t)b * w, s, m, j, b, G,
                       flag);
    QFS_HIP(hipGetLastError());
    const int rest = w - b;
    if (rest > 0) {
      const c128 *panel = G + (int64_t)j * m + j + b;
      QFS_TRY(launch_zgemm(true, rest, rest, b, mone, panel, m, panel, m, one,
                           G + (int64_t)(j + b) * m + j + b, m, s));
    }
    j += b;
  }
  hipLaunchKernelGGL(k_zero_lower, dim3((unsigned)std::min<int64_t>(((int64_t)m * m + 255) / 256, 4096)),
                     dim3(256), 0, s, m, G);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// T = R^-1 for upper-triangular R (m x m): one wave per column c of T, back
// substitution T[i][c] = -(sum_{k=i+1..c} R[i][k] T[k][c]) / R[i][i] with each dot
// product split over the 64 lanes and combined by a butterfly (every lane ends with
// the same sum); the column being built lives in LDS.
__global__ __launch_bounds__(64) void k_tri_inverse_upper(int m, const c128 *R, c128 *T) {
  extern __shared__ c128 tcol[];
  const int c = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < m; i += 64) tcol[i] = cmake(0.0, 0.0);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
  if (lane == 0) tcol[c] = cmake(1.0 / R[(int64_t)c * m + c].re, 0.0);
  __syncthreads();
  for (int i = c - 1; i >= 0; --i) {
    c128 acc = cmake(0.0, 0.0);
    for (int k = i + 1 + lane; k <= c; k += 64) cfma(acc, R[(int64_t)i * m + k], tcol[k]);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      acc.re += __shfl_xor(acc.re, o);
      acc.im += __shfl_xor(acc.im, o);
    }
    const double rii = R[(int64_t)i * m + i].re;
    if (lane == 0) tcol[i] = cscale(acc, -1.0 / rii);
    __syncthreads();
  }
  for (int i = lane; i < m; i += 64) T[(int64_t)i * m + c] = tcol[i];
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long v = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// T = R^-1 for m <= 64 NJ, one wave per row c of T: from T R = I,
//   T[c][k] = (delta_ck - sum_{c <= j < k} T[c][j] R[j][k]) / R[k][k],  k = c .. m - 1.
// Lane l keeps the running sums s_i of the rows i = l + 64 u of row c; at step k the lane
// holding k finishes T[c][k] (reciprocal diagonal taken beforehand), every lane reads it
// from that lane's registers, and the lanes add T[c][k] R[k][i] to s_i for i > k, reading
// row k of R (contiguous; four rows are loaded while the four before them are used). No
// reduction and no barrier per step, unlike the dot-product form above.
template <int NJ>
__global__ __launch_bounds__(64) void k_tri_inverse_rows(int m, const c128 *__restrict__ R,
                                                         c128 *__restrict__ T) {
  const int c = blockIdx.x, lane = threadIdx.x;
  c128 sv[NJ];
  double inv[NJ];
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int i = lane + 64 * u;
    sv[u] = cmake(0.0, 0.0);
    inv[u] = i < m ? 1.0 / R[(int64_t)i * m + i].re : 0.0;
  }
#pragma unroll
  for (int uk = 0; uk < NJ; ++uk) {
    const int ks = max(c, 64 * uk), k1 = min(m, 64 * uk + 64);
    if (ks >= k1) continue;
    c128 buf[4][NJ], nbuf[4][NJ];
    auto load4 = [&](int kb, c128 (&dst)[4][NJ]) __attribute__((always_inline)) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kb + q;
#pragma unroll
        for (int u = uk; u < NJ; ++u) {
          const int i = lane + 64 * u;
          dst[q][u] = (k < k1 && i > k && i < m) ? R[(int64_t)k * m + i] : cmake(0.0, 0.0);
        }
      }
    };
    load4(ks, buf);
    for (int kb = ks; kb < k1; kb += 4) {
      load4(kb + 4, nbuf);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kb + q;
        if (k < k1) {
          const int kl = k & 63;
          const double dre = (k == c ? 1.0 : 0.0) - sv[uk].re, dim = -sv[uk].im;
          const double tre = readlane_f64(dre * inv[uk], kl), tim = readlane_f64(dim * inv[uk], kl);
          if (lane == kl) sv[uk] = cmake(tre, tim);  // this slot now holds T[c][k]
#pragma unroll
          for (int u = uk; u < NJ; ++u) {
            const int i = lane + 64 * u;
            if (i > k) {
              const c128 r = buf[q][u];
              sv[u].re += tre * r.re - tim * r.im;
              sv[u].im += tre * r.im + tim * r.re;
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = uk; u < NJ; ++u) buf[q][u] = nbuf[q][u];
    }
  }
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int i = lane + 64 * u;
    if (i < m) T[(int64_t)c * m + i] = i < c ? cmake(0.0, 0.0) : sv[u];
  }
}

__global__ void k_copy_cols(int64_t rows, int cols, const c128 *src, int lds, c128 *dst, int ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols;
    const int j = (int)(e - i * cols);
    dst[i * ldd + j] = src[i * lds + j];
  }
}

size_t work_bytes_orth(int64_t rows, int64_t cols) {
  const size_t m = (size_t)cols;
  // gram_parts(x) x^2 over x <= m is at most max(min(16 m^2, 2^21), m^2)
  const size_t parts = std::max(std::min(16 * m * m, size_t(1) << 21), m * m);
  return sizeof(c128) * (m * m * 3 + parts + (size_t)rows * m) + 256;
}

int orthonormalize_columns(int64_t rows, int64_t ld, int64_t c0, int64_t c1, c128 *A, void *work,
                           hipStream_t s, int *flag_dev) {
  const int m = (int)(c1 - c0);
  if (m <= 0) return QFS_OK;
  c128 *P = static_cast<c128 *>(work);          // c0 x m (<= c1 x c1)
  c128 *Gm = P + (size_t)c1 * c1;                 // m x m
  c128 *T = Gm + (size_t)m * m;                   // m x m
  c128 *Tmp = T + (size_t)m * m;                  // rows x m
  c128 *parts = Tmp + (size_t)rows * m;           // gram_parts(m) x m x m
  int *flag = flag_dev ? flag_dev : reinterpret_cast<int *>(parts + (size_t)gram_parts(m) * m * m);
  if (!flag_dev) QFS_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  c128 *An = A + c0;
  const c128 one = cmake(1.0, 0.0), zero = cmake(0.0, 0.0), mone = cmake(-1.0, 0.0);
  if (c0 > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      QFS_TRY(launch_zgemm(true, (int)c0, m, (int)rows, one, A, (int)ld, An, (int)ld, zero, P, m, s));
      QFS_TRY(launch_zgemm(false, (int)rows, m, (int)c0, mone, A, (int)ld, P, m, one, An, (int)ld, s));
    }
  }
  for (int pass = 0; pass < 2; ++pass) {
    QFS_TRY(gram_splitk(m, m, (int)rows, An, (int)ld, An, (int)ld, Gm, parts, s));
    QFS_TRY(cholesky_upper_blocked(m, Gm, flag, s));
    if (m <= 256)
      hipLaunchKernelGGL(k_tri_inverse_rows<4>, dim3(m), dim3(64), 0, s, m, Gm, T);
    else
      hipLaunchKernelGGL(k_tri_inverse_upper, dim3(m), dim3(64), sizeof(c128) * (size_t)m, s, m, Gm, T);
    QFS_HIP(hipGetLastError());
    QFS_TRY(launch_zgemm(false, (int)rows, m, m, one, An, (int)ld, T, m, zero, Tmp, m, s));
    const int64_t total = rows * m;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)),
                       dim3(256), 0, s, rows, m, Tmp, m, An, (int)ld);
    QFS_HIP(hipGetLastError());
  }
  if (flag_dev) return QFS_OK;  // the caller reads the flag
  int h_flag = 0;
  QFS_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  if (h_flag) {
    set_error_detail("orthonormalisation: non-positive Cholesky pivot (dependent columns)");
    return QFS_ENUMERIC;
  }
  return QFS_OK;
}

// ------------------------------------------------------------------ layout conversions
// sample-major [M][N] c128 -> chunked amplitude-major (32x32 LDS transpose tiles);
// element (i, j) of the chunked set is at (j >> logC) * N * C + i * C + (j & (C - 1)).
template <typename R>
__global__ __launch_bounds__(256) void k_to_internal(int n, int64_t M, int logC, int64_t cols,
                                                     const c128 *src, cx<R> *dst) {
  __shared__ c128 tile[32][33];
  const int64_t N = int64_t(1) << n;
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows per pass
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r, i = i0 + tx;
    tile[r][tx] = (j < M && i < N) ? src[j * N + i] : cmake(0.0, 0.0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    if (i < N && j < cols) {
      const c128 v = tile[tx][r];
      dst[((j >> logC) << (n + logC)) + (i << logC) + (j & ((1 << logC) - 1))] =
          cmake<R>((R)v.re, (R)v.im);
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_from_internal(int n, int64_t M, int logC, const cx<R> *src,
                                                       c128 *dst) {
  __shared__ c128 tile[32][33];
  const int64_t N = int64_t(1) << n;
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    if (i < N && j < M) {
      const cx<R> v = src[((j >> logC) << (n + logC)) + (i << logC) + (j & ((1 << logC) - 1))];
      tile[r][tx] = cmake<double>(v.re, v.im);
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r, i = i0 + tx;
    if (j < M && i < N) dst[j * N + i] = tile[tx][r];
  }
}

template <typename R>
int launch_to_internal(int n, int64_t M, int logC, int64_t nch, const c128 *src, cx<R> *dst,
                       hipStream_t s) {
  const int64_t N = int64_t(1) << n, cols = nch << logC;
  dim3 grid((unsigned)((N + 31) / 32), (unsigned)((cols + 31) / 32));
  hipLaunchKernelGGL(k_to_internal<R>, grid, dim3(256), 0, s, n, M, logC, cols, src, dst);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

template <typename R>
int launch_from_internal(int n, int64_t M, int logC, const cx<R> *src, c128 *dst, hipStream_t s) {
  const int64_t N = int64_t(1) << n;
  dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
  hipLaunchKernelGGL(k_from_internal<R>, grid, dim3(256), 0, s, n, M, logC, src, dst);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

template int launch_to_internal<float>(int, int64_t, int, int64_t, const c128 *, c64 *, hipStream_t);
template int launch_to_internal<double>(int, int64_t, int, int64_t, const c128 *, c128 *, hipStream_t);
template int launch_from_internal<float>(int, int64_t, int, const c64 *, c128 *, hipStream_t);
template int launch_from_internal<double>(int, int64_t, int, const c128 *, c128 *, hipStream_t);

__global__ void k_narrow(int64_t count, const c128 *src, c64 *dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = cmake<float>((float)src[e].re, (float)src[e].im);
}

int launch_narrow(int64_t count, const c128 *src, c64 *dst, hipStream_t s) {
  if (count <= 0) return QFS_OK;
  hipLaunchKernelGGL(k_narrow, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 65536)),
                     dim3(256), 0, s, count, src, dst);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

__global__ void k_copy_slots(const int32_t *slots, SlotCopy c) {
  const int64_t s = slots[blockIdx.y];
  for (int b = 0; b < SlotCopy::kBufs; ++b) {
    const int64_t u = c.units[b];
    if (u == 0) continue;
    const uint4 *src = c.src[b] + s * u;
    uint4 *dst = c.dst[b] + s * u;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < u; e += (int64_t)gridDim.x * blockDim.x)
      dst[e] = src[e];
  }
}

int launch_copy_slots(const int32_t *slots, int nslots, const SlotCopy &c, hipStream_t s) {
  if (nslots <= 0) return QFS_OK;
  int64_t umax = 0;
  for (int b = 0; b < SlotCopy::kBufs; ++b) umax = std::max(umax, c.units[b]);
  if (umax == 0) return QFS_OK;
  const unsigned bx = (unsigned)std::min<int64_t>((umax + 255) / 256, 64);
  hipLaunchKernelGGL(k_copy_slots, dim3(bx, (unsigned)nslots), dim3(256), 0, s, slots, c);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// Fill with zeros by a kernel (safe inside captured graphs).
__global__ void k_zero(uint4 *p, int64_t n16) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n16;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = make_uint4(0, 0, 0, 0);
}

int launch_zero(void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return QFS_OK;
  if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(p) & 15) != 0) {
    QFS_HIP(hipMemsetAsync(p, 0, bytes, s));
    return QFS_OK;
  }
  const int64_t n16 = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>((n16 + 255) / 256, 65536)), dim3(256),
                     0, s, static_cast<uint4 *>(p), n16);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

// Columns 0..N-1 of the N x ld matrix A set to the computational basis (A zeroed before):
// A[i][i] = 1.
__global__ void k_unit_columns(int64_t N, int64_t ld, c128 *A) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    A[i * ld + i] = cmake(1.0, 0.0);
}

int launch_unit_columns(int64_t N, int64_t ld, c128 *A, hipStream_t s) {
  if (N <= 0 || ld < N) return QFS_EINVAL;
  hipLaunchKernelGGL(k_unit_columns, dim3((unsigned)std::min<int64_t>((N + 255) / 256, 4096)), dim3(256), 0,
                     s, N, ld, A);
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

}  // namespace qfs
