// Environment of one gate (Sec. 3, Eq. 10; Fig. env_calc_tensor) without device
// allocation: the same result as qfs_environment, computed straight from the caller's
// row-major state sets, with the work-group partial sums in a fixed device array of this
// library instead of a buffer allocated per call.
#include <algorithm>
#include <mutex>

#include "qfs_internal.h"

namespace qfs {
namespace {

constexpr int kNaThreads = 256;                  // threads per work-group
constexpr int kNaBlocks = 1024;                  // most work-groups, so most partials
constexpr int64_t kNaItemsPerThread = 1 << 10;   // most (sample, other-qubit) items a thread sums
constexpr int64_t kNaMaxItems = (int64_t)kNaBlocks * kNaThreads * kNaItemsPerThread;  // 2^28

// The partials: 16 complex128 per work-group, 256 KiB. Each GPU the library runs on holds
// its own copy until the process ends; every call on a GPU shares it.
static __device__ __align__(256) c128 scratch[kNaBlocks * 16];

// Item it = (sample j, value r of the n - 2 other qubits): the four amplitudes of a_j and
// b_j that differ in qubits qa, qb (qubit q is bit n - 1 - q of the amplitude index; the
// local index of the pair is 2 bit(qa) + bit(qb)). Each thread sums its items' 16 products
// a(q) conj(b(p)); the work-group's sums go to part[blockIdx.x][q * 4 + p], reduced over
// the threads in a fixed order.
__global__ __launch_bounds__(kNaThreads) void k_env_rows(int n, int64_t items, const c128 *a, const c128 *b,
                                                         int qa, int qb, c128 *part) {
  __shared__ c128 red[kNaThreads];
  const int pa = n - 1 - qa, pb = n - 1 - qb;
  const int lo = std::min(pa, pb), hi = std::max(pa, pb);
  const int64_t N = int64_t(1) << n;
  const int64_t rmask = (int64_t(1) << (n - 2)) - 1;
  c128 acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = cmake(0.0, 0.0);
  for (int64_t it = blockIdx.x * (int64_t)kNaThreads + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * kNaThreads) {
    const int64_t j = it >> (n - 2);
    int64_t r = it & rmask;
    // zero bits at positions lo and hi of the amplitude index
    r = ((r >> lo) << (lo + 1)) | (r & ((int64_t(1) << lo) - 1));
    r = ((r >> hi) << (hi + 1)) | (r & ((int64_t(1) << hi) - 1));
    const c128 *aj = a + j * N + r, *bj = b + j * N + r;
    c128 av[4], bv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t off = (int64_t((q >> 1) & 1) << pa) | (int64_t(q & 1) << pb);
      av[q] = aj[off];
      bv[q] = bj[off];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int p = 0; p < 4; ++p) cfma(acc[q * 4 + p], av[q], cconj(bv[p]));
  }
  for (int e = 0; e < 16; ++e) {
    red[threadIdx.x] = acc[e];
    __syncthreads();
    for (int w = kNaThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 16 + e] = red[0];
    __syncthreads();
  }
}

// gamma[e] = sum over the P partials in order.
__global__ __launch_bounds__(16) void k_env_rows_sum(const c128 *part, int P, c128 *gamma) {
  const int e = threadIdx.x;
  c128 s = cmake(0.0, 0.0);
  for (int p = 0; p < P; ++p) s = s + part[(int64_t)p * 16 + e];
  gamma[e] = s;
}

// Device address of `scratch` on each GPU, looked up once per device (the array's name in
// host code is only a stand-in, not a device address).
int scratch_ptr(c128 **out) {
  constexpr int kDevices = 64;
  static std::mutex mu;
  static c128 *ptr[kDevices] = {};
  int dev = 0;
  QFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kDevices) {
    set_error_detail("qfs_environment_noalloc: device index out of range");
    return QFS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void *p = nullptr;
    QFS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error_detail("qfs_environment_noalloc: no device address for the partials array");
      return QFS_EDEVICE;
    }
    ptr[dev] = static_cast<c128 *>(p);
  }
  *out = ptr[dev];
  return QFS_OK;
}

}  // namespace
}  // namespace qfs

using namespace qfs;

extern "C" int qfs_environment_noalloc(int32_t n, int32_t M, const qfs_c128 *a, const qfs_c128 *b, int32_t qa,
                                       int32_t qb, qfs_c128 *gamma, void *hip_stream) {
  if (n < 2 || n > 24 || qa < 0 || qb < 0 || qa >= n || qb >= n || qa == qb) {
    set_error_detail("qfs_environment_noalloc: need 2 <= n <= 24 and two distinct qubits below n");
    return QFS_EINVAL;
  }
  if (M < 1 || !a || !b || !gamma) return QFS_EINVAL;
  const int64_t items = (int64_t)M << (n - 2);
  if (items > kNaMaxItems) {
    set_error_detail("qfs_environment_noalloc: M 2^(n-2) = " + std::to_string(items) + " exceeds " +
                     std::to_string(kNaMaxItems) + " (1024 work-group partials of 256 x 1024 items)");
    return QFS_EINVAL;
  }
  c128 *part = nullptr;
  QFS_TRY(scratch_ptr(&part));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int P = (int)std::min<int64_t>(kNaBlocks, (items + kNaThreads - 1) / kNaThreads);
  hipLaunchKernelGGL(k_env_rows, dim3(P), dim3(kNaThreads), 0, s, n, items, reinterpret_cast<const c128 *>(a),
                     reinterpret_cast<const c128 *>(b), qa, qb, part);
  QFS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_env_rows_sum, dim3(1), dim3(16), 0, s, part, P, reinterpret_cast<c128 *>(gamma));
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}
