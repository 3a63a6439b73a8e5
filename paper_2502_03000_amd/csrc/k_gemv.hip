// Matrix-vector products (the xGEMV mapping of a product with a vector,
// Sec. II), with an optional element-wise epilogue evaluated on the result
// before it is stored, so that e.g. trans(A)*u + 0.5*(d % e) is one pass.
//
// y = alpha * A x    (trans = 0): a workgroup owns 64 rows (one per lane) and
//                    its 16 waves split the columns; a fixed-order LDS
//                    reduction combines them.
// y = alpha * A^T x  (trans = 1): one wave per output entry reduces a column
//                    with its 64 lanes (coalesced reads down the column).
// Both are HBM-bound: each element of A is read once.
#include <hip/hip_runtime.h>

#include "ew_device.h"

namespace hexla {
namespace k {

namespace {

constexpr int kWavesN = 16;

template <typename T>
__global__ __launch_bounds__(64 * kWavesN) void gemv_n_kernel(int64_t ms, int64_t ns, T alpha,
                                                              const T* __restrict__ A, int64_t lda,
                                                              const T* __restrict__ x,
                                                              int64_t incx, T* __restrict__ y,
                                                              int64_t incy, EwProgram epi,
                                                              int has_epi) {
  __shared__ T red[kWavesN][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t i = int64_t(blockIdx.x) * 64 + lane;
  T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  if (i < ms) {
    int64_t j = w;
    for (; j + 3 * kWavesN < ns; j += 4 * kWavesN) {
      const T a0 = A[i + j * lda], a1 = A[i + (j + kWavesN) * lda];
      const T a2 = A[i + (j + 2 * kWavesN) * lda], a3 = A[i + (j + 3 * kWavesN) * lda];
      acc0 += a0 * x[j * incx];
      acc1 += a1 * x[(j + kWavesN) * incx];
      acc2 += a2 * x[(j + 2 * kWavesN) * incx];
      acc3 += a3 * x[(j + 3 * kWavesN) * incx];
    }
    for (; j < ns; j += kWavesN) acc0 += A[i + j * lda] * x[j * incx];
  }
  red[w][lane] = (acc0 + acc1) + (acc2 + acc3);
  __syncthreads();
  if (w == 0 && i < ms) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < kWavesN; ++q) s += red[q][lane];
    T v = alpha * s;
    if (has_epi) v = ew_eval_at<T>(epi, i, v);
    y[i * incy] = v;
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void gemv_t_kernel(int64_t ms, int64_t ns, T alpha,
                                                     const T* __restrict__ A, int64_t lda,
                                                     const T* __restrict__ x, int64_t incx,
                                                     T* __restrict__ y, int64_t incy,
                                                     EwProgram epi, int has_epi) {
  const int lane = threadIdx.x & 63;
  const int64_t j = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (j >= ns) return;
  const T* col = A + j * lda;
  T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  int64_t i = lane;
  for (; i + 192 < ms; i += 256) {
    acc0 += col[i] * x[i * incx];
    acc1 += col[i + 64] * x[(i + 64) * incx];
    acc2 += col[i + 128] * x[(i + 128) * incx];
    acc3 += col[i + 192] * x[(i + 192) * incx];
  }
  for (; i < ms; i += 64) acc0 += col[i] * x[i * incx];
  const T s = wave_sum((acc0 + acc1) + (acc2 + acc3));
  if (lane == 0) {
    T v = alpha * s;
    if (has_epi) v = ew_eval_at<T>(epi, j, v);
    y[j * incy] = v;
  }
}

template <typename T>
hipError_t launch_typed(int trans, int64_t ms, int64_t ns, double alpha, const void* A,
                        int64_t lda, const void* x, int64_t incx, void* y, int64_t incy,
                        const EwProgram* epi, hipStream_t s) {
  EwProgram e{};
  const int has_epi = epi != nullptr;
  if (epi) e = *epi;
  const T* a = static_cast<const T*>(A);
  const T* xv = static_cast<const T*>(x);
  T* yv = static_cast<T*>(y);
  if (trans == 0) {
    if (ms == 0) return hipSuccess;
    const int64_t blocks = (ms + 63) / 64;
    hipLaunchKernelGGL((gemv_n_kernel<T>), dim3(unsigned(blocks)), dim3(64 * kWavesN), 0, s, ms,
                       ns, T(alpha), a, lda, xv, incx, yv, incy, e, has_epi);
  } else {
    if (ns == 0) return hipSuccess;
    const int64_t blocks = (ns + 3) / 4;
    hipLaunchKernelGGL((gemv_t_kernel<T>), dim3(unsigned(blocks)), dim3(256), 0, s, ms, ns,
                       T(alpha), a, lda, xv, incx, yv, incy, e, has_epi);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t gemv_launch(int dtype, int trans, int64_t ms, int64_t ns, double alpha,
                       const void* A, int64_t lda, const void* x, int64_t incx, void* y,
                       int64_t incy, const EwProgram* epi, hipStream_t s) {
  return dtype == 0
             ? launch_typed<double>(trans, ms, ns, alpha, A, lda, x, incx, y, incy, epi, s)
             : launch_typed<float>(trans, ms, ns, alpha, A, lda, x, incx, y, incy, epi, s);
}

}  // namespace k
}  // namespace hexla
