// Kernels of the mixed-precision solve: type conversion of column-major
// blocks, infinity norms (max row sum of |a|) and the correction update
// X += D with D in the low precision. The refinement loop itself is driven
// by the evaluator (it reads one small status block per iteration).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace hexla {
namespace k {

namespace {

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// b(i, j) = a(i, j) converted; a(i, j) = a[i*asi + j*asj] (any view).
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void cast_kernel(int64_t rows, int64_t cols, const Ti* __restrict__ a,
                                                   int64_t asi, int64_t asj, To* __restrict__ b,
                                                   int64_t ldb) {
  const int64_t total = rows * cols;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % rows, j = e / rows;
    b[i + j * ldb] = To(a[i * asi + j * asj]);
  }
}

// Stage 1: each workgroup owns up to 256 rows; partial[block] = max row sum.
template <typename T>
__global__ __launch_bounds__(256) void rowsum_max_kernel(int64_t rows, int64_t cols, const T* __restrict__ a,
                                                         int64_t lda, double* __restrict__ partial) {
  __shared__ double red[256];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double s = 0.0;
  if (i < rows)
    for (int64_t j = 0; j < cols; ++j) s += fabs(double(a[i + j * lda]));
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void max_reduce_kernel(const double* __restrict__ partial, int64_t n,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, partial[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

template <typename Td>
__global__ __launch_bounds__(256) void add_mixed_kernel(int64_t rows, int64_t cols, double* __restrict__ x,
                                                        int64_t ldx, const Td* __restrict__ d, int64_t ldd) {
  const int64_t total = rows * cols;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % rows, j = e / rows;
    x[i + j * ldx] += double(d[i + j * ldd]);
  }
}

unsigned grid_for(int64_t n) { return unsigned(std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 8192))); }

}  // namespace

hipError_t cast_launch(int from, int to, int64_t rows, int64_t cols, const void* a, int64_t asi,
                       int64_t asj, void* b, int64_t ldb, hipStream_t s) {
  if (rows * cols == 0) return hipSuccess;
  const unsigned g = grid_for(rows * cols);
  if (from == 0 && to == 1)
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(g), dim3(256), 0, s, rows, cols,
                       static_cast<const double*>(a), asi, asj, static_cast<float*>(b), ldb);
  else if (from == 1 && to == 0)
    hipLaunchKernelGGL((cast_kernel<float, double>), dim3(g), dim3(256), 0, s, rows, cols,
                       static_cast<const float*>(a), asi, asj, static_cast<double*>(b), ldb);
  else if (from == 0)
    hipLaunchKernelGGL((cast_kernel<double, double>), dim3(g), dim3(256), 0, s, rows, cols,
                       static_cast<const double*>(a), asi, asj, static_cast<double*>(b), ldb);
  else
    hipLaunchKernelGGL((cast_kernel<float, float>), dim3(g), dim3(256), 0, s, rows, cols,
                       static_cast<const float*>(a), asi, asj, static_cast<float*>(b), ldb);
  return hipGetLastError();
}

size_t norm_scratch_elems(int64_t rows) { return size_t(cdiv(std::max<int64_t>(rows, 1), 256)); }

hipError_t norm_inf_launch(int dtype, int64_t rows, int64_t cols, const void* a, int64_t lda,
                           double* scratch, double* out, hipStream_t s) {
  const int64_t blocks = cdiv(std::max<int64_t>(rows, 1), 256);
  if (dtype == 0)
    hipLaunchKernelGGL((rowsum_max_kernel<double>), dim3(unsigned(blocks)), dim3(256), 0, s, rows,
                       cols, static_cast<const double*>(a), lda, scratch);
  else
    hipLaunchKernelGGL((rowsum_max_kernel<float>), dim3(unsigned(blocks)), dim3(256), 0, s, rows,
                       cols, static_cast<const float*>(a), lda, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, scratch, blocks, out);
  return hipGetLastError();
}

hipError_t add_mixed_launch(int dtype_d, int64_t rows, int64_t cols, double* x, int64_t ldx,
                            const void* d, int64_t ldd, hipStream_t s) {
  if (rows * cols == 0) return hipSuccess;
  const unsigned g = grid_for(rows * cols);
  if (dtype_d == 1)
    hipLaunchKernelGGL((add_mixed_kernel<float>), dim3(g), dim3(256), 0, s, rows, cols, x, ldx,
                       static_cast<const float*>(d), ldd);
  else
    hipLaunchKernelGGL((add_mixed_kernel<double>), dim3(g), dim3(256), 0, s, rows, cols, x, ldx,
                       static_cast<const double*>(d), ldd);
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
