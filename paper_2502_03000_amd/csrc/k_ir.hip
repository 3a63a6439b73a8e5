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

// Infinity norm, stage 1: a workgroup takes 64 rows (one per lane) and one
// chunk of columns, split between its four waves (eight loads in flight per
// lane); the waves' row sums are added in LDS in wave order and
// part[chunk][row] receives the chunk's row sum. Stage 2 adds the chunks of
// each row in chunk order and keeps the largest row sum of 256 rows; stage 3
// (max_reduce_kernel) takes the largest of those.
constexpr int kNormChunks = 32;  // column chunks at most

template <typename T>
__global__ __launch_bounds__(256) void rowsum_part_kernel(int64_t rows, int64_t cols,
                                                          const T* __restrict__ a, int64_t lda,
                                                          int64_t chunk, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = int64_t(blockIdx.x) * 64 + lane;
  const int64_t ic = i < rows ? i : rows - 1;
  const int64_t j0 = int64_t(blockIdx.y) * chunk;
  const int64_t j1 = j0 + chunk < cols ? j0 + chunk : cols;
  double s = 0.0;
  for (int64_t j = j0 + wave * 8; j < j1; j += 32) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a[ic + (j + u < j1 ? j + u : j) * lda];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += j + u < j1 ? fabs(double(v[u])) : 0.0;
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && i < rows)
    part[int64_t(blockIdx.y) * rows + i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void rowsum_max_kernel(int64_t rows, int nchunks,
                                                         const double* __restrict__ part,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double s = 0.0;
  if (i < rows)
    for (int c = 0; c < nchunks; ++c) s += part[int64_t(c) * rows + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
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

size_t norm_scratch_elems(int64_t rows) {
  const int64_t r = std::max<int64_t>(rows, 1);
  return size_t(kNormChunks * r + cdiv(r, 256));
}

hipError_t norm_inf_launch(int dtype, int64_t rows, int64_t cols, const void* a, int64_t lda,
                           double* scratch, double* out, hipStream_t s) {
  if (rows <= 0 || cols <= 0) {
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, scratch, int64_t(0), out);
    return hipGetLastError();
  }
  // chunks of at least 256 columns, at most kNormChunks of them
  const int64_t chunk = std::max<int64_t>(256, cdiv(cols, kNormChunks));
  const int nchunks = int(cdiv(cols, chunk));
  const dim3 g1(unsigned(cdiv(rows, 64)), unsigned(nchunks));
  if (dtype == 0)
    hipLaunchKernelGGL((rowsum_part_kernel<double>), g1, dim3(256), 0, s, rows, cols,
                       static_cast<const double*>(a), lda, chunk, scratch);
  else
    hipLaunchKernelGGL((rowsum_part_kernel<float>), g1, dim3(256), 0, s, rows, cols,
                       static_cast<const float*>(a), lda, chunk, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t blocks = cdiv(rows, 256);
  double* bmax = scratch + int64_t(kNormChunks) * rows;
  hipLaunchKernelGGL(rowsum_max_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, rows, nchunks,
                     scratch, bmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, bmax, blocks, out);
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
