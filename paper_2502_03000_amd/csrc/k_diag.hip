// Diagonal partial products and multiply-and-sum reductions (expressions (4),
// (5) and (7) of Sec. III): only the diagonal of a product is formed,
// d_i = sum_k op(A)_ik op(B)_ki, and a trace or a vector-diagonal-vector
// product is one pass that multiplies and sums, with no temporary matrix.
//
// All of it is bound by HBM: each operand element is read once. The
// diagonal product takes 64 diagonal entries and a range of k per
// workgroup; both operand tiles (64 x 64) are loaded with the wave running
// along the contiguous storage direction of each operand (i for an operand
// stored with i fastest, k for the other) and meet in LDS, so every global
// load is coalesced whatever the transposes. Long contractions are split
// over workgroups; the partial sums are added in a fixed order by a second
// kernel, so results are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ew_device.h"
#include "kernels.h"

namespace hexla {
namespace k {

namespace {

constexpr int kTI = 64;        // diagonal entries per workgroup
constexpr int kTK = 64;        // k per step
constexpr int kThreads = 256;  // 4 waves; wave w sums k = 16 w .. 16 w + 15 of each step
constexpr int kSumThreads = 1024;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// One 64 x 64 tile of an operand into LDS as s[k][i]. ROW: the operand's
// storage runs along i (element (i, k) at p[i + k * ld]); otherwise along k
// (element at p[k + i * ld]). Out-of-range elements read as zero; their
// addresses are clamped so that every load is issued unconditionally.
template <typename T, bool ROW>
__device__ __forceinline__ void load_tile(const T* __restrict__ p, int64_t ld, int64_t i0,
                                          int64_t k0, int64_t ni, int64_t nk, T (*s)[kTI + 1]) {
  const int t = threadIdx.x;
  const int fast = t & 63, slow = t >> 6;
  T v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t il = ROW ? fast : slow + 4 * r;  // tile row index (i)
    const int64_t kl = ROW ? slow + 4 * r : fast;  // tile column index (k)
    const int64_t i = std::min<int64_t>(i0 + il, ni - 1);
    const int64_t k = std::min<int64_t>(k0 + kl, nk - 1);
    v[r] = ROW ? p[i + k * ld] : p[k + i * ld];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int il = ROW ? fast : slow + 4 * r;
    const int kl = ROW ? slow + 4 * r : fast;
    const bool in = (i0 + il < ni) & (k0 + kl < nk);
    s[kl][il] = in ? v[r] : T(0);
  }
}

// TA: op(A) = A^T (element (i, k) of op(A) at A[k + i lda]); TB: op(B) = B^T
// (element (k, i) of op(B) at B[i + k ldb]).
template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void diagprod_kernel(int64_t nd, int64_t kk, const T* A,
                                                            int64_t lda, const T* B, int64_t ldb,
                                                            int64_t kchunk, T alpha, T* d,
                                                            int64_t incd, T* partial) {
  __shared__ T sa[kTK][kTI + 1];
  __shared__ T sb[kTK][kTI + 1];
  __shared__ T red[kThreads / 64][kTI];
  const int64_t i0 = int64_t(blockIdx.x) * kTI;
  const int64_t kb = int64_t(blockIdx.y) * kchunk;
  const int64_t ke = std::min<int64_t>(kk, kb + kchunk);
  const int t = threadIdx.x, il = t & 63, w = t >> 6;
  T acc = T(0);
  for (int64_t k0 = kb; k0 < ke; k0 += kTK) {
    // op(A) is stored along i when not transposed; op(B)'s element (k, i)
    // is stored along i when B is transposed
    load_tile<T, !TA>(A, lda, i0, k0, nd, ke, sa);
    load_tile<T, TB>(B, ldb, i0, k0, nd, ke, sb);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += sa[16 * w + q][il] * sb[16 * w + q][il];
    __syncthreads();
  }
  red[w][il] = acc;
  __syncthreads();
  if (w == 0) {
    const T s = (red[0][il] + red[1][il]) + (red[2][il] + red[3][il]);
    const int64_t i = i0 + il;
    if (i < nd) {
      if (partial) partial[int64_t(blockIdx.y) * nd + i] = s;
      else d[i * incd] = alpha * s;
    }
  }
}

// d[i incd] = alpha * sum over s of part[s nd + i], s in order.
template <typename T>
__global__ __launch_bounds__(256) void colsum_kernel(int64_t nd, int S, const T* part, T alpha,
                                                     T* d, int64_t incd) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= nd) return;
  T s = T(0);
  for (int q = 0; q < S; ++q) s += part[int64_t(q) * nd + i];
  d[i * incd] = alpha * s;
}

// Block-wide sum of one value per thread, in a fixed order.
template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T sh[NT];
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  return sh[0];
}

// out[0] = alpha * sum of x[0 .. n): one workgroup, thread t takes
// t, t + 1024, ... in order, then a fixed tree.
template <typename T>
__global__ __launch_bounds__(kSumThreads) void sum_all_kernel(int64_t n, const T* x, T alpha,
                                                              T* out) {
  T s = T(0);
  for (int64_t i = threadIdx.x; i < n; i += kSumThreads) s += x[i];
  s = block_sum<T, kSumThreads>(s);
  if (threadIdx.x == 0) out[0] = alpha * s;
}

// Sum of an element-wise program over its rows x cols elements (any
// strides): each workgroup sums a contiguous range of flat indices; one
// workgroup writes alpha * sum to out directly, more write partials.
template <typename T>
__global__ __launch_bounds__(256) void ew_sum_kernel(EwProgram p, int64_t per_block, T alpha,
                                                     T* out, T* partial) {
  const int64_t count = p.rows * p.cols;
  const int64_t b0 = int64_t(blockIdx.x) * per_block;
  const int64_t b1 = std::min<int64_t>(count, b0 + per_block);
  T s = T(0);
  for (int64_t e = b0 + threadIdx.x; e < b1; e += 256) s += ew_eval_at<T>(p, e, T(0));
  s = block_sum<T, 256>(s);
  if (threadIdx.x == 0) {
    if (partial) partial[blockIdx.x] = s;
    else out[0] = alpha * s;
  }
}

// The same sum for views of at least kSumColRows rows: tiles of 256 x
// kSumV rows of one column (row and column found once per tile, kSumV
// elements per lane, a 16-byte pack's worth, with their loads in flight
// together); workgroup b takes tiles b, b + G, b + 2G, ... (G workgroups),
// so the order of the additions is fixed.
template <typename T>
constexpr int kSumV = 16 / int(sizeof(T));
constexpr int64_t kSumColRows = 64;
template <typename T>
__global__ __launch_bounds__(256) void ew_sum_columns_kernel(EwProgram p, int64_t tiles_per_col,
                                                             int64_t tiles, T alpha, T* out,
                                                             T* partial) {
  T s = T(0);
  for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
    const int64_t j = b / tiles_per_col;
    const int64_t i0 = (b - j * tiles_per_col) * (256 * kSumV<T>) + threadIdx.x;
    const Pack<T, kSumV<T>> r = ew_eval_col<T, kSumV<T>, 256>(p, i0, j);
#pragma unroll
    for (int e = 0; e < kSumV<T>; ++e) s += (i0 + int64_t(e) * 256 < p.rows) ? r.v[e] : T(0);
  }
  s = block_sum<T, 256>(s);
  if (threadIdx.x == 0) {
    if (partial) partial[blockIdx.x] = s;
    else out[0] = alpha * s;
  }
}

int diag_split(int64_t nd, int64_t kk) {
  // about 2048 workgroups in flight (8 per CU), each over at least 4 steps
  const int64_t blocks = cdiv(nd, kTI);
  const int64_t want = cdiv(2048, std::max<int64_t>(blocks, 1));
  const int64_t most = std::max<int64_t>(1, cdiv(kk, 4 * kTK));
  return int(std::max<int64_t>(1, std::min(want, most)));
}

template <typename T>
hipError_t diagprod_typed(int ta, int tb, int64_t nd, int64_t kk, double alpha, const T* A,
                          int64_t lda, const T* B, int64_t ldb, T* d, int64_t incd, bool sum,
                          T* partial, hipStream_t s) {
  if (nd <= 0 || kk <= 0) {  // an empty diagonal or contraction: zeros
    if (sum)
      hipLaunchKernelGGL((sum_all_kernel<T>), dim3(1), dim3(kSumThreads), 0, s, int64_t(0),
                         static_cast<const T*>(nullptr), T(alpha), d);
    else if (nd > 0)
      hipLaunchKernelGGL((colsum_kernel<T>), dim3(unsigned(cdiv(nd, 256))), dim3(256), 0, s, nd, 0,
                         static_cast<const T*>(nullptr), T(alpha), d, incd);
    return hipGetLastError();
  }
  const int S = diag_split(nd, kk);
  const int64_t chunk = cdiv(cdiv(kk, S), kTK) * kTK;
  const int Sr = int(cdiv(kk, chunk));
  const bool direct = !sum && Sr == 1;
  T* part = direct ? nullptr : partial;
  if (!direct && !part) return hipErrorInvalidValue;
  const dim3 grid(unsigned(cdiv(nd, kTI)), unsigned(Sr));
#define HEXLA_DIAG_LAUNCH(TA_, TB_)                                                               \
  hipLaunchKernelGGL((diagprod_kernel<T, TA_, TB_>), grid, dim3(kThreads), 0, s, nd, kk, A, lda, \
                     B, ldb, chunk, T(alpha), d, incd, part)
  if (ta && tb) HEXLA_DIAG_LAUNCH(true, true);
  else if (ta) HEXLA_DIAG_LAUNCH(true, false);
  else if (tb) HEXLA_DIAG_LAUNCH(false, true);
  else HEXLA_DIAG_LAUNCH(false, false);
#undef HEXLA_DIAG_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || direct) return e;
  if (sum) {
    hipLaunchKernelGGL((sum_all_kernel<T>), dim3(1), dim3(kSumThreads), 0, s, int64_t(Sr) * nd,
                       static_cast<const T*>(part), T(alpha), d);
  } else {
    hipLaunchKernelGGL((colsum_kernel<T>), dim3(unsigned(cdiv(nd, 256))), dim3(256), 0, s, nd, Sr,
                       static_cast<const T*>(part), T(alpha), d, incd);
  }
  return hipGetLastError();
}

int64_t ew_sum_blocks(int64_t count) {
  // one workgroup up to 64 Ki elements; beyond, 4 Ki elements per workgroup
  // up to 2048 workgroups
  if (count <= (int64_t(1) << 16)) return 1;
  return std::min<int64_t>(2048, cdiv(count, 4096));
}

template <typename T>
hipError_t ew_sum_typed(const EwProgram& p, double alpha, T* out, T* partial, hipStream_t s) {
  const int64_t count = p.rows * p.cols;
  const int64_t nb = ew_sum_blocks(count);
  const int64_t per = std::max<int64_t>(1, cdiv(count, nb));
  if (nb > 1 && !partial) return hipErrorInvalidValue;
  if (p.rows >= kSumColRows) {
    const int64_t per_col = cdiv(p.rows, 256 * kSumV<T>);
    hipLaunchKernelGGL((ew_sum_columns_kernel<T>), dim3(unsigned(nb)), dim3(256), 0, s, p, per_col,
                       per_col * p.cols, T(alpha), out,
                       nb > 1 ? partial : static_cast<T*>(nullptr));
  } else {
    hipLaunchKernelGGL((ew_sum_kernel<T>), dim3(unsigned(nb)), dim3(256), 0, s, p, per, T(alpha),
                       out, nb > 1 ? partial : static_cast<T*>(nullptr));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  hipLaunchKernelGGL((sum_all_kernel<T>), dim3(1), dim3(kSumThreads), 0, s, nb,
                     static_cast<const T*>(partial), T(alpha), out);
  return hipGetLastError();
}

}  // namespace

size_t diagprod_partial_bytes(int dtype, int64_t nd, int64_t kk, bool sum) {
  if (nd <= 0 || kk <= 0) return 0;
  const int S = diag_split(nd, kk);
  const int64_t chunk = cdiv(cdiv(kk, S), kTK) * kTK;
  const int64_t Sr = cdiv(kk, chunk);
  if (!sum && Sr == 1) return 0;
  return size_t(Sr) * size_t(nd) * (dtype == 0 ? 8 : 4);
}

hipError_t diagprod_launch(int dtype, int ta, int tb, int64_t nd, int64_t kk, double alpha,
                           const void* A, int64_t lda, const void* B, int64_t ldb, void* d,
                           int64_t incd, bool sum, void* partial, hipStream_t s) {
  if (dtype == 0)
    return diagprod_typed<double>(ta, tb, nd, kk, alpha, static_cast<const double*>(A), lda,
                                  static_cast<const double*>(B), ldb, static_cast<double*>(d),
                                  incd, sum, static_cast<double*>(partial), s);
  return diagprod_typed<float>(ta, tb, nd, kk, alpha, static_cast<const float*>(A), lda,
                               static_cast<const float*>(B), ldb, static_cast<float*>(d), incd,
                               sum, static_cast<float*>(partial), s);
}

size_t ew_sum_partial_bytes(int dtype, int64_t count) {
  const int64_t nb = ew_sum_blocks(count);
  return nb > 1 ? size_t(nb) * (dtype == 0 ? 8 : 4) : 0;
}

hipError_t ew_sum_launch(int dtype, const EwProgram& p, double alpha, void* out, void* partial,
                         hipStream_t s) {
  if (dtype == 0)
    return ew_sum_typed<double>(p, alpha, static_cast<double*>(out), static_cast<double*>(partial), s);
  return ew_sum_typed<float>(p, alpha, static_cast<float*>(out), static_cast<float*>(partial), s);
}

}  // namespace k
}  // namespace hexla
