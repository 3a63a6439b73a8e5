// Structure-aware solves (expression (10) of Sec. III and the solve of the
// call trace in Sec. IV): the system matrix is examined before a solver is
// chosen, so that a diagonal, triangular, tridiagonal or symmetric positive
// definite matrix does not pay for a general LU.
//
//   structure   one pass over S (64 x 64 tiles paired with their mirror
//               tiles) finds the lower and upper bandwidths, whether S equals
//               its transpose, whether its diagonal is positive, and zero
//               diagonal entries;
//   Cholesky    right-looking, 64-column blocks: each diagonal block is
//               factored by one wave with its rows in registers, which also
//               inverts the block's factor; the block column below is
//               L21 = A21 L11^-T (a product with that inverse) and the
//               trailing matrix takes a symmetric rank-64 update (the SYRK
//               tile map). No pivoting, so no per-column exchange between
//               workgroups;
//   triangular  per 64-row block: the inverse of the diagonal block applied,
//               then a product updating the rows still to solve;
//   tridiagonal Gaussian elimination with partial pivoting between adjacent
//               rows (a fill-in of one extra superdiagonal), one lane per
//               right-hand side.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace hexla {
namespace k {

namespace {

constexpr int kB = 64;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ structure

// info[0] = lower bandwidth, info[1] = upper bandwidth, info[2] = 1 if some
// S_ij != S_ji or is NaN, info[3] = 1 if some diagonal entry is not > 0,
// info[5] = 1 if some diagonal entry is zero; the 64-bit words at info + 8
// and info + 10 get max |S_ij| and max |S_ij - S_ji| (as FP64 bit patterns,
// which order like the values for non-negative numbers). A product X X^T
// formed by a general GEMM is symmetric only up to its summation order, so
// the caller compares the two maxima. Tile t enumerates the pairs I >= J.
template <typename T>
__global__ __launch_bounds__(256) void structure_kernel(int64_t n, const T* __restrict__ S,
                                                        int64_t lds, int32_t* info) {
  __shared__ T sa[kB][kB + 1];
  __shared__ T sm[kB][kB + 1];
  __shared__ int s_red[4][4];
  __shared__ double s_max[4][2];
  const int64_t t = blockIdx.x;
  int64_t I = int64_t((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int64_t J = t - I * (I + 1) / 2;
  const int r = threadIdx.x & 63, cq = threadIdx.x >> 6;
  // tile (I, J) into sa[r][c]; tile (J, I) into sm[r][c] (both by columns)
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = cq + 4 * q;
    const int64_t i = I * kB + r, j = J * kB + c;
    const int64_t i2 = J * kB + r, j2 = I * kB + c;
    const bool in1 = i < n && j < n, in2 = i2 < n && j2 < n;
    sa[r][c] = in1 ? S[std::min<int64_t>(i, n - 1) + std::min<int64_t>(j, n - 1) * lds] : T(0);
    sm[r][c] = in2 ? S[std::min<int64_t>(i2, n - 1) + std::min<int64_t>(j2, n - 1) * lds] : T(0);
  }
  __syncthreads();
  int kl = 0, ku = 0, asym = 0, nonpos = 0, zero = 0;
  double amax = 0.0, dmax = 0.0;
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int c = cq + 4 * q;
    const int64_t i = I * kB + r, j = J * kB + c;  // element of tile (I, J)
    if (i < n && j < n) {
      const T a = sa[r][c];
      const T b = sm[c][r];  // element (j, i)
      if (a != T(0)) {
        if (i > j) kl = max(kl, int(std::min<int64_t>(i - j, 0x7fffffff)));
        if (j > i) ku = max(ku, int(std::min<int64_t>(j - i, 0x7fffffff)));
      }
      if (b != T(0)) {  // the mirror element (j, i) counts for the other band
        if (j > i) kl = max(kl, int(std::min<int64_t>(j - i, 0x7fffffff)));
        if (i > j) ku = max(ku, int(std::min<int64_t>(i - j, 0x7fffffff)));
      }
      if (!(a == b)) asym = 1;  // NaN compares unequal
      const double da = fmax(fabs(double(a)), fabs(double(b)));
      const double dd = fabs(double(a) - double(b));
      amax = da > amax ? da : amax;  // a NaN never replaces the maximum ...
      dmax = dd > dmax ? dd : dmax;
      if (a != a || b != b) dmax = __builtin_inf();  // ... but makes S unsymmetric
      if (i == j) {
        if (!(a > T(0))) nonpos = 1;
        if (a == T(0)) zero = 1;
      }
    }
  }
  // workgroup maxima, then one atomic per workgroup and field
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    amax = fmax(amax, __shfl_xor(amax, off));
    dmax = fmax(dmax, __shfl_xor(dmax, off));
    kl = max(kl, __shfl_xor(kl, off));
    ku = max(ku, __shfl_xor(ku, off));
    asym |= __shfl_xor(asym, off);
    nonpos |= __shfl_xor(nonpos, off);
    zero |= __shfl_xor(zero, off);
  }
  if (lane == 0) {
    s_max[w][0] = amax;
    s_max[w][1] = dmax;
    s_red[w][0] = kl;
    s_red[w][1] = ku;
    s_red[w][2] = asym;
    s_red[w][3] = (nonpos ? 1 : 0) | (zero ? 2 : 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int q = 0; q < 4; ++q) {
      a0 = max(a0, s_red[q][0]);
      a1 = max(a1, s_red[q][1]);
      a2 |= s_red[q][2];
      a3 |= s_red[q][3];
    }
    double m0 = 0.0, m1 = 0.0;
    for (int q = 0; q < 4; ++q) {
      m0 = fmax(m0, s_max[q][0]);
      m1 = fmax(m1, s_max[q][1]);
    }
    unsigned long long* words = reinterpret_cast<unsigned long long*>(info + 8);
    if (m0 > 0.0) atomicMax(words, static_cast<unsigned long long>(__double_as_longlong(m0)));
    if (m1 > 0.0) atomicMax(words + 1, static_cast<unsigned long long>(__double_as_longlong(m1)));
    if (a0) atomicMax(info + 0, a0);
    if (a1) atomicMax(info + 1, a1);
    if (a2) atomicOr(info + 2, 1);
    if (a3 & 1) atomicOr(info + 3, 1);
    if (a3 & 2) atomicOr(info + 5, 1);
  }
}

// ------------------------------------------------ 64 x 64 triangular blocks

// Inverse of the lower-triangular (non-unit) 64 x 64 matrix in sL (rows past
// jb hold the identity): thread i computes column i of X = L^-1 by forward
// substitution, X written to inv (column-major, ld 64).
template <typename T>
__device__ void invert_lower_block(T (*sL)[kB + 1], T (*sX)[kB + 1], T* inv) {
  const int i = threadIdx.x;
  for (int c = 0; c < kB; ++c) {
    T x;
    if (c < i) {
      x = T(0);
    } else if (c == i) {
      x = T(1) / sL[c][c];
    } else {
      T s = T(0);
      for (int k = i; k < c; ++k) s += sL[c][k] * sX[k][i];
      x = -s / sL[c][c];
    }
    sX[c][i] = x;  // only this thread reads column i of sX
    inv[c + i * kB] = x;
  }
}

// Cholesky of the diagonal block at (k0, k0) (jb <= 64 rows): thread i
// holds row i with the current column rotated into v[0]. The factor L11 is
// written over the block's lower triangle and L11^-1 to inv. A pivot that is
// not > 0 sets info[4] (the block is then not factored further).
template <typename T>
__global__ __launch_bounds__(kB) void potrf_block_kernel(T* __restrict__ A, int64_t lda,
                                                         int64_t k0, int jb, T* inv,
                                                         int32_t* info) {
  __shared__ T col[kB];
  __shared__ T sL[kB][kB + 1];
  __shared__ T sX[kB][kB + 1];
  __shared__ int s_bad;
  const int i = threadIdx.x;
  const bool own = i < jb;
  T v[kB];
#pragma unroll
  for (int c = 0; c < kB; ++c) {
    const bool in = own && c < jb;
    v[c] = in ? A[(k0 + i) + (k0 + c) * lda] : (i == c ? T(1) : T(0));
  }
  if (i == 0) s_bad = 0;
  __syncthreads();
#pragma unroll 1
  for (int j = 0; j < kB; ++j) {
    if (i == j) col[0] = v[0];
    __syncthreads();
    const T d = col[0];
    const bool ok = d > T(0);
    if (!ok && i == 0) s_bad = 1;
    const T ljj = ok ? sqrt(d) : T(1);
    const T lij = i > j ? v[0] / ljj : (i == j ? ljj : T(0));
    __syncthreads();
    col[i] = lij;
    sL[i][j] = lij;
    __syncthreads();
    // trailing columns k = j + c: a_ik -= l_ij l_kj for rows i > j
#pragma unroll
    for (int c = 1; c < kB; ++c) {
      const int kk = j + c < kB ? j + c : kB - 1;
      const T lkj = j + c < kB ? col[kk] : T(0);
      v[c] -= lij * lkj;
    }
#pragma unroll
    for (int c = 0; c < kB - 1; ++c) v[c] = v[c + 1];
    v[kB - 1] = T(0);
  }
  __syncthreads();
  if (s_bad) {
    if (i == 0) info[4] = 1;
    return;
  }
  if (own) {
    for (int c = 0; c <= i && c < jb; ++c) A[(k0 + i) + (k0 + c) * lda] = sL[i][c];
  }
  invert_lower_block<T>(sL, sX, inv);
}

// Inverses of the 64 x 64 diagonal blocks of a triangular matrix (non-unit;
// LOWER or upper), one block per workgroup: inv[p] = (S_pp)^-1, stored
// column-major with ld 64. An upper block is inverted as the transpose of
// its (lower) transpose. A zero diagonal entry sets info[6].
template <typename T, bool LOWER>
__global__ __launch_bounds__(kB) void trinv_block_kernel(const T* __restrict__ S, int64_t lds,
                                                         int64_t n, T* inv, int32_t* info) {
  __shared__ T sL[kB][kB + 1];
  __shared__ T sX[kB][kB + 1];
  __shared__ T sT[kB * kB];
  const int64_t p = blockIdx.x, k0 = p * kB;
  const int jb = int(std::min<int64_t>(kB, n - k0));
  const int i = threadIdx.x;
  // row i of L: for a lower block S[k0 + i][k0 + c]; for an upper block the
  // transpose, S[k0 + c][k0 + i] (read down column i: coalesced by c... the
  // loads run along each thread's own column)
  bool zero = false;
  for (int c = 0; c < kB; ++c) {
    T x;
    if (i < jb && c < jb) x = LOWER ? S[(k0 + i) + (k0 + c) * lds] : S[(k0 + c) + (k0 + i) * lds];
    else x = i == c ? T(1) : T(0);
    if (c > i) x = T(0);
    if (c == i && x == T(0)) zero = true;
    sL[i][c] = x;
  }
  if (zero) info[6] = 1;
  __syncthreads();
  T* out = inv + p * kB * kB;
  if (LOWER) {
    invert_lower_block<T>(sL, sX, out);
  } else {
    invert_lower_block<T>(sL, sX, sT);  // (U^T)^-1 ...
    __syncthreads();
    for (int c = 0; c < kB; ++c) out[c + i * kB] = sT[i + c * kB];  // ... transposed
  }
}

// ------------------------------------------------------------ tridiagonal

// Forward elimination with partial pivoting of the tridiagonal part of S
// (sub l_i = S[i][i-1], diagonal d_i, super u_i = S[i][i+1]) applied to the
// right-hand sides in X (lane r: column col0 + r). The final upper
// triangular rows (d', u', w': the diagonal, the superdiagonal and the fill
// two to the right) go to coef[3 i ..]; workgroup 0 writes them, the others
// compute the same values. A zero pivot sets info[5].
template <typename T>
__global__ __launch_bounds__(64) void gtsv_forward_kernel(int64_t n, const T* __restrict__ S,
                                                          int64_t lds, T* X, int64_t ldx,
                                                          int64_t nrhs, T* coef, int32_t* info) {
  const int64_t col = int64_t(blockIdx.x) * 64 + threadIdx.x;
  const bool has = col < nrhs;
  T* x = X + std::min<int64_t>(col, nrhs - 1) * ldx;
  const bool writer = blockIdx.x == 0 && threadIdx.x == 0;
  // the current row i: (d, u, w) at columns i, i+1, i+2, and its rhs
  T d = S[0], u = n > 1 ? S[lds] : T(0), w = T(0);
  T b = x[0];
  bool singular = false;
  for (int64_t i = 0; i + 1 < n; ++i) {
    const T l1 = S[(i + 1) + i * lds];
    const T d1 = S[(i + 1) + (i + 1) * lds];
    const T u1 = i + 2 < n ? S[(i + 1) + (i + 2) * lds] : T(0);
    const T b1 = x[i + 1];
    T pd, pu, pw, pb, nd, nu, nb;
    if (fabs(d) >= fabs(l1)) {  // keep row i as the pivot row
      const T m = d != T(0) ? l1 / d : T(0);
      pd = d, pu = u, pw = w, pb = b;
      nd = d1 - m * u;
      nu = u1 - m * w;
      nb = b1 - m * b;
    } else {  // row i + 1 becomes the pivot row
      const T m = d / l1;
      pd = l1, pu = d1, pw = u1, pb = b1;
      nd = u - m * d1;
      nu = w - m * u1;
      nb = b - m * b1;
    }
    if (pd == T(0)) singular = true;
    if (writer) {
      coef[3 * i] = pd;
      coef[3 * i + 1] = pu;
      coef[3 * i + 2] = pw;
    }
    if (has) x[i] = pb;
    // the new current row i + 1: (nd, nu) at columns i + 1, i + 2 and no
    // fill at i + 3 yet
    d = nd;
    u = nu;
    w = T(0);
    b = nb;
  }
  if (d == T(0)) singular = true;
  if (writer) {
    coef[3 * (n - 1)] = d;
    coef[3 * (n - 1) + 1] = T(0);
    coef[3 * (n - 1) + 2] = T(0);
  }
  if (has) x[n - 1] = b;
  if (singular && threadIdx.x == 0 && blockIdx.x == 0) info[5] = 1;
}

// Back substitution with the rows coef: x_i = (b_i - u'_i x_{i+1} -
// w'_i x_{i+2}) / d'_i.
template <typename T>
__global__ __launch_bounds__(64) void gtsv_backward_kernel(int64_t n, const T* __restrict__ coef,
                                                           T* X, int64_t ldx, int64_t nrhs) {
  const int64_t col = int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (col >= nrhs) return;
  T* x = X + col * ldx;
  T x1 = T(0), x2 = T(0);
  for (int64_t i = n - 1; i >= 0; --i) {
    const T xi = (x[i] - coef[3 * i + 1] * x1 - coef[3 * i + 2] * x2) / coef[3 * i];
    x[i] = xi;
    x2 = x1;
    x1 = xi;
  }
}

// ------------------------------------------------------------- host side

template <typename T>
hipError_t gemm_t(int dtype, int mode, int ta, int tb, int64_t m, int64_t n, int64_t kk,
                  double alpha, const T* A, int64_t lda, const T* B, int64_t ldb, double beta,
                  T* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0 || kk <= 0) return hipSuccess;
  GemmConfig c = gemm_choose(dtype, 0, mode, m, n, kk);
  c.split = 1;
  return gemm_launch(dtype, 0, mode, ta, tb, m, n, kk, alpha, A, lda, B, ldb, beta, C, ldc,
                     nullptr, c, s);
}

template <typename T>
hipError_t copy_cols(T* dst, int64_t ldd, const T* src, int64_t lds, int64_t rows, int64_t cols,
                     hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  return hipMemcpy2DAsync(dst, size_t(ldd) * sizeof(T), src, size_t(lds) * sizeof(T),
                          size_t(rows) * sizeof(T), size_t(cols), hipMemcpyDeviceToDevice, s);
}

template <typename T>
hipError_t chol_factor_typed(int dtype, int64_t n, T* A, int64_t lda, T* inv, T* W,
                             int32_t* info, hipStream_t s) {
  const int64_t np = cdiv(n, kB);
  for (int64_t p = 0; p < np; ++p) {
    const int64_t k0 = p * kB;
    const int jb = int(std::min<int64_t>(kB, n - k0));
    T* invp = inv + p * kB * kB;
    hipLaunchKernelGGL((potrf_block_kernel<T>), dim3(1), dim3(kB), 0, s, A, lda, k0, jb, invp,
                       info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t m = n - k0 - jb;
    if (m <= 0) continue;
    T* a21 = A + (k0 + jb) + k0 * lda;
    // W = A21 L11^-T, then A21 = W and A22 -= W W^T (lower tiles, mirrored)
    e = gemm_t<T>(dtype, 0, 0, 1, m, jb, jb, 1.0, a21, lda, invp, kB, 0.0, W, m, s);
    if (e == hipSuccess) e = copy_cols<T>(a21, lda, W, m, m, jb, s);
    if (e == hipSuccess)
      e = gemm_t<T>(dtype, 1, 0, 1, m, m, jb, -1.0, W, m, W, m, 1.0,
                    A + (k0 + jb) + (k0 + jb) * lda, lda, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Forward L Y = B block by block (the inverse blocks of the non-unit lower
// factor), then back substitution U X = Y where U = L^T (chol) or, for a
// triangular matrix, only one of the two.
template <typename T>
hipError_t forward_typed(int dtype, int64_t n, int64_t r, const T* L, int64_t ldl,
                         const T* inv, T* Xin, int64_t ldx, T* Y, hipStream_t s) {
  const int64_t np = cdiv(n, kB);
  for (int64_t p = 0; p < np; ++p) {
    const int64_t r0 = p * kB;
    const int jb = int(std::min<int64_t>(kB, n - r0));
    hipError_t e = gemm_t<T>(dtype, 0, 0, 0, jb, r, jb, 1.0, inv + p * kB * kB, kB, Xin + r0, ldx,
                             0.0, Y + r0, n, s);
    if (e == hipSuccess)
      e = gemm_t<T>(dtype, 0, 0, 0, n - r0 - jb, r, jb, -1.0, L + (r0 + jb) + r0 * ldl, ldl, Y + r0,
                    n, 1.0, Xin + r0 + jb, ldx, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// U X = Y with U upper (upper = true: U stored in the upper triangle) or
// U = L^T (upper = false: L stored in the lower triangle, inverse blocks of
// L, so the blocks of U^-1 are their transposes).
template <typename T>
hipError_t backward_typed(int dtype, bool upper, int64_t n, int64_t r, const T* M, int64_t ldm,
                          const T* inv, T* Y, int64_t ldy, T* X, int64_t ldx, hipStream_t s) {
  const int64_t np = cdiv(n, kB);
  for (int64_t p = np - 1; p >= 0; --p) {
    const int64_t r0 = p * kB;
    const int jb = int(std::min<int64_t>(kB, n - r0));
    hipError_t e = gemm_t<T>(dtype, 0, upper ? 0 : 1, 0, jb, r, jb, 1.0, inv + p * kB * kB, kB,
                             Y + r0, ldy, 0.0, X + r0, ldx, s);
    if (e != hipSuccess) return e;
    if (r0 == 0) continue;
    // rows above: Y[0:r0] -= U[0:r0, r0:r0+jb] X_p
    if (upper)
      e = gemm_t<T>(dtype, 0, 0, 0, r0, r, jb, -1.0, M + r0 * ldm, ldm, X + r0, ldx, 1.0, Y, ldy, s);
    else  // U[0:r0, p] = (L[p, 0:r0])^T
      e = gemm_t<T>(dtype, 0, 1, 0, r0, r, jb, -1.0, M + r0, ldm, X + r0, ldx, 1.0, Y, ldy, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t struct_inv_bytes(int dtype, int64_t n) {
  return size_t(cdiv(std::max<int64_t>(n, 1), kB)) * kB * kB * (dtype == 0 ? 8 : 4);
}

hipError_t structure_launch(int dtype, int64_t n, const void* S, int64_t lds, int32_t* info,
                            hipStream_t s) {
  hipError_t e = fill_i32_launch(info, 16, 0, s);
  if (e != hipSuccess || n <= 0) return e;
  const int64_t nb = cdiv(n, kB);
  const unsigned tiles = unsigned(nb * (nb + 1) / 2);
  if (dtype == 0)
    hipLaunchKernelGGL((structure_kernel<double>), dim3(tiles), dim3(256), 0, s, n,
                       static_cast<const double*>(S), lds, info);
  else
    hipLaunchKernelGGL((structure_kernel<float>), dim3(tiles), dim3(256), 0, s, n,
                       static_cast<const float*>(S), lds, info);
  return hipGetLastError();
}

hipError_t chol_factor_launch(int dtype, int64_t n, void* A, int64_t lda, void* inv, void* W,
                              int32_t* info, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dtype == 0)
    return chol_factor_typed<double>(0, n, static_cast<double*>(A), lda,
                                     static_cast<double*>(inv), static_cast<double*>(W), info, s);
  return chol_factor_typed<float>(1, n, static_cast<float*>(A), lda, static_cast<float*>(inv),
                                  static_cast<float*>(W), info, s);
}

hipError_t trinv_launch(int dtype, bool lower, int64_t n, const void* S, int64_t lds, void* inv,
                        int32_t* info, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = unsigned(cdiv(n, kB));
  if (dtype == 0) {
    if (lower)
      hipLaunchKernelGGL((trinv_block_kernel<double, true>), dim3(nb), dim3(kB), 0, s,
                         static_cast<const double*>(S), lds, n, static_cast<double*>(inv), info);
    else
      hipLaunchKernelGGL((trinv_block_kernel<double, false>), dim3(nb), dim3(kB), 0, s,
                         static_cast<const double*>(S), lds, n, static_cast<double*>(inv), info);
  } else {
    if (lower)
      hipLaunchKernelGGL((trinv_block_kernel<float, true>), dim3(nb), dim3(kB), 0, s,
                         static_cast<const float*>(S), lds, n, static_cast<float*>(inv), info);
    else
      hipLaunchKernelGGL((trinv_block_kernel<float, false>), dim3(nb), dim3(kB), 0, s,
                         static_cast<const float*>(S), lds, n, static_cast<float*>(inv), info);
  }
  return hipGetLastError();
}

hipError_t tri_solve_launch(int dtype, int which, int64_t n, int64_t nrhs, const void* M,
                            int64_t ldm, const void* inv, void* B, int64_t ldb, void* Y,
                            void* X, int64_t ldx, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (dtype == 0) {
    const double* m = static_cast<const double*>(M);
    const double* iv = static_cast<const double*>(inv);
    double *b = static_cast<double*>(B), *y = static_cast<double*>(Y), *x = static_cast<double*>(X);
    hipError_t e = hipSuccess;
    if (which == 2) return backward_typed<double>(0, true, n, nrhs, m, ldm, iv, b, ldb, x, ldx, s);
    e = forward_typed<double>(0, n, nrhs, m, ldm, iv, b, ldb, y, s);
    if (e != hipSuccess) return e;
    if (which == 1) return copy_cols<double>(x, ldx, y, n, n, nrhs, s);
    return backward_typed<double>(0, false, n, nrhs, m, ldm, iv, y, n, x, ldx, s);
  }
  const float* m = static_cast<const float*>(M);
  const float* iv = static_cast<const float*>(inv);
  float *b = static_cast<float*>(B), *y = static_cast<float*>(Y), *x = static_cast<float*>(X);
  hipError_t e = hipSuccess;
  if (which == 2) return backward_typed<float>(1, true, n, nrhs, m, ldm, iv, b, ldb, x, ldx, s);
  e = forward_typed<float>(1, n, nrhs, m, ldm, iv, b, ldb, y, s);
  if (e != hipSuccess) return e;
  if (which == 1) return copy_cols<float>(x, ldx, y, n, n, nrhs, s);
  return backward_typed<float>(1, false, n, nrhs, m, ldm, iv, y, n, x, ldx, s);
}

hipError_t gtsv_launch(int dtype, int64_t n, int64_t nrhs, const void* S, int64_t lds, void* X,
                       int64_t ldx, void* coef, int32_t* info, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  const unsigned g = unsigned(cdiv(nrhs, 64));
  if (dtype == 0) {
    hipLaunchKernelGGL((gtsv_forward_kernel<double>), dim3(g), dim3(64), 0, s, n,
                       static_cast<const double*>(S), lds, static_cast<double*>(X), ldx, nrhs,
                       static_cast<double*>(coef), info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gtsv_backward_kernel<double>), dim3(g), dim3(64), 0, s, n,
                       static_cast<const double*>(coef), static_cast<double*>(X), ldx, nrhs);
  } else {
    hipLaunchKernelGGL((gtsv_forward_kernel<float>), dim3(g), dim3(64), 0, s, n,
                       static_cast<const float*>(S), lds, static_cast<float*>(X), ldx, nrhs,
                       static_cast<float*>(coef), info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gtsv_backward_kernel<float>), dim3(g), dim3(64), 0, s, n,
                       static_cast<const float*>(coef), static_cast<float*>(X), ldx, nrhs);
  }
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
