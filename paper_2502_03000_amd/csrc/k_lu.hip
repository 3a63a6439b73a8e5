// LU factorisation with partial pivoting and the triangular solves behind
// solve(A, B) and the inv(A)*B rewrite (the xGESV mapping of Sec. I / Sec. II;
// expression (9) of Sec. III).
//
// Right-looking blocked algorithm, panel width 64:
//   panel    one cooperative launch factors the n-k x jb panel. Each thread
//            holds one panel row in registers; per column the workgroups
//            publish their best pivot candidate (largest |a|, lowest row on
//            ties), meet at a grid barrier, and all pick the same winner.
//   laswp    the panel's row interchanges, as a gather of the moved rows, on
//            every column outside the panel and on the row-origin vector.
//   trsm     U12 = L11^-1 A12 (unit lower, 64 x 64 in LDS, one column/thread).
//   gemm     A22 -= L21 U12 on the MFMA GEMM.
// Grid barriers spin a bounded number of times; a timeout sets a status bit
// instead of hanging, and every wave still reaches the end of the kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ew_device.h"
#include "kernels.h"

namespace hexla {
namespace k {

namespace {

constexpr int kNB = 64;         // panel width
constexpr int kPT = 256;        // panel threads per workgroup (one row each)
constexpr int kSlot = kNB + 3;  // |a|, row, origin, row values
constexpr unsigned kSpinLimit = 1u << 20;
constexpr int kStatusSingular = 5;  // HEXLA_E_SINGULAR

struct LuWork {
  double* slots;       // [2][G][kSlot]
  double* diag;        // [2][kNB + 1]
  unsigned* barrier;   // [n_panels]
  int32_t* swap_cnt;   // [n_panels]
  int32_t* swap_list;  // [n_panels][2 * kNB][2]   (dst, src)
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

LuWork carve(void* work, int64_t n) {
  const int64_t np = cdiv(n, kNB);
  const int64_t gmax = cdiv(n, kPT);
  char* p = static_cast<char*>(work);
  LuWork w;
  w.slots = reinterpret_cast<double*>(p);
  p += size_t(2 * gmax * kSlot) * sizeof(double);
  w.diag = reinterpret_cast<double*>(p);
  p += size_t(2 * (kNB + 1)) * sizeof(double);
  w.barrier = reinterpret_cast<unsigned*>(p);
  p += size_t(np) * sizeof(unsigned);
  w.swap_cnt = reinterpret_cast<int32_t*>(p);
  p += size_t(np) * sizeof(int32_t);
  w.swap_list = reinterpret_cast<int32_t*>(p);
  return w;
}

__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier; the counter is monotonic within the launch. A wait longer
// than kSpinLimit polls, or an abort raised by another workgroup, makes it
// return false (for every thread of the workgroup) instead of waiting on.
__device__ bool grid_barrier(unsigned* counter, unsigned target, int* abort_flag, int* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit ||
          __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <typename T>
__global__ __launch_bounds__(kPT) void panel_kernel(T* __restrict__ A, int64_t lda, int64_t n,
                                                    int64_t k, int jb, int G, double* slots,
                                                    double* diag, unsigned* barrier,
                                                    int32_t* swap_cnt, int32_t* swap_list,
                                                    int32_t* status) {
  __shared__ double s_abs[kPT / 64];
  __shared__ int64_t s_row[kPT / 64];
  __shared__ double s_gabs[kPT];
  __shared__ int64_t s_grow[kPT];
  __shared__ T s_piv[kNB];
  __shared__ T s_dia[kNB];
  __shared__ int s_win, s_pdi_origin, s_piv_origin, s_flag, s_ok;
  __shared__ int64_t s_prow, s_best;

  const int g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t mp = n - k;
  const int64_t r = int64_t(g) * kPT + tid;  // panel row of this thread
  const bool own = r < mp;
  // a barrier timed out in an earlier panel: the factorisation is void, exit
  if (__hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  T v[kNB];
  int origin = int(r);  // panel row this content held before the panel
#pragma unroll
  for (int c = 0; c < kNB; ++c) v[c] = (own && c < jb) ? A[(k + r) + (k + c) * lda] : T(0);
  if (tid == 0) s_ok = 1;

#pragma unroll 1
  for (int j = 0; j < jb; ++j) {
    {
      // 1. local candidate: largest |a_rj| over rows r >= j, lowest row on ties
      double a = -1.0;
      int64_t idx = int64_t(1) << 40;  // no candidate
      T vj = T(0);  // v[j] without a dynamic register index
#pragma unroll
      for (int c = 0; c < kNB; ++c) vj = (c == j) ? v[c] : vj;
      if (own && r >= j) {
        a = fabs(double(vj));
        idx = r;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double a2 = __shfl_xor(a, off, 64);
        const int64_t i2 = __shfl_xor(idx, off, 64);
        if (a2 > a || (a2 == a && i2 < idx)) {
          a = a2;
          idx = i2;
        }
      }
      if (lane == 0) {
        s_abs[wave] = a;
        s_row[wave] = idx;
      }
      __syncthreads();
      if (tid == 0) {
        double ba = s_abs[0];
        int64_t bi = s_row[0];
        for (int q = 1; q < kPT / 64; ++q)
          if (s_abs[q] > ba || (s_abs[q] == ba && s_row[q] < bi)) {
            ba = s_abs[q];
            bi = s_row[q];
          }
        s_best = bi;
        double* slot = slots + (size_t((j & 1) * G + g)) * kSlot;
        st_agent(slot + 0, ba);
        st_agent(slot + 1, double(bi));
      }
      __syncthreads();
      // 2. publish the candidate row and the current row j
      const int64_t best = s_best;
      if (own && r == best) {
        double* slot = slots + (size_t((j & 1) * G + g)) * kSlot;
        st_agent(slot + 2, double(origin));
#pragma unroll
        for (int c = 0; c < kNB; ++c)
          if (c < jb) st_agent(slot + 3 + c, double(v[c]));
        __threadfence();
      }
      if (own && r == j) {
        double* d = diag + (j & 1) * (kNB + 1);
        st_agent(d + kNB, double(origin));
#pragma unroll
        for (int c = 0; c < kNB; ++c)
          if (c < jb) st_agent(d + c, double(v[c]));
        __threadfence();
      }
      if (tid == 0) __threadfence();
      if (!grid_barrier(barrier, unsigned(G) * unsigned(j + 1), status + 1, &s_flag)) {
        if (tid == 0) s_ok = 0;
        break;  // every thread of the workgroup sees the same flag
      }
      // 3. every workgroup picks the same winner
      for (int q = tid; q < G; q += kPT) {
        const double* slot = slots + (size_t((j & 1) * G + q)) * kSlot;
        s_gabs[q] = ld_agent(slot + 0);
        s_grow[q] = int64_t(ld_agent(slot + 1));
      }
      __syncthreads();
      if (tid == 0) {
        int w = 0;
        for (int q = 1; q < G; ++q)
          if (s_gabs[q] > s_gabs[w] || (s_gabs[q] == s_gabs[w] && s_grow[q] < s_grow[w])) w = q;
        s_win = w;
        s_prow = s_grow[w];
      }
      __syncthreads();
      {
        const double* slot = slots + (size_t((j & 1) * G + s_win)) * kSlot;
        const double* d = diag + (j & 1) * (kNB + 1);
        if (tid < jb) {
          s_piv[tid] = T(ld_agent(slot + 3 + tid));
          s_dia[tid] = T(ld_agent(d + tid));
        }
        if (tid == kNB) {
          s_piv_origin = int(ld_agent(slot + 2));
          s_pdi_origin = int(ld_agent(d + kNB));
        }
      }
      __syncthreads();
      const int64_t prow = s_prow;
      const T pivot = s_piv[j];
      if (g == 0 && tid == 0 && pivot == T(0)) {
        const int col = int(k + j);
        if (atomicCAS(status, 0, kStatusSingular) == 0) status[2] = col;
      }
      // 4. interchange rows j and prow
      if (prow != j && own) {
        if (r == j) {
#pragma unroll
          for (int c = 0; c < kNB; ++c)
            if (c < jb) v[c] = s_piv[c];
          origin = s_piv_origin;
        } else if (r == prow) {
#pragma unroll
          for (int c = 0; c < kNB; ++c)
            if (c < jb) v[c] = s_dia[c];
          origin = s_pdi_origin;
        }
      }
      // 5. eliminate below the pivot
      if (own && r > j && pivot != T(0)) {
        T cur = T(0);
#pragma unroll
        for (int c = 0; c < kNB; ++c) cur = (c == j) ? v[c] : cur;
        const T l = cur / pivot;
#pragma unroll
        for (int c = 0; c < kNB; ++c) {
          if (c == j) v[c] = l;
          else if (c > j && c < jb) v[c] -= l * s_piv[c];
        }
      }
      __syncthreads();
    }
  }

  __syncthreads();
  if (!s_ok) {  // barrier timeout: leave the panel as it is, flag the failure
    if (tid == 0) atomicOr(status + 1, 1);
    return;
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < kNB; ++c)
      if (c < jb) A[(k + r) + (k + c) * lda] = v[c];
    if (origin != int(r)) {
      const int e = atomicAdd(swap_cnt, 1);
      if (e < 2 * kNB) {
        swap_list[2 * e] = int(k + r);
        swap_list[2 * e + 1] = int(k + origin);
      }
    }
  }
}

// Gather of the moved rows on the columns outside the panel; column index n
// stands for the row-origin vector. One wave per column.
template <typename T>
__global__ __launch_bounds__(256) void laswp_kernel(T* __restrict__ A, int64_t lda, int64_t n,
                                                    int64_t k, int jb, const int32_t* swap_cnt,
                                                    const int32_t* swap_list, int32_t* rowid) {
  const int lane = threadIdx.x & 63;
  int64_t c = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (c >= n - jb + 1) return;
  if (c >= k) c += jb;  // skip the panel's own columns; c == n is rowid
  const int cnt = min(*swap_cnt, 2 * kNB);
  if (c == n) {
    int32_t a0 = 0, a1 = 0;
    if (lane < cnt) a0 = rowid[swap_list[2 * lane + 1]];
    if (lane + 64 < cnt) a1 = rowid[swap_list[2 * (lane + 64) + 1]];
    __builtin_amdgcn_wave_barrier();
    if (lane < cnt) rowid[swap_list[2 * lane]] = a0;
    if (lane + 64 < cnt) rowid[swap_list[2 * (lane + 64)]] = a1;
    return;
  }
  T* col = A + c * lda;
  T a0 = 0, a1 = 0;
  if (lane < cnt) a0 = col[swap_list[2 * lane + 1]];
  if (lane + 64 < cnt) a1 = col[swap_list[2 * (lane + 64) + 1]];
  __builtin_amdgcn_wave_barrier();
  if (lane < cnt) col[swap_list[2 * lane]] = a0;
  if (lane + 64 < cnt) col[swap_list[2 * (lane + 64)]] = a1;
}

// X = L^-1 X for a jb x jb unit-lower block L (at L0, ldl) and columns of X
// (at X0, ldx): one thread per column, block in LDS.
template <typename T>
__global__ __launch_bounds__(256) void trsm_lower_unit_kernel(const T* __restrict__ L0,
                                                              int64_t ldl, T* __restrict__ X0,
                                                              int64_t ldx, int jb, int64_t ncols) {
  __shared__ T Ls[kNB][kNB + 1];
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int i = e % kNB, j = e / kNB;
    Ls[i][j] = (i < jb && j < jb) ? L0[i + j * ldl] : T(0);
  }
  __syncthreads();
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ncols) return;
  T* x = X0 + c * ldx;
  T v[kNB];
#pragma unroll
  for (int i = 0; i < kNB; ++i) v[i] = (i < jb) ? x[i] : T(0);
  // column-oriented substitution; inner loops are static so v stays in registers
#pragma unroll 1
  for (int l = 0; l < jb - 1; ++l) {
    T xl = T(0);
#pragma unroll
    for (int i = 0; i < kNB; ++i) xl = (i == l) ? v[i] : xl;
#pragma unroll
    for (int i = 0; i < kNB; ++i)
      if (i > l) v[i] -= Ls[i][l] * xl;
  }
#pragma unroll
  for (int i = 0; i < kNB; ++i)
    if (i < jb) x[i] = v[i];
}

// X = U^-1 X for a jb x jb upper block U (non-unit diagonal).
template <typename T>
__global__ __launch_bounds__(256) void trsm_upper_kernel(const T* __restrict__ U0, int64_t ldu,
                                                         T* __restrict__ X0, int64_t ldx, int jb,
                                                         int64_t ncols) {
  __shared__ T Us[kNB][kNB + 1];
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int i = e % kNB, j = e / kNB;
    Us[i][j] = (i < jb && j < jb) ? U0[i + j * ldu] : T(i == j ? 1 : 0);
  }
  __syncthreads();
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ncols) return;
  T* x = X0 + c * ldx;
  T v[kNB];
#pragma unroll
  for (int i = 0; i < kNB; ++i) v[i] = (i < jb) ? x[i] : T(0);
#pragma unroll 1
  for (int l = jb - 1; l >= 0; --l) {
    T xl = T(0);
#pragma unroll
    for (int i = 0; i < kNB; ++i) xl = (i == l) ? v[i] : xl;
    xl = xl / Us[l][l];
#pragma unroll
    for (int i = 0; i < kNB; ++i) {
      if (i == l) v[i] = xl;
      else if (i < l) v[i] -= Us[i][l] * xl;
    }
  }
#pragma unroll
  for (int i = 0; i < kNB; ++i)
    if (i < jb) x[i] = v[i];
}

template <typename T>
__global__ void gather_rows_kernel(const T* __restrict__ B, int64_t ldb, const int32_t* rowid,
                                   T* __restrict__ X, int64_t ldx, int64_t n, int64_t nrhs) {
  const int64_t total = n * nrhs;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % n, c = e / n;
    X[i + c * ldx] = B[rowid[i] + c * ldb];
  }
}

__global__ void iota_kernel(int32_t* p, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = int32_t(i);
}

// C (m x ncol) -= A (m x kk) * B (kk x ncol), through GEMM or GEMV.
template <typename T>
hipError_t update(int dtype, int64_t m, int64_t ncol, int64_t kk, const T* A, int64_t lda,
                  const T* B, int64_t ldb, T* C, int64_t ldc, hipStream_t s, int prec = 0) {
  if (m <= 0 || ncol <= 0 || kk <= 0) return hipSuccess;
  if (ncol == 1) {
    EwProgram epi{};
    epi.n_instr = 3;
    epi.n_leaf = 1;
    epi.rows = m;
    epi.cols = 1;
    epi.op[0] = EW_EXTRA;
    epi.op[1] = EW_LEAF;
    epi.arg[1] = 0;
    epi.op[2] = EW_ADD;
    epi.leaf[0].ptr = C;
    epi.leaf[0].si = 1;
    epi.leaf[0].sj = ldc;
    return gemv_launch(dtype, 0, m, kk, -1.0, A, lda, B, 1, C, 1, &epi, s);
  }
  GemmConfig cfg = gemm_choose(dtype, prec, 0, m, ncol, kk);
  cfg.split = 1;
  return gemm_launch(dtype, prec, 0, 0, 0, m, ncol, kk, -1.0, A, lda, B, ldb, 1.0, C, ldc,
                     nullptr, cfg, s);
}

template <typename T>
hipError_t factor_typed(int dtype, int64_t n, T* A, int64_t lda, int32_t* rowid, void* work,
                        int32_t* status, hipStream_t s, int prec) {
  if (n == 0) return hipSuccess;
  const int64_t np = cdiv(n, kNB);
  LuWork w = carve(work, n);
  hipError_t e = fill_i32_launch(reinterpret_cast<int32_t*>(w.barrier), 2 * np, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(iota_kernel, dim3(unsigned(std::min<int64_t>(cdiv(n, 256), 1024))), dim3(256),
                     0, s, rowid, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t k = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - k));
    const int G = int(cdiv(n - k, kPT));
    int32_t* list = w.swap_list + p * (4 * kNB);
    hipLaunchKernelGGL((panel_kernel<T>), dim3(G), dim3(kPT), 0, s, A, lda, n, k, jb, G, w.slots,
                       w.diag, w.barrier + p, w.swap_cnt + p, list, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t cols = n - jb + 1;
    hipLaunchKernelGGL((laswp_kernel<T>), dim3(unsigned(cdiv(cols, 4))), dim3(256), 0, s, A, lda,
                       n, k, jb, w.swap_cnt + p, list, rowid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t right = n - k - jb;
    if (right > 0) {
      T* a11 = A + k + k * lda;
      T* a12 = A + k + (k + jb) * lda;
      hipLaunchKernelGGL((trsm_lower_unit_kernel<T>), dim3(unsigned(cdiv(right, 256))), dim3(256),
                         0, s, a11, lda, a12, lda, jb, right);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      e = update<T>(dtype, n - k - jb, right, jb, A + (k + jb) + k * lda, lda, a12, lda,
                    A + (k + jb) + (k + jb) * lda, lda, s, prec);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename T>
hipError_t solve_typed(int dtype, int64_t n, int64_t nrhs, const T* LU, int64_t lda,
                       const int32_t* rowid, const T* B, int64_t ldb, T* X, int64_t ldx,
                       hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL((gather_rows_kernel<T>), dim3(unsigned(std::min<int64_t>(cdiv(n * nrhs, 256), 2048))),
                     dim3(256), 0, s, B, ldb, rowid, X, ldx, n, nrhs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t np = cdiv(n, kNB);
  const unsigned gx = unsigned(cdiv(nrhs, 256));
  for (int64_t p = 0; p < np; ++p) {  // forward: L y = P b
    const int64_t r0 = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - r0));
    hipLaunchKernelGGL((trsm_lower_unit_kernel<T>), dim3(gx), dim3(256), 0, s, LU + r0 + r0 * lda,
                       lda, X + r0, ldx, jb, nrhs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = update<T>(dtype, n - r0 - jb, nrhs, jb, LU + (r0 + jb) + r0 * lda, lda, X + r0, ldx,
                  X + r0 + jb, ldx, s);
    if (e != hipSuccess) return e;
  }
  for (int64_t p = np - 1; p >= 0; --p) {  // backward: U x = y
    const int64_t r0 = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - r0));
    hipLaunchKernelGGL((trsm_upper_kernel<T>), dim3(gx), dim3(256), 0, s, LU + r0 + r0 * lda, lda,
                       X + r0, ldx, jb, nrhs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = update<T>(dtype, r0, nrhs, jb, LU + r0 * lda, lda, X + r0, ldx, X, ldx, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t lu_workspace_bytes(int, int64_t n) {
  const int64_t np = cdiv(std::max<int64_t>(n, 1), kNB);
  const int64_t gmax = cdiv(std::max<int64_t>(n, 1), kPT);
  size_t b = size_t(2 * gmax * kSlot) * sizeof(double);
  b += size_t(2 * (kNB + 1)) * sizeof(double);
  b += size_t(np) * (sizeof(unsigned) + sizeof(int32_t));
  b += size_t(np) * 4 * kNB * sizeof(int32_t);
  return (b + 255) & ~size_t(255);
}

hipError_t lu_factor_launch(int dtype, int64_t n, void* A, int64_t lda, int32_t* rowid,
                            void* work, int32_t* status, hipStream_t s, int update_precision) {
  return dtype == 0
             ? factor_typed<double>(0, n, static_cast<double*>(A), lda, rowid, work, status, s, 0)
             : factor_typed<float>(1, n, static_cast<float*>(A), lda, rowid, work, status, s,
                                   update_precision);
}

hipError_t lu_solve_launch(int dtype, int64_t n, int64_t nrhs, const void* LU, int64_t lda,
                           const int32_t* rowid, const void* B, int64_t ldb, void* X, int64_t ldx,
                           hipStream_t s) {
  return dtype == 0
             ? solve_typed<double>(0, n, nrhs, static_cast<const double*>(LU), lda, rowid,
                                   static_cast<const double*>(B), ldb, static_cast<double*>(X), ldx, s)
             : solve_typed<float>(1, n, nrhs, static_cast<const float*>(LU), lda, rowid,
                                  static_cast<const float*>(B), ldb, static_cast<float*>(X), ldx, s);
}

}  // namespace k
}  // namespace hexla
