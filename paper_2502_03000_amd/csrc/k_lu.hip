// LU factorisation with partial pivoting and the triangular solves behind
// solve(A, B) and the inv(A)*B rewrite (the xGESV mapping of Sec. I / Sec. II;
// expression (9) of Sec. III).
//
// Right-looking blocked algorithm, panel width 64:
//   panel    one launch factors the n-k x jb panel. Each thread holds one
//            panel row in registers; per column the workgroups publish their
//            best pivot candidate (largest |a|, lowest row on ties) with its
//            row, meet at one grid barrier, read every candidate in one round
//            trip and all pick the same winner. The participants share one
//            XCD when there are at most 32.
//   laswp    the panel's row interchanges, as a gather of the moved rows, on
//            every column outside the panel and on the row-origin vector.
//   trsm     U12 = L11^-1 A12 as an in-place product with the explicit
//            inverse of the 64 x 64 unit lower block (MFMA GEMM).
//   gemm     A22 -= L21 U12 on the MFMA GEMM.
// The solves apply the inverses of the diagonal blocks (kept in the
// workspace) and update the remaining rows with GEMM.
// Grid barriers spin a bounded number of times; a timeout sets a status bit
// instead of hanging, and every wave still reaches the end of the kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ew_device.h"
#include "kernels.h"
#include "wave_device.h"

namespace hexla {
namespace k {

namespace {

constexpr int kNB = 64;         // panel width
constexpr int kPT = 256;        // panel threads per workgroup (one row each)
constexpr int kSlot = kNB + 3;  // |a|, row, origin, row values
constexpr int kMaxG = 64;       // panel workgroups (rows up to kMaxG * kPT)
constexpr unsigned kSpinLimit = 1u << 20;
constexpr int kStatusSingular = 5;  // HEXLA_E_SINGULAR

struct LuWork {
  void* inv;           // [n_panels][2][kNB][kNB]: L11^-1 and U11^-1 of each diagonal block
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
  w.inv = p;
  p += size_t(np) * 2 * kNB * kNB * sizeof(double);
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

// Waits until every vector memory operation of this thread has completed
// (stores acknowledged), so that relaxed agent-scope stores issued before it
// are visible to any agent-scope load that follows a later signal.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Grid barrier among the G participants; the counter is monotonic within the
// launch. Each thread's agent-scope stores are complete before the
// workgroup's arrival is counted. A wait longer than kSpinLimit polls, or an
// abort raised by another workgroup, makes it return false (for every thread
// of the workgroup) instead of waiting on.
__device__ bool grid_barrier(unsigned* counter, unsigned target, int* abort_flag, int* s_flag) {
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
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

// Panel factorisation. Participants are the workgroups with blockIdx a
// multiple of `stride` (8 places them on one XCD, where the barrier and the
// exchange stay within one L2); the others return at once. Each thread holds
// one panel row in registers, kept rotated so that the current column is
// always v[0]: after step j every row turns left by one, and a row still
// below the pivot appends its multiplier l_j where column j left, while a
// finished row appends column j itself. All register indices are static.
// After jb steps every row is rotated by jb, so v[c] belongs to column
// (c + jb) mod kNB. Per column: every workgroup publishes its best candidate
// (largest |a|, lowest row on ties) with the candidate's row and origin,
// the owner of row j publishes row j, all meet at one barrier, and every
// workgroup reads all candidates in one round trip and picks the same winner.
template <typename T>
__global__ __launch_bounds__(kPT) void panel_kernel(T* __restrict__ A, int64_t lda, int64_t n,
                                                    int64_t k, int jb, int G, int stride,
                                                    double* slots, double* diag,
                                                    unsigned* barrier, int32_t* swap_cnt,
                                                    int32_t* swap_list, int32_t* status) {
  if (blockIdx.x % stride) return;  // not a participant
  __shared__ double s_abs[kPT / 64];
  __shared__ int s_row[kPT / 64];
  __shared__ double s_pub[kNB + 1], s_pubj[kNB + 1];  // rows staged for publishing
  __shared__ double s_cand[kMaxG * kSlot];
  __shared__ double s_dia[kNB + 1];
  __shared__ T s_prow[kNB];  // pivot row, rotated, with its multiplier part zeroed
  __shared__ int s_win, s_flag, s_ok;

  const int g = blockIdx.x / stride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mp = int(n - k);
  const int r = g * kPT + tid;  // panel row of this thread
  const bool own = r < mp;
  // a barrier timed out in an earlier panel: the factorisation is void, exit
  if (__hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  T v[kNB];
  int origin = r;  // panel row this content held before the panel
#pragma unroll
  for (int c = 0; c < kNB; ++c) v[c] = (own && c < jb) ? A[(k + r) + (k + c) * lda] : T(0);
  if (tid == 0) s_ok = 1;

#pragma unroll 1
  for (int j = 0; j < jb; ++j) {
    double* slot_base = slots + size_t(j & 1) * G * kSlot;
    double* d = diag + (j & 1) * (kNB + 1);
    // 1. local candidate: largest |a_rj| over rows r >= j, lowest row on ties
    double ba = -1.0;
    int bi = 1 << 30;  // no candidate
    {
      double a = -1.0;
      int idx = 1 << 30;
      if (own && r >= j && v[0] == v[0]) {  // NaN is never a candidate
        a = fabs(double(v[0]));
        idx = r;
      }
      wave_argmax(a, idx);
      if (lane == 0) {
        s_abs[wave] = a;
        s_row[wave] = idx;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPT / 64; ++q)
        if (s_abs[q] > ba || (s_abs[q] == ba && s_row[q] < bi)) {
          ba = s_abs[q];
          bi = s_row[q];
        }
    }
    // 2. publish the candidate and row j (rotated rows): their owners stage
    // them in LDS, then one wave stores each with one instruction per field
    const bool owns_j = j / kPT == g;
    if (own && r == bi) {
#pragma unroll
      for (int c = 0; c < kNB; ++c) s_pub[c] = double(v[c]);
      s_pub[kNB] = double(origin);
    }
    if (own && r == j) {
#pragma unroll
      for (int c = 0; c < kNB; ++c) s_pubj[c] = double(v[c]);
      s_pubj[kNB] = double(origin);
    }
    __syncthreads();
    if (wave == 0) {
      double* slot = slot_base + size_t(g) * kSlot;
      st_agent(slot + 3 + lane, s_pub[lane]);
      if (lane == 0) {
        st_agent(slot + 0, ba);
        st_agent(slot + 1, double(bi));
        st_agent(slot + 2, s_pub[kNB]);
      }
    } else if (wave == 1 && owns_j) {
      st_agent(d + lane, s_pubj[lane]);
      if (lane == 0) st_agent(d + kNB, s_pubj[kNB]);
    }
    if (!grid_barrier(barrier, unsigned(G) * unsigned(j + 1), status + 1, &s_flag)) {
      if (tid == 0) s_ok = 0;
      break;  // every thread of the workgroup sees the same flag
    }
    // 3. all candidates and row j in one round trip
    for (int e = tid; e < G * kSlot; e += kPT) s_cand[e] = ld_agent(slot_base + e);
    if (tid <= kNB) s_dia[tid] = ld_agent(d + tid);
    __syncthreads();
    // 4. every workgroup picks the same winner (G <= 64: one lane each)
    if (wave == 0) {
      double a = lane < G ? s_cand[lane * kSlot + 0] : -2.0;
      int idx = lane < G ? int(s_cand[lane * kSlot + 1]) : (1 << 30);
      wave_argmax(a, idx);
      int w = idx / kPT;  // the workgroup that published row idx
      w = a >= 0.0 ? w : -1;  // -1: no comparable candidate
      if (lane == 0) s_win = w;
      // the pivot row for the elimination: rotated like every row, with the
      // multipliers it carries (positions >= kNB - j) zeroed
      const double* src = w >= 0 ? s_cand + w * kSlot + 3 : s_dia;
      s_prow[lane] = lane < kNB - j ? T(src[lane]) : T(0);
    }
    __syncthreads();
    const int win = s_win;
    const int prow = win >= 0 ? int(s_cand[win * kSlot + 1]) : j;
    const T pivot = s_prow[0];
    if (g == 0 && tid == 0 && !(pivot != T(0) && win >= 0)) {
      const int col = int(k + j);
      if (atomicCAS(status, 0, kStatusSingular) == 0) status[2] = col;
    }
    // 5. interchange rows j and prow (whole rotated rows)
    if (prow != j && own) {
      if (r == j) {
        const double* src = s_cand + win * kSlot;
#pragma unroll
        for (int c = 0; c < kNB; ++c) v[c] = T(src[3 + c]);
        origin = int(src[2]);
      } else if (r == prow) {
#pragma unroll
        for (int c = 0; c < kNB; ++c) v[c] = T(s_dia[c]);
        origin = int(s_dia[kNB]);
      }
    }
    // 6. eliminate below the pivot, then rotate
    const bool active = own && r > j && pivot != T(0);
    const T l = active ? v[0] / pivot : T(0);
#pragma unroll
    for (int c = 1; c < kNB; ++c) v[c] -= l * s_prow[c];
    const T last = active ? l : v[0];
#pragma unroll
    for (int c = 0; c < kNB - 1; ++c) v[c] = v[c + 1];
    v[kNB - 1] = last;
    __syncthreads();
  }

  __syncthreads();
  if (!s_ok) {  // barrier timeout: leave the panel as it is, flag the failure
    if (tid == 0) atomicOr(status + 1, 1);
    return;
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
      const int col = (c + jb) % kNB;  // every row is rotated by jb
      if (col < jb) A[(k + r) + (k + col) * lda] = v[c];
    }
    if (origin != r) {
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

// Inverses of the diagonal blocks (jb x jb, padded to kNB x kNB with the
// identity), one thread per column, the block in LDS and the column in
// registers: L11^-1 (unit lower, forward substitution) for the panel's
// triangular solve and the forward solve, U11^-1 (backward substitution)
// for the backward solve. block p of the grid takes rows/columns p * kNB.
template <typename T, bool UPPER>
__global__ __launch_bounds__(kNB) void inv_block_kernel(const T* __restrict__ A, int64_t lda,
                                                        int64_t n, int64_t first_block,
                                                        T* __restrict__ inv) {
  __shared__ T Ls[kNB][kNB + 1];
  const int64_t p = first_block + blockIdx.x;
  const int64_t k = p * kNB;
  const int jb = int(std::min<int64_t>(kNB, n - k));
  for (int e = threadIdx.x; e < kNB * kNB; e += kNB) {
    const int i = e % kNB, j = e / kNB;
    Ls[i][j] = (i < jb && j < jb) ? A[(k + i) + (k + j) * lda] : T(i == j ? 1 : 0);
  }
  __syncthreads();
  const int c = threadIdx.x;
  T x[kNB];
  if (!UPPER) {
#pragma unroll
    for (int i = 0; i < kNB; ++i) {
      T s = i == c ? T(1) : T(0);
#pragma unroll
      for (int l = 0; l < i; ++l) s -= Ls[i][l] * x[l];
      x[i] = s;
    }
  } else {
#pragma unroll
    for (int i = kNB - 1; i >= 0; --i) {
      T s = i == c ? T(1) : T(0);
#pragma unroll
      for (int l = i + 1; l < kNB; ++l) s -= Ls[i][l] * x[l];
      x[i] = s / Ls[i][i];
    }
  }
  T* out = inv + size_t(p) * 2 * kNB * kNB + (UPPER ? kNB * kNB : 0);
#pragma unroll
  for (int i = 0; i < kNB; ++i) out[i + c * kNB] = x[i];
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

// A second stream for the lookahead: the trailing update beyond the next
// panel's columns runs there while the next panel is factored. Default
// priority, like the caller's stream; released when the factorization has
// been issued (its work completes first).
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
  hipError_t open() {
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    return e;
  }
  ~SideStream() {
    if (done) (void)hipEventDestroy(done);
    if (ready) (void)hipEventDestroy(ready);
    if (s) (void)hipStreamDestroy(s);
  }
};

template <typename T>
hipError_t factor_typed(int dtype, int64_t n, T* A, int64_t lda, int32_t* rowid, void* work,
                        int32_t* status, hipStream_t s, int prec) {
  if (n == 0) return hipSuccess;
  if (n > kLuMaxN) return hipErrorInvalidValue;
  const int64_t np = cdiv(n, kNB);
  LuWork w = carve(work, n);
  // Lookahead from three panels on, outside graph capture (a captured
  // sequence stays on one stream).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t ce = hipStreamIsCapturing(s, &cap);
  if (ce != hipSuccess) return ce;
  SideStream side;
  const bool lookahead = np >= 3 && cap == hipStreamCaptureStatusNone;
  if (lookahead && (ce = side.open()) != hipSuccess) return ce;
  bool pending = false;  // the side stream holds an update the next interchanges must wait for
  hipError_t e = fill_i32_launch(reinterpret_cast<int32_t*>(w.barrier), 2 * np, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(iota_kernel, dim3(unsigned(std::min<int64_t>(cdiv(n, 256), 1024))), dim3(256),
                     0, s, rowid, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t k = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - k));
    const int G = int(cdiv(n - k, kPT));
    // up to 32 participants share one XCD (every 8th workgroup id)
    const int stride = G <= 32 ? 8 : 1;
    int32_t* list = w.swap_list + p * (4 * kNB);
    hipLaunchKernelGGL((panel_kernel<T>), dim3(G * stride), dim3(kPT), 0, s, A, lda, n, k, jb, G,
                       stride, w.slots, w.diag, w.barrier + p, w.swap_cnt + p, list, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pending) {  // the interchanges touch the columns the side stream updates
      if ((e = hipStreamWaitEvent(s, side.done, 0)) != hipSuccess) return e;
      pending = false;
    }
    const int64_t cols = n - jb + 1;
    hipLaunchKernelGGL((laswp_kernel<T>), dim3(unsigned(cdiv(cols, 4))), dim3(256), 0, s, A, lda,
                       n, k, jb, w.swap_cnt + p, list, rowid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t right = n - k - jb;
    if (right > 0) {
      T* a12 = A + k + (k + jb) * lda;
      // U12 = L11^-1 A12 as a product with the explicit inverse, in place:
      // a tile's workgroup (BM >= kNB rows, no split) reads all of its
      // columns of A12 before it writes them, and no other workgroup reads them
      T* linv = static_cast<T*>(w.inv) + size_t(p) * 2 * kNB * kNB;
      hipLaunchKernelGGL((inv_block_kernel<T, false>), dim3(1), dim3(kNB), 0, s, A, lda, n, p,
                         static_cast<T*>(w.inv));
      if ((e = hipGetLastError()) != hipSuccess) return e;
      GemmConfig tc = gemm_choose(dtype, 0, 0, jb, right, jb);
      tc.split = 1;
      e = gemm_launch(dtype, 0, 0, 0, 0, jb, right, jb, 1.0, linv, kNB, a12, lda, 0.0, a12, lda,
                      nullptr, tc, s);
      if (e != hipSuccess) return e;
      // A22 -= L21 U12: the next panel's columns on s, so that the next
      // panel starts at once; with lookahead the rest on the side stream
      const int64_t near = lookahead ? std::min<int64_t>(kNB, right) : right;
      if (near < right) {
        if ((e = hipEventRecord(side.ready, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(side.s, side.ready, 0)) != hipSuccess) return e;
      }
      e = update<T>(dtype, n - k - jb, near, jb, A + (k + jb) + k * lda, lda, a12, lda,
                    A + (k + jb) + (k + jb) * lda, lda, s, prec);
      if (e != hipSuccess) return e;
      if (near < right) {
        e = update<T>(dtype, n - k - jb, right - near, jb, A + (k + jb) + k * lda, lda,
                      a12 + near * lda, lda, A + (k + jb) + (k + jb + near) * lda, lda, side.s,
                      prec);
        if (e != hipSuccess) return e;
        if ((e = hipEventRecord(side.done, side.s)) != hipSuccess) return e;
        pending = true;
      }
    }
  }
  if (pending && (e = hipStreamWaitEvent(s, side.done, 0)) != hipSuccess) return e;
  // the last block's L11^-1 (no update followed it) and every U11^-1, for the solves
  hipLaunchKernelGGL((inv_block_kernel<T, false>), dim3(1), dim3(kNB), 0, s, A, lda, n, np - 1,
                     static_cast<T*>(w.inv));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((inv_block_kernel<T, true>), dim3(unsigned(np)), dim3(kNB), 0, s, A, lda, n,
                     int64_t(0), static_cast<T*>(w.inv));
  return hipGetLastError();
}

// x <- (diagonal block inverse) x, in place (same argument as the panel's
// triangular solve: BM >= kNB covers every row, no split-K).
template <typename T>
hipError_t apply_inverse(int dtype, int jb, int64_t nrhs, const T* inv, T* X, int64_t ldx,
                         hipStream_t s) {
  GemmConfig c = gemm_choose(dtype, 0, 0, jb, nrhs, jb);
  c.split = 1;
  return gemm_launch(dtype, 0, 0, 0, 0, jb, nrhs, jb, 1.0, inv, kNB, X, ldx, 0.0, X, ldx, nullptr,
                     c, s);
}

template <typename T>
hipError_t solve_typed(int dtype, int64_t n, int64_t nrhs, const T* LU, int64_t lda,
                       const int32_t* rowid, const void* work, const T* B, int64_t ldb, T* X,
                       int64_t ldx, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL((gather_rows_kernel<T>), dim3(unsigned(std::min<int64_t>(cdiv(n * nrhs, 256), 2048))),
                     dim3(256), 0, s, B, ldb, rowid, X, ldx, n, nrhs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t np = cdiv(n, kNB);
  const T* inv = static_cast<const T*>(work);  // the carve() places the inverses first
  for (int64_t p = 0; p < np; ++p) {  // forward: L y = P b
    const int64_t r0 = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - r0));
    e = apply_inverse<T>(dtype, jb, nrhs, inv + size_t(p) * 2 * kNB * kNB, X + r0, ldx, s);
    if (e != hipSuccess) return e;
    e = update<T>(dtype, n - r0 - jb, nrhs, jb, LU + (r0 + jb) + r0 * lda, lda, X + r0, ldx,
                  X + r0 + jb, ldx, s);
    if (e != hipSuccess) return e;
  }
  for (int64_t p = np - 1; p >= 0; --p) {  // backward: U x = y
    const int64_t r0 = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - r0));
    e = apply_inverse<T>(dtype, jb, nrhs, inv + size_t(p) * 2 * kNB * kNB + kNB * kNB, X + r0,
                         ldx, s);
    if (e != hipSuccess) return e;
    e = update<T>(dtype, r0, nrhs, jb, LU + r0 * lda, lda, X + r0, ldx, X, ldx, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t lu_workspace_bytes(int, int64_t n) {
  const int64_t np = cdiv(std::max<int64_t>(n, 1), kNB);
  const int64_t gmax = cdiv(std::max<int64_t>(n, 1), kPT);
  size_t b = size_t(np) * 2 * kNB * kNB * sizeof(double);
  b += size_t(2 * gmax * kSlot) * sizeof(double);
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
                           const int32_t* rowid, const void* work, const void* B, int64_t ldb,
                           void* X, int64_t ldx, hipStream_t s) {
  return dtype == 0
             ? solve_typed<double>(0, n, nrhs, static_cast<const double*>(LU), lda, rowid, work,
                                   static_cast<const double*>(B), ldb, static_cast<double*>(X), ldx, s)
             : solve_typed<float>(1, n, nrhs, static_cast<const float*>(LU), lda, rowid, work,
                                  static_cast<const float*>(B), ldb, static_cast<float*>(X), ldx, s);
}

}  // namespace k
}  // namespace hexla
