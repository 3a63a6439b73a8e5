// MFMA GEMM core for gfx950 (FP32 and FP64 16x16x4 matrix instructions):
// C = alpha * op(A) op(B) + beta * C, column-major, the dense products the
// paper maps onto xGEMM (Sec. II). A 256-thread workgroup (4 waves, 2 x 2)
// computes a BM x BN tile; K advances in BK steps through double-buffered LDS.
//
// LDS layout follows the global layout so that global loads and LDS stores
// are both 16-byte vectors: an operand that is contiguous along K is kept as
// [row][k] (each lane then reads its BK/4 consecutive k values with one wide
// LDS read), an operand contiguous along M (or N) is kept as [k][row].
// The k values an MFMA step consumes are assigned as k = g*(BK/4) + s for
// lane group g = lane/16 and step s; A and B use the same assignment, so the
// sum over k is unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace hexla {
namespace k {

struct GemmArgs {
  int64_t m, n, k;
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;
  int64_t ldc;
  double alpha, beta;
  void* partial;     // split > 1: split * m * n elements, [z][i + j*m]
  int64_t k_chunk;   // K range of one split (multiple of BK)
  int32_t tiles_m, tiles_n;
  int32_t mode;      // 0 full, 1 lower-triangle tiles + mirror (square tiles)
  int32_t split;
  int32_t ct;        // split-BF16 family, split 1, mode 0: the kernel computes
                     // C^T (m x n here) and stores element (i, j) at C[j + i*ldc]
};

template <typename T>
struct Mfma;
// Both instructions take A[i][k] from lane i + 16k and B[k][j] from lane
// j + 16k. The 16x16 result is spread differently: FP32 lane l, register r
// holds row 4*(l/16) + r; FP64 holds row l/16 + 4*r (column l%16 in both).
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T, int N>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(N)));
};

// Lower-triangle tile t -> (ti, tj), ti >= tj, t = ti*(ti+1)/2 + tj.
__device__ __forceinline__ void tri_tile(int t, int& ti, int& tj) {
  int r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

template <typename T, bool TA, bool TB, int BM, int BN, int BK, bool VEC>
struct GemmTile {
  static constexpr int kThreads = 256;
  static constexpr int VW = VEC ? 16 / int(sizeof(T)) : 1;  // elements per global vector
  static constexpr int PAD = 4;  // keeps rows 16-byte aligned (32 for FP64 k-vectors)
  // A: TA -> contiguous along k -> [BM][BK+PAD]; else [BK][BM+PAD]
  static constexpr int A_LD = TA ? (BK + PAD) : (BM + PAD);
  static constexpr int A_SIZE = TA ? BM * A_LD : BK * A_LD;
  // B: !TB -> contiguous along k -> [BN][BK+PAD]; else [BK][BN+PAD]
  static constexpr int B_LD = !TB ? (BK + PAD) : (BN + PAD);
  static constexpr int B_SIZE = !TB ? BN * B_LD : BK * B_LD;
  static constexpr int STAGE = A_SIZE + B_SIZE;
  static constexpr int LA = BM * BK / (kThreads * VW);  // global vectors per thread
  static constexpr int LB = BN * BK / (kThreads * VW);
  static constexpr int WM = BM / 2, WN = BN / 2;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static constexpr int KS = BK / 4;  // MFMA steps per BK
  static_assert(LA >= 1 && LB >= 1, "tile too small for 256 threads");
  static_assert(BM * BK % (kThreads * VW) == 0 && BN * BK % (kThreads * VW) == 0, "tile");
  using V = typename VecOf<T, VW>::type;
  using acc_t = typename Mfma<T>::acc_t;

  // Global -> registers for one BK step starting at k0 (k_end bounds the split).
  static __device__ __forceinline__ void load(const GemmArgs& g, int64_t m0, int64_t n0,
                                              int64_t k0, int64_t k_end, V (&ra)[LA],
                                              V (&rb)[LB]) {
    const T* A = static_cast<const T*>(g.A);
    const T* B = static_cast<const T*>(g.B);
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = tid + kThreads * r;
      int64_t row, kk;  // element coordinates of the first vector element
      if (TA) {
        row = m0 + e / (BK / VW);
        kk = k0 + (e % (BK / VW)) * VW;
      } else {
        kk = k0 + e / (BM / VW);
        row = m0 + (e % (BM / VW)) * VW;
      }
      V v;
      if (TA) {  // op(A)(row, kk..) = A[kk.. + row*lda]
        const T* p = A + kk + row * g.lda;
        if (row < g.m && kk + VW <= k_end) {
          v = *reinterpret_cast<const V*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) v[q] = (row < g.m && kk + q < k_end) ? p[q] : T(0);
        }
      } else {  // op(A)(row.., kk) = A[row.. + kk*lda]
        const T* p = A + row + kk * g.lda;
        if (kk < k_end && row + VW <= g.m) {
          v = *reinterpret_cast<const V*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) v[q] = (kk < k_end && row + q < g.m) ? p[q] : T(0);
        }
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = tid + kThreads * r;
      int64_t col, kk;
      if (!TB) {
        col = n0 + e / (BK / VW);
        kk = k0 + (e % (BK / VW)) * VW;
      } else {
        kk = k0 + e / (BN / VW);
        col = n0 + (e % (BN / VW)) * VW;
      }
      V v;
      if (!TB) {  // op(B)(kk.., col) = B[kk.. + col*ldb]
        const T* p = B + kk + col * g.ldb;
        if (col < g.n && kk + VW <= k_end) {
          v = *reinterpret_cast<const V*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) v[q] = (col < g.n && kk + q < k_end) ? p[q] : T(0);
        }
      } else {  // op(B)(kk, col..) = B[col.. + kk*ldb]
        const T* p = B + col + kk * g.ldb;
        if (kk < k_end && col + VW <= g.n) {
          v = *reinterpret_cast<const V*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) v[q] = (kk < k_end && col + q < g.n) ? p[q] : T(0);
        }
      }
      rb[r] = v;
    }
  }

  static __device__ __forceinline__ void store(T* sa, T* sb, const V (&ra)[LA], const V (&rb)[LB]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = tid + kThreads * r;
      int off;
      if (TA)
        off = (e / (BK / VW)) * A_LD + (e % (BK / VW)) * VW;
      else
        off = (e / (BM / VW)) * A_LD + (e % (BM / VW)) * VW;
      *reinterpret_cast<V*>(sa + off) = ra[r];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = tid + kThreads * r;
      int off;
      if (!TB)
        off = (e / (BK / VW)) * B_LD + (e % (BK / VW)) * VW;
      else
        off = (e / (BN / VW)) * B_LD + (e % (BN / VW)) * VW;
      *reinterpret_cast<V*>(sb + off) = rb[r];
    }
  }

  static __device__ __forceinline__ void compute(const T* sa, const T* sb, int wm, int wn,
                                                 acc_t (&acc)[FM][FN]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, l16 = lane & 15;
    T a[FM][KS], b[FN][KS];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      const int row = wm * WM + f * 16 + l16;
      if (TA) {
        using KV = typename VecOf<T, KS>::type;
        const KV v = *reinterpret_cast<const KV*>(sa + row * A_LD + g * KS);
#pragma unroll
        for (int s = 0; s < KS; ++s) a[f][s] = v[s];
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) a[f][s] = sa[(g * KS + s) * A_LD + row];
      }
    }
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int col = wn * WN + f * 16 + l16;
      if (!TB) {
        using KV = typename VecOf<T, KS>::type;
        const KV v = *reinterpret_cast<const KV*>(sb + col * B_LD + g * KS);
#pragma unroll
        for (int s = 0; s < KS; ++s) b[f][s] = v[s];
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) b[f][s] = sb[(g * KS + s) * B_LD + col];
      }
    }
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = Mfma<T>::mma(a[fm][s], b[fn][s], acc[fm][fn]);
  }
};

// Work item of this workgroup in a (tile, split) grid of gridDim.x tiles by
// gridDim.y splits. Workgroups go to the 8 XCDs in turn (dispatch order,
// x fastest), and each XCD has its own L2; the remap hands each XCD a
// contiguous run of the split-major order, so the workgroups resident on one
// XCD work on the same K range of neighbouring tiles and share operand lines
// in its L2. A bijection of [0, total) for any total; the placement only
// affects speed.
__device__ __forceinline__ void xcd_work_item(int& tile, int& z) {
  const int tiles = int(gridDim.x);
  const int total = tiles * int(gridDim.y);
  const int l = int(blockIdx.x) + int(blockIdx.y) * tiles;
  const int x = l % 8, j = l / 8;
  const int per = total / 8, rem = total % 8;
  const int q = x * per + min(x, rem) + j;
  z = q / tiles;
  tile = q - z * tiles;
}

// WPE: waves per SIMD the register allocation must allow (2 caps a wave at
// 256 registers, so two workgroups of a small-LDS tile share a CU)
template <typename T, bool TA, bool TB, int BM, int BN, int BK, bool VEC, int WPE = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void gemm_kernel(GemmArgs g) {
  using G = GemmTile<T, TA, TB, BM, BN, BK, VEC>;
  __shared__ __attribute__((aligned(16))) T smem[2 * G::STAGE];

  int tile, z, tm, tn;
  xcd_work_item(tile, z);
  if (g.mode == 1) {
    tri_tile(tile, tm, tn);
  } else {
    tm = tile % g.tiles_m;
    tn = tile / g.tiles_m;
  }
  const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;
  const int64_t kb = int64_t(z) * g.k_chunk;
  int64_t ke = kb + g.k_chunk;
  if (ke > g.k) ke = g.k;

  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  typename G::acc_t acc[G::FM][G::FN];
#pragma unroll
  for (int a = 0; a < G::FM; ++a)
#pragma unroll
    for (int b = 0; b < G::FN; ++b) acc[a][b] = typename G::acc_t{0, 0, 0, 0};

  typename G::V ra[G::LA], rb[G::LB];
  const int64_t nk = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    G::load(g, m0, n0, kb, ke, ra, rb);
    G::store(smem, smem + G::A_SIZE, ra, rb);
  }
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    T* cur = smem + (t & 1) * G::STAGE;
    T* nxt = smem + ((t + 1) & 1) * G::STAGE;
    const bool more = t + 1 < nk;
    if (more) G::load(g, m0, n0, kb + (t + 1) * BK, ke, ra, rb);
    G::compute(cur, cur + G::A_SIZE, wm, wn, acc);
    if (more) G::store(nxt, nxt + G::A_SIZE, ra, rb);
    __syncthreads();
  }

  // epilogue: lane owns rows Mfma<T>::row(lane, r) of column lane%16 in each 16x16 tile
  const int lane = threadIdx.x & 63;
  const T alpha = T(g.alpha), beta = T(g.beta);
  T* C = static_cast<T*>(g.C);
  T* P = static_cast<T*>(g.partial);
  if constexpr (sizeof(T) == 4) {
    // FP32 split-K partials: a lane's four registers are four consecutive
    // rows of one column, written as one 16-byte store (m % 4 == 0 keeps
    // every such store inside the column and 16-byte aligned)
    if (g.split > 1 && (g.m & 3) == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
#pragma unroll
      for (int fm = 0; fm < G::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < G::FN; ++fn) {
          const int64_t i = m0 + wm * G::WM + fm * 16 + Mfma<T>::row(lane, 0);
          const int64_t j = n0 + wn * G::WN + fn * 16 + (lane & 15);
          if (i >= g.m || j >= g.n) continue;
          *reinterpret_cast<typename G::acc_t*>(P + int64_t(z) * g.m * g.n + i + j * g.m) =
              acc[fm][fn];
        }
      return;
    }
  }
#pragma unroll
  for (int fm = 0; fm < G::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < G::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + wm * G::WM + fm * 16 + Mfma<T>::row(lane, r);
        const int64_t j = n0 + wn * G::WN + fn * 16 + (lane & 15);
        if (i >= g.m || j >= g.n) continue;
        const T v = acc[fm][fn][r];
        if (g.split > 1) {
          P[int64_t(z) * g.m * g.n + i + j * g.m] = v;
        } else if (g.mode == 1) {
          if (i >= j) {
            T out = alpha * v;
            if (beta != T(0)) out += beta * C[i + j * g.ldc];
            C[i + j * g.ldc] = out;
            if (i > j) C[j + i * g.ldc] = out;
          }
        } else {
          T out = alpha * v;
          if (beta != T(0)) out += beta * C[i + j * g.ldc];
          C[i + j * g.ldc] = out;
        }
      }
}

// C = alpha * sum_z P[z] + beta * C, summed in a fixed order (deterministic).
// Full mode with m % 4 == 0: one workgroup per 64 quads of consecutive
// elements of a column (16- or 32-byte loads); lane = quad, and wave w sums
// the partials z = w, w + 4, ... in ascending z, up to four loads in flight,
// so that a launch has four times the quads' parallelism and a few memory
// round trips; the four wave sums are added in w order. Other modes: one
// element per thread, z ascending, over a grid-stride loop.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g) {
  const int64_t total = g.m * g.n;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const T* P = static_cast<const T*>(g.partial);
  T* C = static_cast<T*>(g.C);
  const T alpha = T(g.alpha), beta = T(g.beta);
  const int S = g.split;
  if (g.mode == 0 && (g.m % 4) == 0) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    __shared__ v4 red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t quads = total / 4, q = int64_t(blockIdx.x) * 64 + lane;
    const int64_t e = (q < quads ? q : quads - 1) * 4;
    v4 acc = {T(0), T(0), T(0), T(0)};
    int z = w;
    for (; z + 12 < S; z += 16) {
      const v4 a0 = *reinterpret_cast<const v4*>(P + int64_t(z) * total + e);
      const v4 a1 = *reinterpret_cast<const v4*>(P + int64_t(z + 4) * total + e);
      const v4 a2 = *reinterpret_cast<const v4*>(P + int64_t(z + 8) * total + e);
      const v4 a3 = *reinterpret_cast<const v4*>(P + int64_t(z + 12) * total + e);
      acc += a0;
      acc += a1;
      acc += a2;
      acc += a3;
    }
    for (; z < S; z += 4) acc += *reinterpret_cast<const v4*>(P + int64_t(z) * total + e);
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && q < quads) {
      const v4 sum = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
      const int64_t i = e % g.m, j = e / g.m;
      T* c = C + i + j * g.ldc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T out = alpha * sum[r];
        if (beta != T(0)) out += beta * c[r];
        c[r] = out;
      }
    }
    return;
  }
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % g.m, j = e / g.m;
    if (g.mode == 1 && i < j) continue;
    T s = 0;
    for (int z = 0; z < S; ++z) s += P[int64_t(z) * total + e];
    T out = alpha * s;
    if (beta != T(0)) out += beta * C[i + j * g.ldc];
    C[i + j * g.ldc] = out;
    if (g.mode == 1 && i > j) C[j + i * g.ldc] = out;
  }
}

// Launches the reduction of a split-K product described by g.
template <typename T>
inline hipError_t splitk_reduce_launch(const GemmArgs& g, hipStream_t s) {
  const int64_t total = g.m * g.n;
  if (total <= 0) return hipSuccess;
  int64_t blocks;
  if (g.mode == 0 && (g.m % 4) == 0)
    blocks = (total / 4 + 63) / 64;
  else
    blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3(unsigned(blocks)), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
