// Split-BF16 products: FP32 operands, BF16 matrix instructions, FP32
// accumulation. The paper names BF16 as a future element type and cites its
// use for higher-precision results (Sec. IV, the Henry et al. reference).
//
// Each FP32 value x is split as hi = rne(x), mid = rne(x - hi)
// (x - hi is exact in FP32), and for three terms lo = rne(x - hi - mid).
// The product keeps the term products of weight >= 2^-16 (three products:
// hi*hi + hi*mid + mid*hi) or >= 2^-24 (six products: + mid*mid + hi*lo +
// lo*hi), each a v_mfma_f32_16x16x32_bf16 accumulating in FP32.
//
// The split happens on the way from HBM to LDS: a 128x128 tile of C reads
// 128x32 FP32 slices of both operands, splits them in registers and stores
// the BF16 terms in LDS as [row][k] (k contiguous, 16-byte fragment reads).
// Lower-triangle tiles + mirrored stores give the symmetric product (SYRK).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gemm_device.h"
#include "kernels.h"

namespace hexla {
namespace k {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float accv __attribute__((ext_vector_type(4)));
typedef accv accv_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// Element type of the terms: bf16 (split products) or fp16 (one term: the
// half-precision trailing updates of the low-precision LU).
template <typename E>
struct Mfma16;
template <>
struct Mfma16<__bf16> {
  typedef bf16x8 v8;
  typedef bf16x4 v4;
  static __device__ __forceinline__ accv_t mma(v8 a, v8 b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16<_Float16> {
  typedef f16x8 v8;
  typedef f16x4 v4;
  static __device__ __forceinline__ accv_t mma(v8 a, v8 b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDK = BK;  // bf16 row stride in LDS (64 bytes), 16-byte chunks swizzled

// LDS position of element k of row `row` in a term's [row][k] tile: the
// 16-byte chunk k / 8 is XORed with bits 2-3 of the row, so that the term
// stores (8 bytes per lane, four consecutive rows per 32 lanes) fill the 64
// banks once and the MFMA fragment reads (16 bytes per lane, 16 consecutive
// rows at one chunk) touch 16 distinct 4-bank groups.
__device__ __forceinline__ int lds_off(int row, int k) {
  return row * LDK + (((k >> 3) ^ ((row >> 2) & 3)) << 3) + (k & 7);
}

template <int TERMS, typename E = __bf16>
__device__ __forceinline__ void split_terms(float x, E (&t)[TERMS]) {
  float rest = x;
#pragma unroll
  for (int q = 0; q < TERMS; ++q) {
    const E h = static_cast<E>(rest);  // round to nearest even
    t[q] = h;
    rest = rest - static_cast<float>(h);
  }
}

template <bool TA, bool TB, int TERMS, typename E>
struct SplitTile {
  typedef typename Mfma16<E>::v4 v4;
  static constexpr int kThreads = 256;
  static constexpr int A_ELEMS = BM * LDK;  // per term
  static constexpr int B_ELEMS = BN * LDK;
  static constexpr int STAGE = TERMS * (A_ELEMS + B_ELEMS);  // bf16 elements
  static constexpr int LV = BM * BK / (kThreads * 4);         // float4 loads per operand per thread

  // Global -> registers (FP32, 4 consecutive elements along the contiguous dim).
  static __device__ __forceinline__ void load(const GemmArgs& g, int64_t m0, int64_t n0,
                                              int64_t k0, int64_t k_end, bool vec, f4 (&ra)[LV],
                                              f4 (&rb)[LV]) {
    const float* A = static_cast<const float*>(g.A);
    const float* B = static_cast<const float*>(g.B);
#pragma unroll
    for (int r = 0; r < LV; ++r) {
      const int e = threadIdx.x + kThreads * r;
      int64_t row, kk;
      if (TA) {  // k contiguous: rows of 32 k
        row = m0 + e / (BK / 4);
        kk = k0 + (e % (BK / 4)) * 4;
        const float* p = A + kk + row * g.lda;
        if (vec && row < g.m && kk + 4 <= k_end) ra[r] = *reinterpret_cast<const f4*>(p);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) ra[r][q] = (row < g.m && kk + q < k_end) ? p[q] : 0.f;
      } else {  // m contiguous: columns of 128 rows
        kk = k0 + e / (BM / 4);
        row = m0 + (e % (BM / 4)) * 4;
        const float* p = A + row + kk * g.lda;
        if (vec && kk < k_end && row + 4 <= g.m) ra[r] = *reinterpret_cast<const f4*>(p);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) ra[r][q] = (kk < k_end && row + q < g.m) ? p[q] : 0.f;
      }
    }
#pragma unroll
    for (int r = 0; r < LV; ++r) {
      const int e = threadIdx.x + kThreads * r;
      int64_t col, kk;
      if (!TB) {  // op(B)(k, col) = B[k + col*ldb]: k contiguous
        col = n0 + e / (BK / 4);
        kk = k0 + (e % (BK / 4)) * 4;
        const float* p = B + kk + col * g.ldb;
        if (vec && col < g.n && kk + 4 <= k_end) rb[r] = *reinterpret_cast<const f4*>(p);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) rb[r][q] = (col < g.n && kk + q < k_end) ? p[q] : 0.f;
      } else {  // op(B)(k, col) = B[col + k*ldb]: n contiguous
        kk = k0 + e / (BN / 4);
        col = n0 + (e % (BN / 4)) * 4;
        const float* p = B + col + kk * g.ldb;
        if (vec && kk < k_end && col + 4 <= g.n) rb[r] = *reinterpret_cast<const f4*>(p);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) rb[r][q] = (kk < k_end && col + q < g.n) ? p[q] : 0.f;
      }
    }
  }

  // Split in registers and store the BF16 terms as [row][k].
  static __device__ __forceinline__ void store(E* sa, E* sb, const f4 (&ra)[LV],
                                               const f4 (&rb)[LV]) {
#pragma unroll
    for (int r = 0; r < LV; ++r) {
      const int e = threadIdx.x + kThreads * r;
      E t[4][TERMS];
#pragma unroll
      for (int q = 0; q < 4; ++q) split_terms<TERMS, E>(ra[r][q], t[q]);
      if (TA) {
        const int row = e / (BK / 4), kk = (e % (BK / 4)) * 4;
#pragma unroll
        for (int s = 0; s < TERMS; ++s) {
          v4 v;
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = t[q][s];
          *reinterpret_cast<v4*>(sa + s * A_ELEMS + lds_off(row, kk)) = v;
        }
      } else {
        const int kk = e / (BM / 4), row = (e % (BM / 4)) * 4;
#pragma unroll
        for (int s = 0; s < TERMS; ++s)
#pragma unroll
          for (int q = 0; q < 4; ++q) sa[s * A_ELEMS + lds_off(row + q, kk)] = t[q][s];
      }
    }
#pragma unroll
    for (int r = 0; r < LV; ++r) {
      const int e = threadIdx.x + kThreads * r;
      E t[4][TERMS];
#pragma unroll
      for (int q = 0; q < 4; ++q) split_terms<TERMS, E>(rb[r][q], t[q]);
      if (!TB) {
        const int col = e / (BK / 4), kk = (e % (BK / 4)) * 4;
#pragma unroll
        for (int s = 0; s < TERMS; ++s) {
          v4 v;
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = t[q][s];
          *reinterpret_cast<v4*>(sb + s * B_ELEMS + lds_off(col, kk)) = v;
        }
      } else {
        const int kk = e / (BN / 4), col = (e % (BN / 4)) * 4;
#pragma unroll
        for (int s = 0; s < TERMS; ++s)
#pragma unroll
          for (int q = 0; q < 4; ++q) sb[s * B_ELEMS + lds_off(col + q, kk)] = t[q][s];
      }
    }
  }
};

template <bool TA, bool TB, int TERMS, typename E>
__global__ __launch_bounds__(256) void gemm_split_kernel(GemmArgs g, int vec) {
  using G = SplitTile<TA, TB, TERMS, E>;
  using M = Mfma16<E>;
  typedef typename M::v8 v8;
  __shared__ __attribute__((aligned(16))) E smem[2 * G::STAGE];
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
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, grp = lane >> 4;

  accv acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = accv{0.f, 0.f, 0.f, 0.f};

  f4 ra[G::LV], rb[G::LV];
  const int64_t nk = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    G::load(g, m0, n0, kb, ke, vec != 0, ra, rb);
    G::store(smem, smem + TERMS * G::A_ELEMS, ra, rb);
  }
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    E* cur = smem + (t & 1) * G::STAGE;
    E* nxt = smem + ((t + 1) & 1) * G::STAGE;
    const bool more = t + 1 < nk;
    if (more) G::load(g, m0, n0, kb + (t + 1) * BK, ke, vec != 0, ra, rb);
    const E* sa = cur;
    const E* sb = cur + TERMS * G::A_ELEMS;
    v8 a[TERMS][4], b[TERMS][4];
#pragma unroll
    for (int s = 0; s < TERMS; ++s)
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        a[s][f] = *reinterpret_cast<const v8*>(sa + s * G::A_ELEMS +
                                               lds_off(wm * 64 + f * 16 + l16, grp * 8));
        b[s][f] = *reinterpret_cast<const v8*>(sb + s * G::B_ELEMS +
                                               lds_off(wn * 64 + f * 16 + l16, grp * 8));
      }
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) {
        // small terms first
        if (TERMS == 3) {
          acc[fm][fn] = M::mma(a[2 % TERMS][fm], b[0][fn], acc[fm][fn]);
          acc[fm][fn] = M::mma(a[0][fm], b[2 % TERMS][fn], acc[fm][fn]);
          acc[fm][fn] = M::mma(a[1 % TERMS][fm], b[1 % TERMS][fn], acc[fm][fn]);
        }
        if (TERMS >= 2) {
          acc[fm][fn] = M::mma(a[1 % TERMS][fm], b[0][fn], acc[fm][fn]);
          acc[fm][fn] = M::mma(a[0][fm], b[1 % TERMS][fn], acc[fm][fn]);
        }
        acc[fm][fn] = M::mma(a[0][fm], b[0][fn], acc[fm][fn]);
      }
    if (more) G::store(nxt, nxt + TERMS * G::A_ELEMS, ra, rb);
    __syncthreads();
  }

  // epilogue (result layout of the 16x16 FP32-accumulating instructions:
  // lane l, register r holds row 4*(l/16) + r, column l%16)
  const float alpha = float(g.alpha), beta = float(g.beta);
  float* C = static_cast<float*>(g.C);
  float* P = static_cast<float*>(g.partial);
  if (g.split > 1 && (g.m & 3) == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
    // split-K partials: a lane's four registers are four consecutive rows
    // of one column, one 16-byte store (in bounds and aligned as m % 4 == 0)
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) {
        const int64_t i = m0 + wm * 64 + fm * 16 + 4 * grp;
        const int64_t j = n0 + wn * 64 + fn * 16 + l16;
        if (i >= g.m || j >= g.n) continue;
        *reinterpret_cast<accv*>(P + int64_t(z) * g.m * g.n + i + j * g.m) = acc[fm][fn];
      }
    return;
  }
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + wm * 64 + fm * 16 + 4 * grp + r;
        const int64_t j = n0 + wn * 64 + fn * 16 + l16;
        if (i >= g.m || j >= g.n) continue;
        const float v = acc[fm][fn][r];
        if (g.split > 1) {
          P[int64_t(z) * g.m * g.n + i + j * g.m] = v;
        } else if (g.mode == 1) {
          if (i >= j) {
            float out = alpha * v;
            if (beta != 0.f) out += beta * C[i + j * g.ldc];
            C[i + j * g.ldc] = out;
            if (i > j) C[j + i * g.ldc] = out;
          }
        } else {
          const int64_t at = g.ct ? j + i * g.ldc : i + j * g.ldc;
          float out = alpha * v;
          if (beta != 0.f) out += beta * C[at];
          C[at] = out;
        }
      }
}


// C -= A B for K <= 64 (the LU's rank-K trailing update) in split terms: A
// m x K, B K x n, C m x n, FP32, column-major. One 256-thread workgroup per
// 64 x 64 tile of C, loaded straight into the accumulators; both operand
// tiles (the whole K range) are split on the way to LDS as [row][k] BF16 (or
// FP16) terms, B negated; the products are computed transposed (operand A
// from B's columns, operand B from A's rows), so a 16-lane group holds 16
// consecutive rows of one column of C and C moves in 64-byte runs. The
// traffic is the C tile twice plus the operand tiles once, as in the plain
// rank-K update: the split terms cost MFMA time only, which stays under the
// C traffic at this K.
constexpr int RU_T = 64;  // tile side
constexpr int RU_K = 64;  // K at most

// LDS position of element k of row `row` in a [row][k] term tile of RU_K
// columns: 16-byte chunk k / 8 XORed with the row's low three bits.
__device__ __forceinline__ int ru_off(int row, int k) {
  return row * RU_K + (((k >> 3) ^ (row & 7)) << 3) + (k & 7);
}

template <int TERMS, typename E>
__global__ __launch_bounds__(256) void rank_update_split_kernel(
    int64_t m, int64_t n, int K, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, float* __restrict__ C, int64_t ldc, int tiles_m,
    int vec) {
  using M = Mfma16<E>;
  typedef typename M::v8 v8;
  typedef typename M::v4 v4;
  constexpr int TE = RU_T * RU_K;  // elements of one term tile
  __shared__ __attribute__((aligned(16))) E sa[TERMS * TE];  // A(row, k)
  __shared__ __attribute__((aligned(16))) E sb[TERMS * TE];  // -B(k, col) as [col][k]
  const int tm = int(blockIdx.x) % tiles_m, tn = int(blockIdx.x) / tiles_m;
  const int64_t m0 = int64_t(tm) * RU_T, n0 = int64_t(tn) * RU_T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int l16 = lane & 15, g = lane >> 4;
  // 1. the C tile into the accumulators: block (fc, fr) register r holds
  // column n0 + 32 wc + 16 fc + 4 g + r, row m0 + 32 wr + 16 fr + l16
  accv acc[2][2];
#pragma unroll
  for (int fc = 0; fc < 2; ++fc)
#pragma unroll
    for (int fr = 0; fr < 2; ++fr)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + 32 * wc + 16 * fc + 4 * g + r;
        const int64_t row = m0 + 32 * wr + 16 * fr + l16;
        const float v = C[std::min<int64_t>(row, m - 1) + std::min<int64_t>(col, n - 1) * ldc];
        acc[fc][fr][r] = (row < m && col < n) ? v : 0.f;
      }
  // 2. the operand tiles: A(row, 4q..4q+3) and B(4q..4q+3, col) per thread
  // and pass, every load in flight at once (clamped addresses, zeros after)
  f4 va[4], vb[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int e = tid + 256 * p;
    const int row = e % RU_T, qa = e / RU_T;  // A: coalesced along rows
    const int64_t gr = std::min<int64_t>(m0 + row, m - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) va[p][q] = A[gr + int64_t(min(4 * qa + q, K - 1)) * lda];
    const int qb = e % (RU_K / 4), col = e / (RU_K / 4);  // B: k contiguous
    const float* pb = B + std::min<int64_t>(n0 + col, n - 1) * ldb;
    if (vec) {
      vb[p] = *reinterpret_cast<const f4*>(pb + 4 * qb);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) vb[p][q] = pb[min(4 * qb + q, K - 1)];
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int e = tid + 256 * p;
    {
      const int row = e % RU_T, qa = e / RU_T;
      E t[4][TERMS];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        split_terms<TERMS, E>((m0 + row < m && 4 * qa + q < K) ? va[p][q] : 0.f, t[q]);
#pragma unroll
      for (int s4 = 0; s4 < TERMS; ++s4) {
        v4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = t[q][s4];
        *reinterpret_cast<v4*>(sa + s4 * TE + ru_off(row, 4 * qa)) = v;
      }
    }
    {
      const int qb = e % (RU_K / 4), col = e / (RU_K / 4);
      E t[4][TERMS];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        split_terms<TERMS, E>((n0 + col < n && 4 * qb + q < K) ? -vb[p][q] : 0.f, t[q]);
#pragma unroll
      for (int s4 = 0; s4 < TERMS; ++s4) {
        v4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = t[q][s4];
        *reinterpret_cast<v4*>(sb + s4 * TE + ru_off(col, 4 * qb)) = v;
      }
    }
  }
  __syncthreads();
  // 3. acc += (-B^T) A^T in term products, small terms first: operand A
  // from lane (i, g) = -B(8 g.., column i), operand B from A(row j, 8 g..)
#pragma unroll
  for (int ks = 0; ks < RU_K / 32; ++ks) {
    v8 a[TERMS][2], b[TERMS][2];
#pragma unroll
    for (int s4 = 0; s4 < TERMS; ++s4)
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        a[s4][f] = *reinterpret_cast<const v8*>(sb + s4 * TE +
                                                ru_off(32 * wc + 16 * f + l16, 32 * ks + 8 * g));
        b[s4][f] = *reinterpret_cast<const v8*>(sa + s4 * TE +
                                                ru_off(32 * wr + 16 * f + l16, 32 * ks + 8 * g));
      }
#pragma unroll
    for (int fc = 0; fc < 2; ++fc)
#pragma unroll
      for (int fr = 0; fr < 2; ++fr) {
        if (TERMS == 3) {
          acc[fc][fr] = M::mma(a[2 % TERMS][fc], b[0][fr], acc[fc][fr]);
          acc[fc][fr] = M::mma(a[0][fc], b[2 % TERMS][fr], acc[fc][fr]);
          acc[fc][fr] = M::mma(a[1 % TERMS][fc], b[1 % TERMS][fr], acc[fc][fr]);
        }
        if (TERMS >= 2) {
          acc[fc][fr] = M::mma(a[1 % TERMS][fc], b[0][fr], acc[fc][fr]);
          acc[fc][fr] = M::mma(a[0][fc], b[1 % TERMS][fr], acc[fc][fr]);
        }
        acc[fc][fr] = M::mma(a[0][fc], b[0][fr], acc[fc][fr]);
      }
  }
  // 4. back to C
#pragma unroll
  for (int fc = 0; fc < 2; ++fc)
#pragma unroll
    for (int fr = 0; fr < 2; ++fr)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + 32 * wc + 16 * fc + 4 * g + r;
        const int64_t row = m0 + 32 * wr + 16 * fr + l16;
        if (row < m && col < n) C[row + col * ldc] = acc[fc][fr][r];
      }
}

typedef void (*SplitFn)(GemmArgs, int);

template <int TERMS, typename E>
SplitFn pick(bool ta, bool tb) {
  if (ta) return tb ? gemm_split_kernel<true, true, TERMS, E> : gemm_split_kernel<true, false, TERMS, E>;
  return tb ? gemm_split_kernel<false, true, TERMS, E> : gemm_split_kernel<false, false, TERMS, E>;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__global__ void split_bf16_kernel(const float* __restrict__ x, int64_t n, uint16_t* hi,
                                  uint16_t* mid, uint16_t* lo, int terms) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    __bf16 t[3];
    split_terms<3, __bf16>(x[i], t);
    hi[i] = __builtin_bit_cast(uint16_t, t[0]);
    mid[i] = __builtin_bit_cast(uint16_t, t[1]);
    if (terms == 3) lo[i] = __builtin_bit_cast(uint16_t, t[2]);
  }
}

}  // namespace

GemmConfig gemm_choose_split(int, int, int mode, int64_t m, int64_t n, int64_t k) {
  int64_t tiles;
  if (mode == 1) {
    const int64_t tt = cdiv(n, BN);
    tiles = tt * (tt + 1) / 2;
  } else {
    tiles = cdiv(m, BM) * cdiv(n, BN);
  }
  // about 1024 workgroups; every workgroup runs at least 16 K steps
  int64_t split = std::max<int64_t>(1, cdiv(1024, tiles));
  split = std::min<int64_t>(split, std::max<int64_t>(1, k / (16 * BK)));
  split = std::min<int64_t>(split, 64);
  if (split > 1) {
    const int64_t chunk = cdiv(cdiv(k, split), BK) * BK;
    split = cdiv(k, chunk);
  }
  return GemmConfig{0, int(split)};
}

hipError_t gemm_split_launch(int dtype, int precision, int mode, int ta, int tb, int64_t m,
                             int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
                             const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                             void* partial, const GemmConfig& cfg, hipStream_t s) {
  if (dtype != 1) return hipErrorNotSupported;  // FP32 storage only
  // Without split-K a full product is computed transposed, C^T = op(B)^T op(A)^T:
  // the accumulator layout then gives each 16-lane group 16 consecutive rows
  // of one column of C, so C is read and written in 64-byte runs (C-bound
  // products such as the LU's rank-64 updates gain most).
  const bool ct = mode == 0 && cfg.split <= 1;
  if (ct) {
    std::swap(m, n);
    std::swap(A, B);
    std::swap(lda, ldb);
    const int t = ta;
    ta = !tb;
    tb = !t;
  }
  GemmArgs g{};
  g.ct = ct ? 1 : 0;
  g.m = m; g.n = n; g.k = k;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.partial = partial;
  g.mode = mode;
  g.split = std::max(cfg.split, 1);
  g.k_chunk = std::max<int64_t>(BK, cdiv(cdiv(k, g.split), BK) * BK);
  g.tiles_m = int(cdiv(m, BM));
  g.tiles_n = int(cdiv(n, BN));
  const int vec = (lda % 4 == 0) && (ldb % 4 == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0) &&
                  (reinterpret_cast<uintptr_t>(B) % 16 == 0);
  const int64_t blocks = mode == 1 ? int64_t(g.tiles_n) * (g.tiles_n + 1) / 2
                                   : int64_t(g.tiles_m) * g.tiles_n;
  SplitFn fn = precision == GEMM_BF16X6 ? pick<3, __bf16>(ta != 0, tb != 0)
              : precision == GEMM_F16  ? pick<1, _Float16>(ta != 0, tb != 0)
                                       : pick<2, __bf16>(ta != 0, tb != 0);
  hipLaunchKernelGGL(fn, dim3(unsigned(blocks), unsigned(g.split)), dim3(256), 0, s, g, vec);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.split <= 1) return e;
  return splitk_reduce_launch<float>(g, s);
}

hipError_t rank_update_split_launch(int precision, int64_t m, int64_t n, int64_t K,
                                    const float* A, int64_t lda, const float* B, int64_t ldb,
                                    float* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0 || K <= 0) return hipSuccess;
  const int64_t tm = cdiv(m, RU_T), tn = cdiv(n, RU_T);
  if (K > RU_K || tm * tn > INT32_MAX) return hipErrorInvalidValue;
  // whole 16-byte B loads when every column's K run is aligned and complete
  const int vec = K == RU_K && ldb % 4 == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  const dim3 grid(unsigned(tm * tn)), block(256);
  if (precision == GEMM_BF16X3)
    hipLaunchKernelGGL((rank_update_split_kernel<2, __bf16>), grid, block, 0, s, m, n, int(K), A,
                       lda, B, ldb, C, ldc, int(tm), vec);
  else if (precision == GEMM_BF16X6)
    hipLaunchKernelGGL((rank_update_split_kernel<3, __bf16>), grid, block, 0, s, m, n, int(K), A,
                       lda, B, ldb, C, ldc, int(tm), vec);
  else if (precision == GEMM_F16)
    hipLaunchKernelGGL((rank_update_split_kernel<1, _Float16>), grid, block, 0, s, m, n, int(K),
                       A, lda, B, ldb, C, ldc, int(tm), vec);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t split_bf16_launch(const float* x, int64_t n, uint16_t* hi, uint16_t* mid, uint16_t* lo,
                             int terms, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = cdiv(n, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(split_bf16_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, x, n, hi, mid, lo,
                     terms);
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
