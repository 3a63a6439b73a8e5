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
//               factored by one wave (a row per lane, in registers), which
//               also inverts it; the block column below is L21 = A21 L11^-T
//               as an MFMA product with that inverse, and the trailing
//               matrix's lower tiles take the rank-64 update L21 L21^T. No
//               pivoting, so no per-column exchange between workgroups;
//   triangular  the inverses of all 64 x 64 diagonal blocks in one launch
//               (substitution against the identity, one column per lane),
//               then per block one launch: the block's solution as the
//               product with its inverse and, in the same workgroups, the
//               update of the rows still to solve (Cholesky: forward with L,
//               backward with L^T), all on the MFMAs;
//   tridiagonal Gaussian elimination with partial pivoting between adjacent
//               rows (a fill-in of one extra superdiagonal), one lane per
//               right-hand side.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gemm_device.h"
#include "kernels.h"

namespace hexla {
namespace k {

namespace {

constexpr int kB = 64;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Makes x a register value at this point: loads issued in a loop before a
// loop of these are all in flight together; without it the compiler moves
// each load next to its first use (or behind the branch of a select), and
// each then waits for a full memory round trip in turn.
template <typename T>
__device__ __forceinline__ void materialize(T& x) {
  asm volatile("" : "+v"(x));
}

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
  __shared__ T sm[kB][kB + 1];  // the mirror tile (J, I): sm[r][c] = S(J*64 + r, I*64 + c)
  __shared__ int s_red[4][4];
  __shared__ double s_max[4][2];
  const int64_t t = blockIdx.x;
  int64_t I = int64_t((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int64_t J = t - I * (I + 1) / 2;
  const int r = threadIdx.x & 63, cq = threadIdx.x >> 6;
  // tile (I, J) into registers and tile (J, I) into LDS, every load issued
  // before any is used (clamped addresses; columns cq + 4 q, coalesced rows)
  T a[16], m[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = cq + 4 * q;
    const int64_t i = std::min<int64_t>(I * kB + r, n - 1), j = std::min<int64_t>(J * kB + c, n - 1);
    const int64_t i2 = std::min<int64_t>(J * kB + r, n - 1), j2 = std::min<int64_t>(I * kB + c, n - 1);
    a[q] = S[i + j * lds];
    m[q] = S[i2 + j2 * lds];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) sm[r][cq + 4 * q] = m[q];
  __syncthreads();
  int kl = 0, ku = 0, asym = 0, nonpos = 0, zero = 0;
  double amax = 0.0, dmax = 0.0;
  const int64_t i = I * kB + r;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = cq + 4 * q;
    const int64_t j = J * kB + c;  // element (i, j) of tile (I, J); its mirror (j, i)
    const bool in = i < n && j < n;
    const T x = a[q];
    const T y = sm[c][r];
    const int d = int(std::min<int64_t>(i > j ? i - j : j - i, 0x7fffffff));
    // x at (i, j) and y at (j, i): a nonzero below the diagonal widens the
    // lower band, one above it the upper band
    const bool low = in && ((i > j && x != T(0)) || (j > i && y != T(0)));
    const bool up = in && ((j > i && x != T(0)) || (i > j && y != T(0)));
    kl = max(kl, low ? d : 0);
    ku = max(ku, up ? d : 0);
    asym |= (in && !(x == y)) ? 1 : 0;  // NaN compares unequal
    const double da = in ? fmax(fabs(double(x)), fabs(double(y))) : 0.0;
    const double dd = in ? fabs(double(x) - double(y)) : 0.0;
    amax = da > amax ? da : amax;  // a NaN never replaces the maximum ...
    dmax = dd > dmax ? dd : dmax;
    if (in && (x != x || y != y)) dmax = __builtin_inf();  // ... but makes S unsymmetric
    const bool diag = in && i == j;
    nonpos |= (diag && !(x > T(0))) ? 1 : 0;
    zero |= (diag && x == T(0)) ? 1 : 0;
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
    // an atomic only where it changes the word: thousands of workgroups
    // updating the same few words would otherwise queue at one L2 channel
    unsigned long long* words = reinterpret_cast<unsigned long long*>(info + 8);
    auto ld64 = [](unsigned long long* p) {
      return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto ld32 = [](int32_t* p) {
      return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    const unsigned long long b0 = static_cast<unsigned long long>(__double_as_longlong(m0));
    const unsigned long long b1 = static_cast<unsigned long long>(__double_as_longlong(m1));
    if (m0 > 0.0 && b0 > ld64(words)) atomicMax(words, b0);
    if (m1 > 0.0 && b1 > ld64(words + 1)) atomicMax(words + 1, b1);
    if (a0 > ld32(info + 0)) atomicMax(info + 0, a0);
    if (a1 > ld32(info + 1)) atomicMax(info + 1, a1);
    if (a2 && !ld32(info + 2)) atomicOr(info + 2, 1);
    if ((a3 & 1) && !ld32(info + 3)) atomicOr(info + 3, 1);
    if ((a3 & 2) && !ld32(info + 5)) atomicOr(info + 5, 1);
  }
}

// ------------------------------------------------ 64 x 64 triangular blocks

// The kernels below hold one 64-element row or column per lane in registers,
// with every index fixed at compile time (fully unrolled loops). A ragged
// last block (jb < 64) is handled by clamped addresses, never by per-element
// conditions around loads or stores: those make the compiler keep all 64
// values live across each branch and spill them.

// Orders a wave's LDS stores before its later LDS loads (one wave works).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Lane `src`'s value of x for the whole wave (src a compile-time constant).
__device__ __forceinline__ float lane_value(float x, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ __forceinline__ double lane_value(double x, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
  return __hiloint2double(hi, lo);
}

// Cholesky of the diagonal block at (k0, k0) (jb <= 64 rows; rows and
// columns past jb are the identity) and its inverse, the block in LDS.
// Blocked over four 16-column panels: wave 0 factors the panel's rows (lane
// r holding row r's 16 panel entries in registers; per column the pivot read
// from its lane with v_readlane, the multipliers published through LDS and
// read back together), then the four waves apply the panel's rank-16 update
// to the lower 16 x 16 tiles right of it with MFMA. A pivot that is not > 0
// sets info[4] and nothing is stored; otherwise L11 is written over the
// block's lower triangle. The inverse R = L11^-1 follows by blocked
// substitution over 16-row blocks: D_b = L_bb^-1 by substitution (wave 0,
// lane (b, c) building column c of D_b), M_bj = D_b L_bj for j < b (MFMA),
// R_b = D_b E_b - sum_j M_bj R_j with E the identity (MFMA, wave w taking
// columns 16w..16w+15); it is stored column-major.
template <typename T>
__global__ __launch_bounds__(256) void potrf_block_kernel(T* __restrict__ A, int64_t lda,
                                                          int64_t k0, int jb, int32_t* info,
                                                          T* __restrict__ inv) {
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc_t;
  constexpr int LA = kB + 4;
  __shared__ T As[kB][LA];          // As[r][c]: the block (lower part), then L11
  __shared__ T colj[16];            // the current column's multipliers in the panel
  __shared__ T rdg[kB];             // 1 / L(j, j)
  __shared__ T Ds[4][16][16 + 4];   // Ds[b][t][i] = D_b(i, t)
  __shared__ T Ms[6][16][16 + 4];   // Ms[p][t][i] = M_bj(i, t), p = b(b-1)/2 + j
  __shared__ T Rs[4][16][kB + 4];   // Rs[w][c][i] = R(i, 16w + c)
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  constexpr int PER = kB * kB / 256;
  {
    T v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {  // element (i, c) from thread e % 64 (coalesced columns)
      const int e = tid + 256 * q, i = e % kB, c = e / kB;
      v[q] = A[(k0 + std::min(i, jb - 1)) + (k0 + std::min(c, jb - 1)) * lda];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q, i = e % kB, c = e / kB;
      As[i][c] = (i < jb && c < jb) ? (c <= i ? v[q] : T(0)) : T(i == c ? 1 : 0);
    }
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (w == 0 && lane >= 16 * b) {  // the panel's rows
      const int r = lane;
      T a[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = As[r][16 * b + c];
#pragma unroll
      for (int c = 0; c < 16; ++c) materialize(a[c]);
      bool bad = false;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * b + jj;
        const T d = lane_value(a[jj], j);  // the pivot, lane j's diagonal entry
        const bool ok = d > T(0);
        bad = bad || !ok;
        // one reciprocal square root on the chain of columns: L(j, j) =
        // d / sqrt(d), the column below it scaled by 1 / sqrt(d)
        const T rs = ok ? rsqrt(d) : T(1);
        const T l = (r == j ? d : a[jj]) * rs;
        if (r == j) rdg[j] = rs;
        a[jj] = l;
        if (jj < 15) {
          if (r >= j && r < 16 * b + 16) colj[r - 16 * b] = l;
          wave_sync();
          T cj[16];
#pragma unroll
          for (int c = jj + 1; c < 16; ++c) cj[c] = colj[c];
#pragma unroll
          for (int c = jj + 1; c < 16; ++c) materialize(cj[c]);
#pragma unroll
          for (int c = jj + 1; c < 16; ++c) a[c] -= l * cj[c];
          wave_sync();  // colj is rewritten by the next column
        }
      }
      if (bad && r == 16 * b) s_bad = 1;
#pragma unroll
      for (int c = 0; c < 16; ++c) As[r][16 * b + c] = 16 * b + c <= r ? a[c] : T(0);
    }
    __syncthreads();
    // the lower tiles (I, J), b < J <= I, minus L_I,b L_J,b^T (operand A[i][k]
    // = L(16I + i, 16b + k), operand B[k][j] = L(16J + j, 16b + k))
    const int nt = (3 - b) * (4 - b) / 2;
    for (int t = w; t < nt; t += 4) {
      int I = b + 1, J = b + 1, u = t;
      while (u > I - (b + 1)) {
        u -= I - b;
        ++I;
      }
      J = b + 1 + u;
      acc_t acc;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[rr] = As[16 * I + Mf::row(lane, rr)][16 * J + l16];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        acc = Mf::mma(-As[16 * I + l16][16 * b + 4 * s4 + g], As[16 * J + l16][16 * b + 4 * s4 + g],
                      acc);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) As[16 * I + Mf::row(lane, rr)][16 * J + l16] = acc[rr];
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) info[4] = 1;
    return;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e % kB, c = e / kB;
    if (i < jb && c <= i) A[(k0 + i) + (k0 + c) * lda] = As[i][c];
  }
  if (w == 0) {  // D_b = L_bb^-1, lane (b, c) = (g, l16) builds column c
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = T(i == l16 ? 1 : 0);
#pragma unroll
    for (int l = 0; l < 16; ++l) {
      const T xl = x[l] * rdg[16 * g + l];
      x[l] = xl;
#pragma unroll
      for (int i = l + 1; i < 16; ++i) x[i] -= As[16 * g + i][16 * g + l] * xl;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Ds[g][l16][i] = x[i];
  }
  __syncthreads();
  // M_bj = D_b L_bj: operand A[i][t] = D_b(i, t), B[t][c] = L(16b + t, 16j + c)
  for (int p = w; p < 6; p += 4) {
    const int b = p < 1 ? 1 : p < 3 ? 2 : 3;
    const int j = p - b * (b - 1) / 2;
    acc_t mm = acc_t{};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
      mm = Mf::mma(Ds[b][4 * s4 + g][l16], As[16 * b + 4 * s4 + g][16 * j + l16], mm);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ms[p][l16][Mf::row(lane, r)] = mm[r];
  }
  __syncthreads();
  // R_b = D_b E_b - sum_{j<b} M_bj R_j on this wave's 16 columns
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    acc_t acc = acc_t{};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int row = 16 * b + 4 * s4 + g;
      acc = Mf::mma(Ds[b][4 * s4 + g][l16], T(row == 16 * w + l16 ? 1 : 0), acc);
    }
#pragma unroll
    for (int j = 0; j < b; ++j) {
      const int p = b * (b - 1) / 2 + j;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        acc = Mf::mma(-Ms[p][4 * s4 + g][l16], Rs[w][l16][16 * j + 4 * s4 + g], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Rs[w][l16][16 * b + Mf::row(lane, r)] = acc[r];
    __builtin_amdgcn_s_waitcnt(0);  // the block is in LDS before the next reads it
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e % kB, c = e / kB;
    inv[e] = Rs[c / 16][c % 16][i];  // (i, c) at i + kB c
  }
}

// The block column under a factored diagonal block, L21 = A21 L11^-T, as a
// product with the inverse that the diagonal block's kernel left in D
// (64 x 64, column-major): one workgroup per 64 rows, in place (the tile is
// read into LDS before it is written). Computed transposed on the MFMAs:
// result row i (an MFMA row) is column i of the tile, so 16 consecutive lanes
// hold 16 consecutive rows of one column for the stores.
template <typename T>
__global__ __launch_bounds__(256) void trsm_right_kernel(T* __restrict__ A, int64_t lda,
                                                         int64_t k0, int jb, int64_t m,
                                                         const T* __restrict__ D) {
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc_t;
  constexpr int LD = kB + 1, WT = kB / 2, F = WT / 16;
  __shared__ T sD[kB][LD];  // sD[k][i] = D(i, k)
  __shared__ T sB[kB][LD];  // sB[k][j] = A21(row j of the tile, k)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, g = lane >> 4;
  const int64_t row0 = k0 + jb + int64_t(blockIdx.x) * kB;  // first row of the tile
  const int64_t rlast = k0 + jb + m - 1;
  constexpr int PER = kB * kB / 256;
  T vd[PER], vb[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, a = e & (kB - 1), c = e / kB;
    vd[q] = D[a + kB * c];
    vb[q] = A[std::min<int64_t>(row0 + a, rlast) + (k0 + std::min(c, jb - 1)) * lda];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, a = e & (kB - 1), c = e / kB;
    sD[c][a] = (a < jb && c < jb) ? vd[q] : T(0);
    sB[c][a] = (c < jb) ? vb[q] : T(0);
  }
  __syncthreads();
  // acc[fc][fr] register r: column wc*WT + fc*16 + Mf::row(lane, r), row
  // wr*WT + fr*16 + l16 of the result; operand A[i][k] = D(column i, k),
  // operand B[k][j] = A21(row j, k)
  acc_t acc[F][F];
#pragma unroll
  for (int fc = 0; fc < F; ++fc)
#pragma unroll
    for (int fr = 0; fr < F; ++fr) acc[fc][fr] = acc_t{};
#pragma unroll 4
  for (int kk = 0; kk < kB; kk += 4) {
    T d[F], b[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      d[f] = sD[kk + g][wc * WT + f * 16 + l16];
      b[f] = sB[kk + g][wr * WT + f * 16 + l16];
    }
#pragma unroll
    for (int fc = 0; fc < F; ++fc)
#pragma unroll
      for (int fr = 0; fr < F; ++fr) acc[fc][fr] = Mf::mma(d[fc], b[fr], acc[fc][fr]);
  }
#pragma unroll
  for (int fc = 0; fc < F; ++fc)
#pragma unroll
    for (int fr = 0; fr < F; ++fr)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = wc * WT + fc * 16 + Mf::row(lane, r);
        const int64_t row = row0 + wr * WT + fr * 16 + l16;
        if (row <= rlast && col < jb) A[row + (k0 + col) * lda] = acc[fc][fr][r];
      }
}

// Inverses of the diagonal 64 x 64 blocks of the lower (UPPER: upper)
// triangle of the n x n M, one workgroup per block, all blocks at once: lane
// j solves T x = e_j by substitution (x in registers, the triangle in LDS)
// for column j of the inverse. inv + 4096 p receives block p's inverse,
// column-major with ld 64; rows and columns past the block's size are those
// of the identity.
template <typename T, bool UPPER>
__global__ __launch_bounds__(64) void trtri_blocks_kernel(const T* __restrict__ M, int64_t ldm,
                                                          int64_t n, T* __restrict__ inv) {
  __shared__ T L[kB][kB + 1];  // L[r][c] = M(r0 + r, r0 + c) on the stored triangle
  const int64_t r0 = int64_t(blockIdx.x) * kB;
  const int jb = int(std::min<int64_t>(kB, n - r0));
  const int t = threadIdx.x;
  {
    T x[kB];  // column c of the block, coalesced down the rows
#pragma unroll
    for (int c = 0; c < kB; ++c) x[c] = M[(r0 + std::min(t, jb - 1)) + (r0 + std::min(c, jb - 1)) * ldm];
#pragma unroll
    for (int c = 0; c < kB; ++c) materialize(x[c]);
#pragma unroll
    for (int c = 0; c < kB; ++c) {
      const bool tri = UPPER ? c >= t : c <= t;
      L[t][c] = (t < jb && c < jb && tri) ? x[c] : (t == c ? T(1) : T(0));
    }
  }
  __syncthreads();
  T x[kB];
#pragma unroll
  for (int c = 0; c < kB; ++c) x[c] = c == t ? T(1) : T(0);
  if (!UPPER) {
#pragma unroll
    for (int c = 0; c < kB; ++c) {
      T s[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < c; ++k) s[k & 3] += L[c][k] * x[k];
      x[c] = (x[c] - ((s[0] + s[1]) + (s[2] + s[3]))) / L[c][c];
    }
  } else {
#pragma unroll
    for (int c = kB - 1; c >= 0; --c) {
      T s[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = c + 1; k < kB; ++k) s[k & 3] += L[c][k] * x[k];
      x[c] = (x[c] - ((s[0] + s[1]) + (s[2] + s[3]))) / L[c][c];
    }
  }
  T* out = inv + int64_t(blockIdx.x) * kB * kB + t * kB;
#pragma unroll
  for (int c = 0; c < kB; ++c) out[c] = x[c];
}

// ------------------------------------------------------------ tridiagonal

// The three diagonals of S into contiguous arrays: sub[i] = S[i+1][i],
// dia[i] = S[i][i], sup[i] = S[i][i+1] (the last sub and sup are zero).
template <typename T>
__global__ __launch_bounds__(256) void tridiag_extract_kernel(int64_t n, const T* __restrict__ S,
                                                              int64_t lds, T* sub, T* dia, T* sup) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  dia[i] = S[i + i * lds];
  sub[i] = i + 1 < n ? S[(i + 1) + i * lds] : T(0);
  sup[i] = i + 1 < n ? S[i + (i + 1) * lds] : T(0);
}

// The right-hand sides pass through LDS in tiles of kGR rows x 64 columns.
// A workgroup has three waves: wave 0 runs the sequential sweep over the
// rows of one tile while wave 1 stages the tiles after it and wave 2 writes
// the one before it back to X, so that the global traffic and the staging
// are off the chain of rows (a wave counts at most 63 memory instructions
// in flight, and a tile takes 64 loads and 64 stores). Wave 1 loads a tile
// with one lane per row (each load instruction reads 64 consecutive rows of
// one column, one coalesced run) into registers a step before it stores it
// to LDS, so that the loads are in flight across a step; the sweep reads it
// with one lane per column. Four buffers: the tile being swept, the next one
// (whose first row the forward sweep reads), the one being staged and the
// one being written back.
constexpr int kGR = 64;
constexpr int kGBuf = 4;
// Rows per group of the sweeps: their LDS operands are read together.
constexpr int kGU = 8;

template <typename T>
struct TileRegs {
  T v[64];  // the tile's row (one per lane) in each of the 64 columns
  T c[3];   // three matrix coefficients of the lane's row
};

// Loads rows [t kGR, t kGR + kGR) of the 64 columns col0 .. (clamped past n
// and nrhs; those values are never used); lane = row in the tile.
template <typename T>
__device__ __forceinline__ void tile_load(TileRegs<T>& R, const T* X, int64_t ldx, int64_t n,
                                          int64_t t, int64_t col0, int64_t nrhs, int lane) {
  const int64_t r = std::min<int64_t>(t * kGR + lane, n - 1);
#pragma unroll
  for (int c = 0; c < 64; ++c) R.v[c] = X[r + std::min<int64_t>(col0 + c, nrhs - 1) * ldx];
}
__device__ __forceinline__ int frexp_exp(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ __forceinline__ int frexp_exp(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ double ldexp2(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ __forceinline__ float ldexp2(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }

// Writes rows [t kGR, t kGR + kGR) of the tile in LDS back (rows < n and
// columns < nrhs only); lane = row in the tile.
template <typename T>
__device__ __forceinline__ void tile_store(const T (*xs)[65], T* X, int64_t ldx, int64_t n,
                                           int64_t t, int64_t col0, int64_t nrhs, int lane) {
  const int64_t r = t * kGR + lane;
  if (r >= n) return;
  const int cols = int(std::min<int64_t>(64, nrhs - col0));
  // 16 columns at a time: their LDS reads are issued together
  for (int c0 = 0; c0 < cols; c0 += 16) {
    T v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = xs[lane][c0 + c];
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c0 + c < cols) X[r + (col0 + c0 + c) * ldx] = v[c];
  }
}

// Forward elimination with partial pivoting of the tridiagonal matrix (sub,
// dia, sup; sup[n - 1] = 0) applied to the right-hand sides in X (lane c of
// wave 0: column col0 + c). The current row i is (d, u, 0) at columns i,
// i+1, i+2; row i+1 is (sub[i], dia[i+1], sup[i+1]); the one of the two with
// the larger entry in column i becomes the pivot row (final row i of U: d',
// u', w', up to a common scale with its right-hand sides), the other is
// eliminated into the new current row. At the end of a tile workgroup 0
// writes its final rows to coef[3 i ..], lane j row i0 + j of the tile that
// starts at row i0; a zero pivot sets info[5].
//
// Staging of a tile (wave 1): each row (its entries l = sub[g - 1] left of
// the diagonal, dia[g], sup[g], and its right-hand sides) is scaled by 2^-k,
// k the exponent of its largest entry, so that products of two rows'
// entries stay in range; l itself is kept for the pivot comparison.
// cs: [l, l 2^-k, dia 2^-k, sup 2^-k][row in tile], ks: k.
template <typename T>
__global__ __launch_bounds__(192) void gtsv_forward_kernel(int64_t n, const T* __restrict__ sub,
                                                           const T* __restrict__ dia,
                                                           const T* __restrict__ sup, T* X,
                                                           int64_t ldx, int64_t nrhs, T* coef,
                                                           int32_t* info) {
  __shared__ T xs[kGBuf][kGR][65];  // [buffer][row in tile][column]
  __shared__ T cs[kGBuf][4][kGR];   // [buffer][as staged][row in tile]
  __shared__ int ks[kGBuf][kGR];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t col0 = int64_t(blockIdx.x) * 64;
  const int64_t nt = (n + kGR - 1) / kGR;
  // wave 1: fetch(t) loads tile t into R, put(t) stages R into LDS
  TileRegs<T> R;
  auto fetch = [&](int64_t t) {
    tile_load(R, X, ldx, n, t, col0, nrhs, lane);
    const int64_t g = std::min<int64_t>(t * kGR + lane, n - 1);
    R.c[0] = g > 0 ? sub[g - 1] : T(0);
    R.c[1] = dia[g];
    R.c[2] = sup[g];
  };
  auto put = [&](int64_t t) {
    const int k = frexp_exp(fmax(fabs(R.c[0]), fmax(fabs(R.c[1]), fabs(R.c[2]))));
    T(*x)[65] = xs[t % kGBuf];
    T(*c)[kGR] = cs[t % kGBuf];
#pragma unroll
    for (int j = 0; j < 64; ++j) x[lane][j] = ldexp2(R.v[j], -k);
    c[0][lane] = R.c[0];
#pragma unroll
    for (int q = 0; q < 3; ++q) c[1 + q][lane] = ldexp2(R.c[q], -k);
    ks[t % kGBuf][lane] = k;
  };
  if (wave == 1) {
    for (int64_t t = 0; t < std::min<int64_t>(nt, 2); ++t) {
      fetch(t);
      put(t);
    }
    if (nt > 2) fetch(2);
  }
  // row 0 as it is (sc = 1; its staged copy could need sc = 2^-k0 out of range)
  T d = dia[0], u = sup[0], sc = T(1);
  T b = X[std::min<int64_t>(col0 + lane, nrhs - 1) * ldx];
  T sd = T(0), su = T(0);  // current row i0 + lane (d, u) as it stood
  bool singular = false;
  __syncthreads();
  for (int64_t t = 0; t < nt; ++t) {
    if (wave == 2) {
      if (t >= 1) tile_store(xs[(t - 1) % kGBuf], X, ldx, n, t - 1, col0, nrhs, lane);
    } else if (wave == 1) {  // tile t + 2 was fetched in the previous step
      if (t + 2 < nt) put(t + 2);
      if (t + 3 < nt) fetch(t + 3);
    } else {
      const int64_t i0 = t * kGR;
      const int cur = int(t % kGBuf), nxt = int((t + 1) % kGBuf);
      const int steps = int(std::min<int64_t>(i0 + kGR, n - 1) - i0);  // rows i0 .. i0 + steps - 1
      // One step on rows i = i0 + q and i + 1. The current row i (d, u, 0, b)
      // is held as sc times its value in the elimination; row i + 1 is (l1,
      // d1, u1, b1) as staged, 2^-k times its value, and lo its entry l1 as it
      // is. The row with the larger entry in column i is the pivot row, final
      // row i (either scaling of it serves the back substitution). Up to its
      // scale, the new current row is d (row i + 1) - l1 (row i) whichever row
      // pivots; its scale is 2^-k times the pivot's magnitude piv = max(|d|,
      // sc |lo|), and the power of two of piv is taken out (sc back in [1/2,
      // 1)). The choice depends on the matrix alone, the same on every lane,
      // and only selects the final row: no division, and one multiply-add, a
      // maximum and a power-of-two rescaling on the chain of rows.
      // Final row i is row i (d, u, 0) if bit q of keeps is set, else row i
      // + 1 as staged; the rows are put together at the end of the tile.
      uint64_t keeps = 0;
      auto step = [&](int q, T lo, T l1, T d1, T u1, int k, T b1) {
        const T sl = sc * fabs(lo);
        const bool keep = fabs(d) >= sl;
        keeps |= __builtin_amdgcn_ballot_w64(keep) & (uint64_t(1) << q);
        singular = singular || (keep && d == T(0));  // |l1| > 0 when row i + 1 pivots
        const bool mine = lane == q;
        sd = mine ? d : sd;
        su = mine ? u : su;
        xs[cur][q][lane] = keep ? b : b1;
        const T piv = fmax(fabs(d), sl);
        const int ep = frexp_exp(piv), e = ep - k;
        const T nd = d * d1 - l1 * u, nu = d * u1, nb = d * b1 - l1 * b;
        sc = ldexp2(piv, -ep);
        d = ldexp2(nd, -e);
        u = ldexp2(nu, -e);
        b = ldexp2(nb, -e);
      };
      // row r of this tile or (r = kGR) the first row of the next one
      auto next_row = [&](int r, T& lo, T& l1, T& d1, T& u1, int& k, T& b1) {
        const int bq = r < kGR ? cur : nxt, rr = r & (kGR - 1);
        lo = cs[bq][0][rr];
        l1 = cs[bq][1][rr];
        d1 = cs[bq][2][rr];
        u1 = cs[bq][3][rr];
        k = ks[bq][rr];
        b1 = xs[bq][rr][lane];
      };
      // kGU steps at a time: their operands are read from LDS before the
      // first of them, off the chain of rows
      int q = 0;
      for (; q + kGU <= steps; q += kGU) {
        T lo[kGU], l1[kGU], d1[kGU], u1[kGU], b1[kGU];
        int k[kGU];
#pragma unroll
        for (int j = 0; j < kGU; ++j) next_row(q + 1 + j, lo[j], l1[j], d1[j], u1[j], k[j], b1[j]);
#pragma unroll
        for (int j = 0; j < kGU; ++j) step(q + j, lo[j], l1[j], d1[j], u1[j], k[j], b1[j]);
      }
      for (; q < steps; ++q) {
        T lo, l1, d1, u1, b1;
        int k;
        next_row(q + 1, lo, l1, d1, u1, k, b1);
        step(q, lo, l1, d1, u1, k, b1);
      }
      if (t == nt - 1) {  // the last row
        singular = singular || d == T(0);
        keeps |= uint64_t(1) << steps;
        const bool mine = lane == steps;
        sd = mine ? d : sd;
        su = mine ? T(0) : su;
        xs[cur][steps][lane] = b;
      }
      if (blockIdx.x == 0 && i0 + lane < n) {
        const bool kp = (keeps >> lane) & 1;
        const int bq = lane + 1 < kGR ? cur : nxt, rr = (lane + 1) & (kGR - 1);
        coef[3 * (i0 + lane)] = kp ? sd : cs[bq][1][rr];
        coef[3 * (i0 + lane) + 1] = kp ? su : cs[bq][2][rr];
        coef[3 * (i0 + lane) + 2] = kp ? T(0) : cs[bq][3][rr];
      }
    }
    __syncthreads();
  }
  if (wave == 2) tile_store(xs[(nt - 1) % kGBuf], X, ldx, n, nt - 1, col0, nrhs, lane);
  if (wave == 0 && singular && lane == 0 && blockIdx.x == 0) info[5] = 1;
}

// Back substitution with the rows coef: x_i = b_i / d'_i - (u'_i / d'_i)
// x_{i+1} - (w'_i / d'_i) x_{i+2}, tiles taken from the last one down, the
// sweep on wave 0, the staging on wave 1 and the write-back on wave 2 as above. The
// three scalings are made for a whole tile as it is staged, off the chain of
// rows, which is then one multiply-add per row: x_i = t_i - (u'_i / d'_i)
// x_{i+1}, with t_i = b_i / d'_i - (w'_i / d'_i) x_{i+2} formed a row earlier.
template <typename T>
__global__ __launch_bounds__(192) void gtsv_backward_kernel(int64_t n, const T* __restrict__ coef,
                                                            T* X, int64_t ldx, int64_t nrhs) {
  __shared__ T xs[kGBuf][kGR][65];
  __shared__ T cs[kGBuf][2][kGR];  // [buffer][u' / d', w' / d'][row in tile]
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t col0 = int64_t(blockIdx.x) * 64;
  const int64_t nt = (n + kGR - 1) / kGR;
  // wave 1: fetch(t) loads tile t into R, put(t) stages R into LDS
  TileRegs<T> R;
  auto fetch = [&](int64_t t) {
    tile_load(R, X, ldx, n, t, col0, nrhs, lane);
    const int64_t g = std::min<int64_t>(t * kGR + lane, n - 1);
#pragma unroll
    for (int q = 0; q < 3; ++q) R.c[q] = coef[3 * g + q];
  };
  auto put = [&](int64_t t) {
    const T rd = T(1) / R.c[0];
    T(*x)[65] = xs[t % kGBuf];
#pragma unroll
    for (int j = 0; j < 64; ++j) x[lane][j] = R.v[j] * rd;
    cs[t % kGBuf][0][lane] = R.c[1] * rd;
    cs[t % kGBuf][1][lane] = R.c[2] * rd;
  };
  if (wave == 1) {
    fetch(nt - 1);
    put(nt - 1);
    if (nt > 1) fetch(nt - 2);
  }
  __syncthreads();
  T x1 = T(0), x2 = T(0);
  for (int64_t t = nt - 1; t >= 0; --t) {
    if (wave == 2) {
      if (t + 1 < nt) tile_store(xs[(t + 1) % kGBuf], X, ldx, n, t + 1, col0, nrhs, lane);
    } else if (wave == 1) {  // tile t - 1 was fetched in the previous step
      if (t >= 1) put(t - 1);
      if (t >= 2) fetch(t - 2);
    } else {
      const int64_t i0 = t * kGR;
      const int cur = int(t % kGBuf);
      auto row = [&](int q, T b, T cu, T cw) {
        const T xi = (b - cw * x2) - cu * x1;
        xs[cur][q][lane] = xi;
        x2 = x1;
        x1 = xi;
      };
      int q = int(std::min<int64_t>(i0 + kGR, n) - i0) - 1;  // rows i0 + q down to i0
      for (; q >= kGU - 1; q -= kGU) {
        T b[kGU], cu[kGU], cw[kGU];
#pragma unroll
        for (int k = 0; k < kGU; ++k) {
          b[k] = xs[cur][q - k][lane];
          cu[k] = cs[cur][0][q - k];
          cw[k] = cs[cur][1][q - k];
        }
#pragma unroll
        for (int k = 0; k < kGU; ++k) row(q - k, b[k], cu[k], cw[k]);
      }
      for (; q >= 0; --q) row(q, xs[cur][q][lane], cs[cur][0][q], cs[cur][1][q]);
    }
    __syncthreads();
  }
  if (wave == 2) tile_store(xs[0], X, ldx, n, 0, col0, nrhs, lane);
}

// ------------------------------------------------------------- host side

template <typename T>
hipError_t chol_panel(T* A, int64_t lda, int64_t n, int64_t k0, int32_t* info, T* inv,
                      hipStream_t s) {
  const int jb = int(std::min<int64_t>(kB, n - k0));
  T* d = inv + (k0 / kB) * kB * kB;  // this diagonal block's inverse
  hipLaunchKernelGGL((potrf_block_kernel<T>), dim3(1), dim3(256), 0, s, A, lda, k0, jb, info, d);
  hipError_t e = hipGetLastError();
  const int64_t m = n - k0 - jb;
  if (e != hipSuccess || m <= 0) return e;
  // L21 = A21 L11^-T in place
  hipLaunchKernelGGL((trsm_right_kernel<T>), dim3(unsigned(cdiv(m, kB))), dim3(256), 0, s, A, lda,
                     k0, jb, m, d);
  return hipGetLastError();
}

// Right-looking by 64-column blocks; the trailing matrix takes
// A22 -= L21 L21^T on its lower tiles (the factorisation reads only the lower
// triangle). With lookahead the update is split: the next block column's
// part on s, directly followed by that block's factorisation, and the part
// right of it on side->s, overlapping the factorisation; the next split
// update waits for it (both write the columns right of the next block).
constexpr int64_t kCholInline = 3072;

template <typename T>
hipError_t chol_factor_typed(int dtype, int64_t n, T* A, int64_t lda, int32_t* info, T* inv,
                             hipStream_t s, const Lookahead* side) {
  const int64_t np = cdiv(n, kB);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return e;
  const bool lookahead = side && side->s && np >= 3 && cap == hipStreamCaptureStatusNone;
  bool pending = false;  // side->s holds an update that the next one must follow
  if ((e = chol_panel<T>(A, lda, n, 0, info, inv, s)) != hipSuccess) return e;
  for (int64_t p = 0; p + 1 < np; ++p) {
    const int64_t k0 = p * kB, k1 = k0 + kB;  // this block, the next
    const int64_t m = n - k1;                  // rows below this block
    const int64_t near = std::min<int64_t>(kB, m);
    const T* W = A + k1 + k0 * lda;  // L21, m x 64
    if (pending) {
      if ((e = hipStreamWaitEvent(s, side->done, 0)) != hipSuccess) return e;
      pending = false;
    }
    // Below kCholInline rows the whole update on s costs less than the two
    // event operations (about 7 us each) and the near part that the
    // lookahead puts on the critical path.
    if (!lookahead || near == m || m <= kCholInline) {
      e = syrk_lower_update_launch(dtype, m, kB, W, lda, A + k1 + k1 * lda, lda, s);
    } else {
      // columns k1 .. k1 + 64 (all rows from k1) on s; the rest on side->s,
      // which needs only L21, so it is released before the near part starts
      e = hipEventRecord(side->ready, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->ready, 0);
      if (e == hipSuccess)
        e = syrk_lower_update_launch(dtype, m - near, kB, W + near, lda,
                                     A + (k1 + near) + (k1 + near) * lda, lda, side->s);
      if (e == hipSuccess) e = hipEventRecord(side->done, side->s);
      pending = e == hipSuccess;
      if (e == hipSuccess)
        e = rank_update_bt_launch(dtype, m, near, kB, W, lda, W, lda, A + k1 + k1 * lda, lda, s);
    }
    if (e != hipSuccess) return e;
    if ((e = chol_panel<T>(A, lda, n, k1, info, inv, s)) != hipSuccess) return e;
  }
  if (pending) e = hipStreamWaitEvent(s, side->done, 0);
  return e;
}

// X <- M^-1 X in place: which 0: M = L L^T (L the lower triangle), 1: M = L
// (lower), 2: M = U (upper). The diagonal blocks' inverses first (one
// launch, unless the Cholesky left them), then the one-launch blocked solve
// per direction (L forward, L^T or U backward).
template <typename T>
hipError_t tri_solve_typed(int dtype, int which, int64_t n, int64_t r, const T* M, int64_t ldm,
                           T* X, int64_t ldx, T* work, bool have_inv, int32_t* status,
                           hipStream_t s) {
  const int64_t np = cdiv(n, kB);
  T* inv = work;
  void* cw = work + np * kB * kB;  // 256-byte aligned: np * 64^2 elements
  if (!have_inv) {
    if (which == 2)
      hipLaunchKernelGGL((trtri_blocks_kernel<T, true>), dim3(unsigned(np)), dim3(kB), 0, s, M,
                         ldm, n, inv);
    else
      hipLaunchKernelGGL((trtri_blocks_kernel<T, false>), dim3(unsigned(np)), dim3(kB), 0, s, M,
                         ldm, n, inv);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t bs = int64_t(kB) * kB;
  if (which == 0)
    return tri_chain_launch(dtype, n, r, M, ldm, 0, inv, bs, 2, inv, bs, X, ldx, cw, status, s);
  return tri_chain_launch(dtype, n, r, M, ldm, which == 1 ? 0 : 1, inv, bs, -1, nullptr, 0, X,
                          ldx, cw, status, s);
}

}  // namespace

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

hipError_t chol_factor_launch(int dtype, int64_t n, void* A, int64_t lda, int32_t* info,
                              void* work, hipStream_t s, const Lookahead* side) {
  if (n <= 0) return hipSuccess;
  if (dtype == 0)
    return chol_factor_typed<double>(0, n, static_cast<double*>(A), lda, info,
                                     static_cast<double*>(work), s, side);
  return chol_factor_typed<float>(1, n, static_cast<float*>(A), lda, info,
                                  static_cast<float*>(work), s, side);
}

size_t tri_solve_workspace_bytes(int dtype, int64_t n, int64_t nrhs) {
  const size_t esz = dtype == 0 ? 8 : 4;
  return esz * size_t(cdiv(n, kB) * kB * kB) + tri_chain_work_bytes(dtype, n, nrhs);
}

hipError_t tri_solve_launch(int dtype, int which, int64_t n, int64_t nrhs, const void* M,
                            int64_t ldm, void* X, int64_t ldx, void* work, bool have_inv,
                            int32_t* status, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (dtype == 0)
    return tri_solve_typed<double>(0, which, n, nrhs, static_cast<const double*>(M), ldm,
                                   static_cast<double*>(X), ldx, static_cast<double*>(work),
                                   have_inv, status, s);
  return tri_solve_typed<float>(1, which, n, nrhs, static_cast<const float*>(M), ldm,
                                static_cast<float*>(X), ldx, static_cast<float*>(work), have_inv,
                                status, s);
}

hipError_t gtsv_launch(int dtype, int64_t n, int64_t nrhs, const void* S, int64_t lds, void* X,
                       int64_t ldx, void* work, int32_t* info, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  const unsigned g = unsigned(cdiv(nrhs, 64)), ge = unsigned(cdiv(n, 256));
  if (dtype == 0) {
    double* w = static_cast<double*>(work);
    hipLaunchKernelGGL((tridiag_extract_kernel<double>), dim3(ge), dim3(256), 0, s, n,
                       static_cast<const double*>(S), lds, w + 3 * n, w + 4 * n, w + 5 * n);
    hipLaunchKernelGGL((gtsv_forward_kernel<double>), dim3(g), dim3(192), 0, s, n, w + 3 * n,
                       w + 4 * n, w + 5 * n, static_cast<double*>(X), ldx, nrhs, w, info);
    hipLaunchKernelGGL((gtsv_backward_kernel<double>), dim3(g), dim3(192), 0, s, n, w,
                       static_cast<double*>(X), ldx, nrhs);
  } else {
    float* w = static_cast<float*>(work);
    hipLaunchKernelGGL((tridiag_extract_kernel<float>), dim3(ge), dim3(256), 0, s, n,
                       static_cast<const float*>(S), lds, w + 3 * n, w + 4 * n, w + 5 * n);
    hipLaunchKernelGGL((gtsv_forward_kernel<float>), dim3(g), dim3(192), 0, s, n, w + 3 * n,
                       w + 4 * n, w + 5 * n, static_cast<float*>(X), ldx, nrhs, w, info);
    hipLaunchKernelGGL((gtsv_backward_kernel<float>), dim3(g), dim3(192), 0, s, n, w,
                       static_cast<float*>(X), ldx, nrhs);
  }
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
