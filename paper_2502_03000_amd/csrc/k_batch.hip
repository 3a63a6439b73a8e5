// Batched evaluation: many small, uneven instances of one vector expression
// (e.g. trans(A)*B*v + solve(S,b) + 2*(p % q)) in one persistent launch.
// Each workgroup takes instances from a cost-ordered atomic queue (largest
// first) and runs the expression's program on one instance with every
// intermediate vector in LDS:
//   GEMV   y = alpha op(M) x      the matrix-vector products a chain ending
//                                 in a vector reduces to (ordering, Sec. II)
//   SOLVE  y = S^-1 x             the inv(S)*b rewrite (Sec. I, Sec. II): LU
//                                 with partial pivoting of the augmented
//                                 matrix [S | x] in per-workgroup scratch,
//                                 panels of PB columns factored in LDS, then
//                                 back substitution
//   EW     element-wise program over vectors (the fused loop of Sec. II)
// One workgroup owns an instance, so the cost is latency: loops that touch
// global memory issue their loads in batches before using them, the trailing
// update loads its next tile while it computes the current one, and global
// accesses go through global-typed pointers with wave-uniform bases (no flat
// instructions, whose loads would also hold up the LDS wait counter).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "wave_device.h"

namespace hexla {
namespace k {

namespace {

template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
using gcptr = const __attribute__((address_space(1))) T*;

constexpr int kStatusSingular = 5;
constexpr int kR = kBMaxN / 64;  // rows per lane of a full column
constexpr int kCW = 128;         // columns per chunk of the trailing update

template <typename T>
__device__ __forceinline__ T bexp(T x);
template <>
__device__ __forceinline__ float bexp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double bexp<double>(double x) { return exp(x); }

// A wave's pivot candidate for one column: |value|, position, and the
// candidate's row (rotated, its multiplier part zeroed).
template <typename T, int PB, int NW>
struct alignas(16) Pub {
  T row[NW][PB];
  T val[NW];
  int pos[NW];
};

template <typename T, int PB, int NT>
struct Smem {
  T slots[kBMaxSlots][kBMaxN];
  T panel[kBMaxN * PB];  // LU panel; GEMV reduction buffer; diagonal blocks of U
  T ustage[PB * kCW];    // A12 chunk of the trailing update [k][column]; L11^-1
  Pub<T, PB, NT / 64> pub[2];  // per column parity
  int piv[kBMaxN];
  int q;
  int swapped;
};

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Orders a wave's LDS accesses (other lanes' writes become visible to the
// wave's following reads); lanes of one wave need no barrier instruction.
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// dst(i, j) = src(i, j) for i < rows <= kBMaxN, j < cols (element offsets
// i + j * ld). Lane l takes rows l + 64 a, wave w columns w, w + NW, ...; two
// columns of up to kR rows per lane are loaded before any is stored.
template <typename T, int NT, typename D, typename S>
__device__ void copy_block(D dst, int ldd, S src, int lds, int rows, int cols) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  for (int j0 = wave; j0 < cols; j0 += 2 * NW) {
    T v[2][kR];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + NW * b;
#pragma unroll
      for (int a = 0; a < kR; ++a) {
        const int i = lane + 64 * a;
        v[b][a] = (i < rows && j < cols) ? src[unsigned(i + j * lds)] : T(0);
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + NW * b;
#pragma unroll
      for (int a = 0; a < kR; ++a) {
        const int i = lane + 64 * a;
        if (i < rows && j < cols) dst[unsigned(i + j * ldd)] = v[b][a];
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ T operand(uint8_t a, const BInst* I, T (*slots)[kBMaxN], int i) {
  if (a & kBSlotBit) return slots[a & 0x7f][i];
  return gcptr<T>(I->leaf[a])[i];
}

// Element-wise program at element i: the opcodes of the single-expression
// interpreter over a 4-deep stack (s0 is the top).
template <typename T>
__device__ T ew_batch(const BProgram& p, const BOp& op, const BInst* I, T (*slots)[kBMaxN],
                      int i) {
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int pc = op.ew_begin; pc < op.ew_end; ++pc) {
    const int o = p.ew_op[pc];
    const uint8_t a = p.ew_arg[pc];
    if (o == EW_LEAF || o == EW_CONST) {
      const T x = o == EW_LEAF ? operand<T>(a, I, slots, i) : T(p.cst[a]);
      s3 = s2;
      s2 = s1;
      s1 = s0;
      s0 = x;
    } else if (o >= EW_ADD && o <= EW_RDIV) {
      T r;
      switch (o) {
        case EW_ADD: r = s1 + s0; break;
        case EW_SUB: r = s1 - s0; break;
        case EW_MUL: r = s1 * s0; break;
        case EW_DIV: r = s1 / s0; break;
        case EW_RSUB: r = s0 - s1; break;
        default: r = s0 / s1; break;  // EW_RDIV
      }
      s0 = r;
      s1 = s2;
      s2 = s3;
    } else {
      switch (o) {
        case EW_NEG: s0 = -s0; break;
        case EW_EXP: s0 = bexp<T>(s0); break;
        case EW_SCALE: s0 = s0 * T(p.cst[a]); break;
        case EW_ADDC: s0 = s0 + T(p.cst[a]); break;
        case EW_LEAFMUL: s0 = s0 * operand<T>(a, I, slots, i); break;
        default: s0 = s0 + operand<T>(a, I, slots, i); break;  // EW_LEAFADD
      }
    }
  }
  return s0;
}

// y = alpha * M x, M n x n (ld). Wave w takes column pairs (w, w + NW),
// (w + 2 NW, ...); lane l rows l + 64 r; per-wave partial sums are added
// through LDS.
template <typename T, int NT>
__device__ void gemv_n(gcptr<T> M, int ld, int n, T alpha, const T* x, T* y, T* red) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  T acc[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) acc[r] = T(0);
  for (int j = wave; j < n; j += 2 * NW) {
    const int j2 = j + NW;
    const T x1 = x[j], x2 = j2 < n ? x[j2] : T(0);
    gcptr<T> c1 = M + unsigned(j * ld);
    gcptr<T> c2 = M + unsigned((j2 < n ? j2 : j) * ld);
    T v1[kR], v2[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int i = lane + 64 * r;
      v1[r] = i < n ? c1[i] : T(0);
      v2[r] = i < n ? c2[i] : T(0);
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) acc[r] += v1[r] * x1 + v2[r] * x2;
  }
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int i = lane + 64 * r;
    if (i < n) red[wave * kBMaxN + i] = acc[r];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    T s = red[i];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += red[w * kBMaxN + i];
    y[i] = alpha * s;
  }
}

// y = alpha * M^T x: one wave per output entry (two at a time), lanes over
// the column.
template <typename T, int NT>
__device__ void gemv_t(gcptr<T> M, int ld, int n, T alpha, const T* x, T* y) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  for (int j = wave; j < n; j += 2 * NW) {
    const int j2 = j + NW;
    gcptr<T> c1 = M + unsigned(j * ld);
    gcptr<T> c2 = M + unsigned((j2 < n ? j2 : j) * ld);
    T a1 = 0, a2 = 0;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int i = lane + 64 * r;
      if (i < n) {
        const T xi = x[i];
        a1 += c1[i] * xi;
        a2 += c2[i] * xi;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      a1 += __shfl_xor(a1, off, 64);
      a2 += __shfl_xor(a2, off, 64);
    }
    if (lane == 0) {
      y[j] = alpha * a1;
      if (j2 < n) y[j2] = alpha * a2;
    }
  }
}

// GEPP of the m x jb panel P (column-major, ld lp; jb <= PB, m <= kBMaxN)
// into sm.panel (ld m): multipliers below the diagonal, U on and above it,
// rows at their final positions. piv[j] = k0 + the position chosen at step j
// (positions j and piv[j] - k0 are interchanged, as in xGETRF). Each thread
// holds rows tid + NT a in registers; rows never move between threads, each
// tracks its current position instead. A row is kept rotated so that the
// current column is v[0] (all register indices are static): after step j it
// turns left by one and appends its multiplier (rows below the pivot) or
// column j itself (finished rows). Per column every wave publishes its best
// candidate (largest |a|, lowest position on ties, NaN below every number)
// with the candidate's row, the workgroup meets at one barrier, and every
// thread picks the same winner. The candidate buffers alternate with the
// column's parity, so one barrier per column suffices.
template <typename T, int PB, int NT>
__device__ void panel_factor(gcptr<T> P, int lp, int m, int jb, Smem<T, PB, NT>& sm, int* piv,
                             int k0, int32_t* status, int instance) {
  constexpr int NW = NT / 64;
  constexpr int RPT = kBMaxN / NT;
  constexpr int kNone = 1 << 29;  // position of a thread's row slot past m
  static_assert(RPT * NT == kBMaxN, "rows per thread");
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  T v[RPT][PB];
  int pos[RPT];
#pragma unroll
  for (int a = 0; a < RPT; ++a) {
    const int r = tid + NT * a;
    pos[a] = r < m ? r : kNone;
    const int rr = min(r, m - 1);  // clamped: every load is issued unconditionally
#pragma unroll
    for (int c = 0; c < PB; ++c) v[a][c] = P[unsigned(rr + min(c, jb - 1) * lp)];
  }
#pragma unroll
  for (int a = 0; a < RPT; ++a)
#pragma unroll
    for (int c = 0; c < PB; ++c)
      if (pos[a] == kNone || c >= jb) v[a][c] = T(0);
  int swapped = 0;
#pragma unroll 1
  for (int j = 0; j < jb; ++j) {
    auto& pub = sm.pub[j & 1];
    T best = T(-2);
    int bp = -1;
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      T x = fabs(v[a][0]);
      x = x == x ? x : T(-0.5);
      const bool take =
          (pos[a] >= j) & (pos[a] < m) & ((x > best) | ((x == best) & (pos[a] < bp)));
      best = take ? x : best;
      bp = take ? pos[a] : bp;
    }
    wave_argmax(best, bp);
    if (lane == 0) {
      pub.val[wave] = best;
      pub.pos[wave] = bp;
    }
    // the candidate's row as it is; then lanes < j zero its multiplier part
    // (the last j positions) in the wave's own slot, after it in LDS order
#pragma unroll
    for (int a = 0; a < RPT; ++a)
      if (pos[a] == bp) {
#pragma unroll
        for (int c = 0; c < PB; ++c) pub.row[wave][c] = v[a][c];
      }
    wave_fence();
    if (lane < j) pub.row[wave][PB - j + lane] = T(0);
    __syncthreads();
    T cv[NW];
    int cp[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      cv[q] = pub.val[q];
      cp[q] = pub.pos[q];
    }
    T wv = cv[0];
    int wp = cp[0], w = 0;
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      const bool take = (cv[q] > wv) | ((cv[q] == wv) & (cp[q] < wp));
      wv = take ? cv[q] : wv;
      wp = take ? cp[q] : wp;
      w = take ? q : w;
    }
    T prow[PB];
#pragma unroll
    for (int c = 0; c < PB; ++c) prow[c] = pub.row[w][c];
    const T pv = prow[0];
    const T rp = T(1) / pv;  // multipliers as a * (1 / pivot)
    if (tid == 0) {
      piv[j] = k0 + wp;
      if (!(wv > T(0)) && atomicCAS(status, 0, kStatusSingular) == 0) status[2] = instance;
    }
    swapped |= wp != j;
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      pos[a] = pos[a] == wp ? j : (pos[a] == j ? wp : pos[a]);
      const bool act = (pos[a] > j) & (pos[a] < m) & (pv != T(0));
      const T v0 = v[a][0];
      const T l = act ? v0 * rp : T(0);
#pragma unroll
      for (int c = 0; c < PB - 1; ++c) v[a][c] = v[a][c + 1] - l * prow[c + 1];
      v[a][PB - 1] = act ? l : v0;
    }
  }
  // a narrow last panel: turn the rows the rest of the way round
#pragma unroll 1
  for (int j = jb; j < PB; ++j)
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      const T v0 = v[a][0];
#pragma unroll
      for (int c = 0; c < PB - 1; ++c) v[a][c] = v[a][c + 1];
      v[a][PB - 1] = v0;
    }
#pragma unroll
  for (int a = 0; a < RPT; ++a)
    if (pos[a] < m)
#pragma unroll
      for (int c = 0; c < PB; ++c)
        if (c < jb) sm.panel[pos[a] + c * m] = v[a][c];
  if (tid == 0) sm.swapped = swapped;
}

// Solves S y = x for one instance by Gaussian elimination with partial
// pivoting on the augmented matrix [S | x] (n x (n+1) in W, ld n): the right-
// hand side rides along as column n, so the multipliers L are never stored
// outside the panel. Panels of PB columns are factored in registers (pivot =
// first largest |value| of the column, as in GEPP); the panel's row interchanges
// are applied to the columns on its right, and one rank-PB update with the
// panel rewritten as G = [I - L11^-1 ; L21 L11^-1] turns the rows k0.. of
// those columns into U12 = L11^-1 A12 and A22 - L21 U12 (no separate
// triangular solve). Then back substitution U y = c. y may be x.
// The first panel and its update read S itself, so S is copied to W only
// when that panel interchanges rows. Offsets are 32-bit: the planner keeps
// every instance matrix within 2^31 bytes.
template <typename T, int PB, int NT>
__device__ void batch_solve(gcptr<T> S, int lds, int n, const T* x, T* y, gptr<T> W,
                            Smem<T, PB, NT>& sm, int32_t* status, int instance) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int ldw = n;
  const int ncol = n + 1;
  T* panel = sm.panel;
  gcptr<T> Wc = W;
  for (int i = tid; i < n; i += NT) W[unsigned(i + n * ldw)] = x[i];
  gcptr<T> src = S;  // columns < n of the matrix being factored: S for the first panel
  int lsrc = lds;
  for (int k0 = 0; k0 < n; k0 += PB) {
    const int jb = min(PB, n - k0), m = n - k0;
    panel_factor<T, PB, NT>(src + unsigned(k0 + k0 * lsrc), lsrc, m, jb, sm, sm.piv + k0, k0,
                            status, instance);
    __syncthreads();
    // U11 back to W (L11 below its diagonal is not needed there)
    for (int c = 0; c < jb; ++c)
      for (int r = tid; r <= c; r += NT) W[unsigned((k0 + r) + (k0 + c) * ldw)] = panel[r + c * m];
    const int c0 = k0 + jb;
    if (c0 < ncol) {
      if (sm.swapped) {
        if (k0 == 0 && c0 < n) {  // interchanges may not touch S: work on a copy
          copy_block<T, NT>(W + unsigned(c0 * ldw), ldw, S + unsigned(c0 * lds), lds, n, n - c0);
          src = Wc;
          lsrc = ldw;
          __syncthreads();
        }
        // the panel's row interchanges on the columns to its right
        for (int c = c0 + tid; c < ncol; c += NT) {
          gptr<T> col = W + unsigned(c * ldw);
          for (int j = 0; j < jb; ++j) {
            const int pr = sm.piv[k0 + j];
            if (pr != k0 + j) {
              const T t = col[k0 + j];
              col[k0 + j] = col[pr];
              col[pr] = t;
            }
          }
        }
      }
      // Linv = L11^-1 (unit lower): lane c of wave 0 solves L11 x = e_c with
      // x in registers; the result goes to ustage
      T* linv = sm.ustage;  // [i + c * PB], reused below after a barrier
      if (wave == 0 && lane < jb) {
        T xc[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
          T s = i == lane ? T(1) : T(0);
          if (i < jb) {
#pragma unroll
            for (int l = 0; l < i; ++l) s -= panel[i + l * m] * xc[l];
          }
          xc[i] = s;
        }
#pragma unroll
        for (int i = 0; i < PB; ++i)
          if (i < jb) linv[i + lane * PB] = xc[i];
      }
      __syncthreads();
      // G = [I - Linv ; L21 Linv] overwrites the panel, so that one update
      // A(k0.., right) -= G A12 gives U12 = Linv A12 in the top jb rows and
      // A22 - L21 U12 below them. Row r of L21 is held in registers.
      for (int r = jb + tid; r < m; r += NT) {
        T lr[PB];
#pragma unroll
        for (int l = 0; l < PB; ++l) lr[l] = l < jb ? panel[r + l * m] : T(0);
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          if (c >= jb) break;
          T s = 0;
#pragma unroll
          for (int l = c; l < PB; ++l)
            if (l < jb) s += lr[l] * linv[l + c * PB];  // linv is unset beyond jb
          panel[r + c * m] = s;
        }
      }
      for (int e = tid; e < jb * jb; e += NT) {
        const int i = e % jb, c = e / jb;
        panel[i + c * m] = (i == c ? T(1) : T(0)) - (i >= c ? linv[i + c * PB] : T(0));
      }
      __syncthreads();
      // A(k0.., c0..) -= G A12 in chunks of kCW columns; the old values of a
      // column come from src (S for the first panel) except the right-hand
      // side, and the new ones go to W. A wave's tile: rows lane + 64 a
      // (a < 4) of a 256-row block by 4 adjacent columns, so the G reads are
      // consecutive across lanes and the A12 reads broadcast; a column's
      // base address is wave-uniform. Two register tiles alternate: one is
      // loaded while the other is updated. Row blocks that end inside the
      // matrix load and store without masks; the last one clamps its load
      // rows (always valid addresses) and masks its stores. G is read
      // unconditionally (rows past m stay inside the panel array and only
      // feed discarded values).
      gcptr<T> colsrc = k0 == 0 ? src : Wc;
      const int colld = k0 == 0 ? lsrc : ldw;
      auto col_in = [&](int col) -> gcptr<T> {  // column `col` (<= n), row k0
        return (col < n ? colsrc + unsigned(col * colld) : Wc + unsigned(n * ldw)) + k0;
      };
      for (int cc = c0; cc < ncol; cc += kCW) {
        const int nc = min(kCW, ncol - cc);
        static_assert((PB * kCW) % NT == 0, "staging loop");
#pragma unroll
        for (int u = 0; u < PB * kCW / NT; ++u) {
          const int e = tid + NT * u;
          const int kk = e / kCW, c = e % kCW;
          const T v = col_in(cc + min(c, nc - 1))[min(kk, jb - 1)];
          sm.ustage[c + kk * kCW] = (kk < jb && c < nc) ? v : T(0);
        }
        __syncthreads();
        const int ncg = (nc + 3) >> 2, nrb = (m + 255) >> 8, ntile = nrb * ncg;
        auto load = [&](T (&v)[4][4], int t) {
          const int rb = t / ncg, cg = t - rb * ncg;
          const int r0 = rb * 256 + lane;
          const bool full = rb * 256 + 256 <= m;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            gcptr<T> cp = col_in(cc + min(cg * 4 + b, nc - 1));
            if (full) {
#pragma unroll
              for (int a = 0; a < 4; ++a) v[a][b] = cp[unsigned(r0 + 64 * a)];
            } else {
#pragma unroll
              for (int a = 0; a < 4; ++a) v[a][b] = cp[unsigned(min(r0 + 64 * a, m - 1))];
            }
          }
        };
        auto update = [&](T (&v)[4][4], int t) {
          const int rb = t / ncg, cg = t - rb * ncg;
          const int r0 = rb * 256 + lane;
          const T* lp = panel + r0;
          const T* up = sm.ustage + cg * 4;
          // products into fresh registers: the loop never waits for the
          // tile's loads, which are only needed after it
          T acc[4][4];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
          for (int kk = 0; kk < jb; ++kk) {
            T av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = lp[64 * a + kk * m];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = up[kk * kCW + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
          }
          const bool full = rb * 256 + 256 <= m;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if (cg * 4 + b >= nc) continue;
            gptr<T> col = W + unsigned((cc + cg * 4 + b) * ldw + k0);
            if (full) {
#pragma unroll
              for (int a = 0; a < 4; ++a) col[unsigned(r0 + 64 * a)] = v[a][b] - acc[a][b];
            } else {
#pragma unroll
              for (int a = 0; a < 4; ++a)
                if (r0 + 64 * a < m) col[unsigned(r0 + 64 * a)] = v[a][b] - acc[a][b];
            }
          }
        };
        T ta[4][4], tb[4][4];
        if (wave < ntile) load(ta, wave);
        for (int t = wave; t < ntile; t += 2 * NW) {
          if (t + NW < ntile) load(tb, t + NW);
          update(ta, t);
          if (t + NW >= ntile) break;
          if (t + 2 * NW < ntile) load(ta, t + 2 * NW);
          update(tb, t + NW);
        }
        __syncthreads();
      }
    }
    src = Wc;
    lsrc = ldw;
    __syncthreads();
  }
  // back substitution U y = c (column n), blocks of up to 64 rows from the
  // bottom: the diagonal block is staged in LDS and solved by wave 0, then
  // every thread updates the rows above it
  for (int i = tid; i < n; i += NT) y[i] = Wc[unsigned(i + n * ldw)];
  T* ub = sm.panel;  // [i + j * 64]
  for (int r1 = n; r1 > 0; r1 -= 64) {
    const int r0 = max(0, r1 - 64), nb = r1 - r0;
    copy_block<T, NT>(ub, 64, Wc + unsigned(r0 + r0 * ldw), ldw, nb, nb);
    __syncthreads();
    if (wave == 0) {
      T yi = lane < nb ? y[r0 + lane] : T(0);
      for (int i = nb - 1; i >= 0; --i) {
        const T xi = __shfl(yi, i, 64) / ub[i + i * 64];
        if (lane == i) yi = xi;
        if (lane < i) yi -= ub[lane + i * 64] * xi;
      }
      if (lane < nb) y[r0 + lane] = yi;
    }
    __syncthreads();
    for (int r = tid; r < r0; r += NT) {
      T s = y[r];
#pragma unroll 16
      for (int i = r0; i < r1; ++i) s -= Wc[unsigned(r + i * ldw)] * y[i];
      y[r] = s;
    }
    __syncthreads();
  }
}

template <typename T, int PB, int NT>
__global__ __launch_bounds__(NT) void batch_kernel(const BProgram* __restrict__ prog,
                                                   const BInst* __restrict__ inst,
                                                   const int32_t* __restrict__ order, int count,
                                                   unsigned* queue, T* scratch,
                                                   int64_t scratch_stride, int32_t* status) {
  __shared__ Smem<T, PB, NT> sm;
  const BProgram& p = *prog;
  const int tid = threadIdx.x;
  gptr<T> W = gptr<T>(scratch) + int64_t(blockIdx.x) * scratch_stride;
  if (tid == 0) sm.q = int(atomicAdd(queue, 1u));
  __syncthreads();
  for (;;) {
    const int q = __builtin_amdgcn_readfirstlane(sm.q);
    __syncthreads();
    if (q >= count) break;
    // claim the next instance now: the atomic's latency overlaps this one
    int next = 0;
    if (tid == 0) next = int(atomicAdd(queue, 1u));
    const int idx = order[q];
    const BInst* I = inst + idx;
    const int n = int(I->n);
    for (int o = 0; o < p.n_ops; ++o) {
      const BOp& op = p.ops[o];
      if (op.kind == B_LOAD) {
        gcptr<T> src = gcptr<T>(I->leaf[op.leaf]);
        for (int i = tid; i < n; i += NT) sm.slots[op.dst][i] = src[i];
      } else if (op.kind == B_GEMV) {
        gcptr<T> M = gcptr<T>(I->leaf[op.leaf]);
        const int ld = int(I->ld[op.leaf]);
        if (!op.trans)
          gemv_n<T, NT>(M, ld, n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst], sm.panel);
        else
          gemv_t<T, NT>(M, ld, n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst]);
      } else if (op.kind == B_SOLVE) {
        batch_solve<T, PB, NT>(gcptr<T>(I->leaf[op.leaf]), int(I->ld[op.leaf]), n,
                               sm.slots[op.src], sm.slots[op.dst], W, sm, status, idx);
      } else if (op.dst == kBOut) {  // B_EW into the output
        gptr<T> out = gptr<T>(I->out);
        for (int i = tid; i < n; i += NT) out[i] = ew_batch<T>(p, op, I, sm.slots, i);
      } else {  // B_EW into a slot
        for (int i = tid; i < n; i += NT) {
          const T v = ew_batch<T>(p, op, I, sm.slots, i);
          sm.slots[op.dst][i] = v;
        }
      }
      __syncthreads();
    }
    if (p.out_slot != kBOut) {
      gptr<T> out = gptr<T>(I->out);
      for (int i = tid; i < n; i += NT) out[i] = sm.slots[p.out_slot][i];
    }
    if (tid == 0) sm.q = next;
    __syncthreads();
  }
}

__global__ void zero_u32_kernel(unsigned* p) { *p = 0u; }

struct Variant {
  int panel, threads;
};
constexpr Variant kF32[] = {{16, 256}, {16, 512}, {32, 256}, {32, 512}};
constexpr Variant kF64[] = {{8, 256}, {8, 512}, {16, 256}, {16, 512}};

template <typename T, int PB, int NT>
void launch_one(int grid, const BProgram* p, const BInst* inst, const int32_t* order, int count,
                unsigned* queue, void* scratch, int64_t stride, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL((batch_kernel<T, PB, NT>), dim3(grid), dim3(NT), 0, s, p, inst, order, count,
                     queue, static_cast<T*>(scratch), stride, status);
}

}  // namespace

int batch_variant_count(int dtype) { return dtype == 0 ? 4 : 4; }

void batch_variant_shape(int dtype, int variant, int* panel, int* threads) {
  const Variant v = dtype == 0 ? kF64[variant] : kF32[variant];
  *panel = v.panel;
  *threads = v.threads;
}

BatchConfig batch_default(int dtype, int64_t count) {
  (void)dtype;
  (void)count;
  return BatchConfig{0, 512};
}

int64_t batch_scratch_stride(int64_t max_n) {
  const int64_t e = max_n * (max_n + 1);
  return (e + 63) & ~int64_t(63);  // 256-byte aligned slices for FP32 and FP64
}

hipError_t batch_launch(int dtype, const BatchConfig& cfg, const BProgram* p, const BInst* inst,
                        const int32_t* order, int64_t count, unsigned* queue, void* scratch,
                        int64_t scratch_stride, int32_t* status, hipStream_t s) {
  if (cfg.variant < 0 || cfg.variant >= batch_variant_count(dtype) || cfg.grid <= 0 ||
      count > INT32_MAX)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || count == 0) return e;
  const int c = int(count);
#define HEXLA_BATCH_CASE(T, PB, NT) \
  launch_one<T, PB, NT>(cfg.grid, p, inst, order, c, queue, scratch, scratch_stride, status, s)
  if (dtype == 0) {
    switch (cfg.variant) {
      case 0: HEXLA_BATCH_CASE(double, 8, 256); break;
      case 1: HEXLA_BATCH_CASE(double, 8, 512); break;
      case 2: HEXLA_BATCH_CASE(double, 16, 256); break;
      default: HEXLA_BATCH_CASE(double, 16, 512); break;
    }
  } else {
    switch (cfg.variant) {
      case 0: HEXLA_BATCH_CASE(float, 16, 256); break;
      case 1: HEXLA_BATCH_CASE(float, 16, 512); break;
      case 2: HEXLA_BATCH_CASE(float, 32, 256); break;
      default: HEXLA_BATCH_CASE(float, 32, 512); break;
    }
  }
#undef HEXLA_BATCH_CASE
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
