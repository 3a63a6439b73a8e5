// Batched evaluation: many small, uneven instances of one vector expression
// (e.g. trans(A)*B*v + solve(S,b) + 2*(p % q)) in one persistent launch.
// Each workgroup takes instances from a cost-ordered atomic queue (largest
// first) and runs the expression's program on one instance with every
// intermediate vector in LDS:
//   GEMV   y = alpha op(M) x      the matrix-vector products a chain ending
//                                 in a vector reduces to (ordering, Sec. II)
//   SOLVE  y = S^-1 x             the inv(S)*b rewrite (Sec. I, Sec. II): LU
//                                 with partial pivoting of the augmented
//                                 matrix [S | x], panels of PB columns held
//                                 in registers, then back substitution
//   EW     element-wise program over vectors (the fused loop of Sec. II)
// One workgroup owns an instance, so the cost is latency and the trailing
// matrix's trips through memory: loops that touch global memory issue their
// loads in batches before using them, the trailing update loads its next
// chunk while it computes the current one, and global accesses go through
// global-typed pointers with wave-uniform bases (no flat instructions, whose
// loads would also hold up the LDS wait counter).
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

template <typename T>
__device__ __forceinline__ T bexp(T x);
template <>
__device__ __forceinline__ float bexp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double bexp<double>(double x) { return exp(x); }

// A wave's pivot candidate for one column: |value| as an ordered key (high
// and low words), position, and the candidate's row (rotated, its
// multiplier part zeroed).
template <typename T, int PB, int NW>
struct alignas(16) Pub {
  T row[NW][PB];
  unsigned kh[NW], kl[NW];
  int pos[NW];
};

// Columns per chunk of the trailing update: two chunks of RPT rows per
// thread stay in registers (64 VGPRs) beside the panel's G rows.
template <typename T, int NT>
constexpr int update_chunk() {
  return 64 / (2 * (kBMaxN / NT) * int(sizeof(T) / 4));
}

template <typename T, int PB, int NT>
struct Smem {
  static constexpr int UC = update_chunk<T, NT>();
  T slots[kBMaxSlots][kBMaxN];
  union {
    T red[NT / 64][kBMaxN];  // GEMV: per-wave partial sums
    T ub[64 * 64];           // back substitution: diagonal block of U
    struct {
      alignas(16) T l11[PB][PB];       // pivot rows of the panel, by position
      alignas(16) T linv[PB][PB + 4];   // L11^-1, rows padded (gathers by row)
      alignas(16) T linvt[PB][PB + 4];  // linvt[c][l] = L11^-1(l, c)
      alignas(16) T ust[2][PB][UC];    // A12 chunk [k][column], by chunk parity
    } lu;
  } u;
  Pub<T, PB, NT / 64> pub[2];  // pivot candidates, by column parity
  int q;
};

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Orders a wave's LDS accesses (other lanes' writes become visible to the
// wave's following reads); lanes of one wave need no barrier instruction.
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Workgroup barrier that orders LDS only: global loads and stores in flight
// stay in flight (a full barrier waits for every one of them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// Columns of M a wave takes per step of the FP32 matrix-vector products:
// their loads are in flight together (one memory round trip per step).
constexpr int kGemvCols = 4;

// y = alpha * M x, M n x n (ld). Wave w takes columns w + NW u (u <
// kGemvCols) per step, then steps on by kGemvCols NW; lane l rows l + 64 r
// (loads at clamped rows, so that none sits behind a branch; rows past n are
// never written). Per-wave partial sums are added through LDS.
template <typename T, int NT>
__device__ void gemv_n(gcptr<T> M, int ld, int n, T alpha, const T* x, T* y, T* red) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  T acc[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) acc[r] = T(0);
  for (int j = wave; j < n; j += kGemvCols * NW) {
    T xs[kGemvCols], v[kGemvCols][kR];
#pragma unroll
    for (int u = 0; u < kGemvCols; ++u) {
      const int ju = j + u * NW;
      xs[u] = ju < n ? x[ju] : T(0);
      gcptr<T> c = M + unsigned((ju < n ? ju : j) * ld);
#pragma unroll
      for (int r = 0; r < kR; ++r) v[u][r] = c[unsigned(min(lane + 64 * r, n - 1))];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      T s = v[0][r] * xs[0];
#pragma unroll
      for (int u = 1; u < kGemvCols; ++u) s += v[u][r] * xs[u];
      acc[r] += s;
    }
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

// y = alpha * M^T x: one wave per output entry (kGemvCols at a time), lanes
// over the column (loads at clamped rows, x zero past n).
template <typename T, int NT>
__device__ void gemv_t(gcptr<T> M, int ld, int n, T alpha, const T* x, T* y) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  for (int j = wave; j < n; j += kGemvCols * NW) {
    T a[kGemvCols], v[kGemvCols][kR];
#pragma unroll
    for (int u = 0; u < kGemvCols; ++u) {
      const int ju = j + u * NW;
      gcptr<T> c = M + unsigned((ju < n ? ju : j) * ld);
#pragma unroll
      for (int r = 0; r < kR; ++r) v[u][r] = c[unsigned(min(lane + 64 * r, n - 1))];
    }
#pragma unroll
    for (int u = 0; u < kGemvCols; ++u) {
      a[u] = T(0);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int i = lane + 64 * r;
        a[u] += v[u][r] * (i < n ? x[i] : T(0));
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) a[u] += __shfl_xor(a[u], off, 64);
    }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < kGemvCols; ++u)
        if (j + u * NW < n) y[j + u * NW] = alpha * a[u];
    }
  }
}

// FP64 forms of the two products: column pairs per step, loads behind the
// row bound (the wider FP32 forms cost the FP64 variants the second wave per
// SIMD).
// y = alpha * M x, M n x n (ld). Wave w takes column pairs (w, w + NW),
// (w + 2 NW, ...); lane l rows l + 64 r; per-wave partial sums are added
// through LDS.
template <typename T, int NT>
__device__ void gemv_n_pairs(gcptr<T> M, int ld, int n, T alpha, const T* x, T* y, T* red) {
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
__device__ void gemv_t_pairs(gcptr<T> M, int ld, int n, T alpha, const T* x, T* y) {
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

// GEPP of the m x jb panel P (column-major, ld lp; jb <= PB <= 64, m <=
// kBMaxN). Thread t holds panel rows ("slots") t + NT a in v[a] and never
// hands them to another thread: pos[a] tracks the slot's current position
// (kNone past m), and the interchange of positions j and p at step j only
// relabels two slots. A row is kept rotated so that the current column is
// v[0] (all register indices are static): after step j it turns left by one
// and appends its multiplier (rows below the pivot) or column j itself
// (finished rows). Per column every wave publishes its best candidate
// (largest |a|, lowest position on ties, NaN below every number) with the
// candidate's row, the workgroup meets at one barrier, and every thread
// picks the same winner; the candidate buffers alternate with the column's
// parity, so one barrier per column suffices. On return v[a][c] is column c
// of the factored row: multipliers left of the row's pivot column, U from it
// on (pivot rows), multipliers throughout (the others); zero beyond jb.
template <typename T, int PB, int NT>
__device__ __forceinline__ void panel_factor(gcptr<T> P, int lp, int m, int jb,
                                             Smem<T, PB, NT>& sm, T (&v)[kBMaxN / NT][PB],
                                             int (&pos)[kBMaxN / NT], int32_t* status,
                                             int instance) {
  constexpr int NW = NT / 64;
  constexpr int RPT = kBMaxN / NT;
  constexpr int kNone = 1 << 29;
  static_assert(RPT * NT == kBMaxN && PB <= 64, "panel shape");
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
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
#pragma unroll 1
  for (int j = 0; j < jb; ++j) {
    auto& pub = sm.pub[j & 1];
    // the thread's best candidate, then the wave's: largest key, lowest
    // position among equal keys (positions of non-candidates: INT_MAX)
    unsigned kh = 0u, kl = 0u;
    int kp = 0x7fffffff;
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      const bool cand = (pos[a] >= j) & (pos[a] < m);
      unsigned h, l;
      abs_key(v[a][0], h, l);
      h = cand ? h : 0u;
      l = cand ? l : 0u;
      const int pp = cand ? pos[a] : 0x7fffffff;
      const bool take = (h > kh) | ((h == kh) & ((l > kl) | ((l == kl) & (pp < kp))));
      kh = take ? h : kh;
      kl = take ? l : kl;
      kp = take ? pp : kp;
    }
    const unsigned mh = wave_max_u32(kh);
    const unsigned ml = sizeof(T) == 8 ? wave_max_u32(kh == mh ? kl : 0u) : 0u;
    const int bp = wave_min_i32(((kh == mh) & (kl == ml)) ? kp : 0x7fffffff);
    if (lane == 0) {
      pub.kh[wave] = mh;
      pub.kl[wave] = ml;
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
    unsigned ch[NW], cl[NW];
    int cp[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      ch[q] = pub.kh[q];
      cl[q] = pub.kl[q];
      cp[q] = pub.pos[q];
    }
    unsigned wh = ch[0], wl = cl[0];
    int wp = cp[0], w = 0;
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      const bool take =
          (ch[q] > wh) | ((ch[q] == wh) & ((cl[q] > wl) | ((cl[q] == wl) & (cp[q] < wp))));
      wh = take ? ch[q] : wh;
      wl = take ? cl[q] : wl;
      wp = take ? cp[q] : wp;
      w = take ? q : w;
    }
    T prow[PB];
#pragma unroll
    for (int c = 0; c < PB; ++c) prow[c] = pub.row[w][c];
    const T pv = prow[0];
    const T rp = T(1) / pv;  // multipliers as a * (1 / pivot)
    // |pivot| > 0: key above (1, 0); a zero or NaN pivot flags the instance
    if (tid == 0 && !((wh > 1u) | ((wh == 1u) & (wl > 0u))) &&
        atomicCAS(status, 0, kStatusSingular) == 0)
      status[2] = instance;
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
}

// Solves S y = x for one instance by Gaussian elimination with partial
// pivoting on the augmented matrix [S | x]: the right-hand side rides along
// as column n, so L is never stored. Per panel of PB columns (k0, jb = its
// width, m = n - k0 rows):
//   1. panel_factor leaves the factored rows in registers, by slot.
//   2. L11 (the pivot rows) goes to LDS, U11 to memory; lanes < PB form
//      L11^-1 column by column.
//   3. Each thread turns its rows into rows of G = [I - L11^-1 ; L21 L11^-1]
//      in place, so that one product A(k0.., right) -= G A12 gives U12 =
//      L11^-1 A12 in the pivot rows and A22 - L21 U12 in the others.
//   4. The columns right of the panel (with the right-hand side) are
//      updated in chunks of UC columns: a thread loads its slots' old
//      values (coalesced), the pivot rows' owners stage them as A12 in LDS,
//      and the thread writes its new values at the slots' final positions.
//      The row interchanges of GEPP thus cost nothing extra. Each panel reads
//      one scratch buffer and writes the other (S itself for the first
//      panel), so no thread's store can reach a value another thread has yet
//      to load, and the chunk barriers need to order LDS only. The next
//      chunk is loaded while the current one is computed.
// Then back substitution U y = c; row i of U and of c sits in the buffer its
// panel wrote. The two buffers W and W + half hold (n+1) x (n+2) matrices
// (ld n+1): row n and column n+1 take the stores of empty slots and of
// columns past the end, so every load and store is issued unconditionally.
// y may be x. Offsets are 32-bit: the planner keeps every instance matrix
// within 2^31 bytes.
template <typename T, int PB, int NT>
__device__ void batch_solve(gcptr<T> S, int lds, int n, const T* x, T* y, gptr<T> W, int64_t half,
                            Smem<T, PB, NT>& sm, int32_t* status, int instance) {
  constexpr int RPT = kBMaxN / NT;
  constexpr int UC = Smem<T, PB, NT>::UC;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int ld = n + 1, ncol = n + 1;
  gptr<T> B0 = W, B1 = W + half;
  for (int i = tid; i < n; i += NT) B1[unsigned(i + n * ld)] = x[i];  // read by the first panel
  __syncthreads();
  int p = 0;
  for (int k0 = 0; k0 < n; k0 += PB, ++p) {
    const int jb = min(PB, n - k0), m = n - k0;
    gptr<T> D = (p & 1) ? B1 : B0;             // written by this panel
    gcptr<T> R = (p & 1) ? B0 : B1;            // written by the previous panel
    gcptr<T> P = p == 0 ? S : R;               // columns < n of the matrix being factored
    const int lp = p == 0 ? lds : ld;
    T v[RPT][PB];
    int pos[RPT];
    panel_factor<T, PB, NT>(P + unsigned(k0 + k0 * lp), lp, m, jb, sm, v, pos, status, instance);

    // 2. the pivot rows: whole rows to LDS (the inverse reads below the
    // diagonal), their U part to memory
#pragma unroll
    for (int a = 0; a < RPT; ++a)
      if (pos[a] < jb) {
#pragma unroll
        for (int c = 0; c < PB; ++c) sm.u.lu.l11[pos[a]][c] = v[a][c];
        gptr<T> dr = D + unsigned(k0 + pos[a]);
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (c >= pos[a] && c < jb) dr[unsigned((k0 + c) * ld)] = v[a][c];
      }
    __syncthreads();
    // L11^-1: thread c < PB solves L11 x = e_c for column c (zero above the
    // diagonal and past jb) and writes it as column c of L11^-1 and as row c
    // of the transposed copy. Up to 32 columns the solve runs in registers;
    // a 64-column panel has no registers to spare and reads its own earlier
    // entries back from LDS.
    if (tid < PB) {
      const int c = tid;
      if constexpr (PB <= 32) {
        T xr[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
          T s = i == c ? T(1) : T(0);
#pragma unroll
          for (int l = 0; l < i; ++l) s -= sm.u.lu.l11[i][l] * xr[l];
          xr[i] = (i < jb) & (c < jb) ? s : T(0);
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
          sm.u.lu.linv[i][c] = xr[i];
          sm.u.lu.linvt[c][i] = xr[i];
        }
      } else {
        for (int i = 0; i < PB; ++i) {
          T s = i == c ? T(1) : T(0);
#pragma unroll 4
          for (int l = 0; l < i; ++l) s -= sm.u.lu.l11[i][l] * sm.u.lu.linv[l][c];
          s = (i < jb) & (c < jb) ? s : T(0);
          sm.u.lu.linv[i][c] = s;
          sm.u.lu.linvt[c][i] = s;
        }
      }
    }
    __syncthreads();

    // 3. rows of G in place: the pivot row at position q takes e_q - row q
    // of L11^-1; the others g_c = sum_{l >= c} v_l L11^-1(l, c), for
    // ascending c (g_c needs v_l for l >= c only)
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      if (pos[a] < jb) {
        const int q = pos[a];
#pragma unroll
        for (int c = 0; c < PB; ++c) v[a][c] = (c == q ? T(1) : T(0)) - sm.u.lu.linv[q][c];
      } else {
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          T s = 0;
#pragma unroll
          for (int l = c & ~3; l < PB; ++l) s += v[a][l] * sm.u.lu.linvt[c][l];
          v[a][c] = s;
        }
      }
    }
    // A12 rows past jb stay zero (G is zero there too, but LDS may hold NaN)
    if (jb < PB)
      for (int e = tid; e < 2 * PB * UC; e += NT) {
        const int k = (e / UC) % PB;
        if (k >= jb) sm.u.lu.ust[e / (PB * UC)][k][e % UC] = T(0);
      }

    // 4. trailing update
    int rowc[RPT], rowd[RPT];
#pragma unroll
    for (int a = 0; a < RPT; ++a) {
      rowc[a] = min(tid + NT * a, m - 1);        // slot to load (clamped)
      rowd[a] = pos[a] < m ? k0 + pos[a] : n;    // row to store (row n: no slot)
    }
    auto colp = [&](int col) -> gcptr<T> {  // old column col (<= n) from row k0
      return (p == 0 && col < n ? S + unsigned(col * lds) : R + unsigned(col * ld)) + k0;
    };
    auto load = [&](T (&o)[RPT][UC], int cc) {
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        gcptr<T> cp = colp(min(cc + u, n));
#pragma unroll
        for (int a = 0; a < RPT; ++a) o[a][u] = cp[unsigned(rowc[a])];
      }
    };
    T cur[RPT][UC], nxt[RPT][UC];
    load(cur, k0 + jb);
    int par = 0;
    for (int cc = k0 + jb; cc < ncol; cc += UC) {
      load(nxt, cc + UC);  // past the end it reloads column n
#pragma unroll
      for (int a = 0; a < RPT; ++a)
        if (pos[a] < jb) {
#pragma unroll
          for (int u = 0; u < UC; ++u) sm.u.lu.ust[par][pos[a]][u] = cur[a][u];
        }
      lds_barrier();
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        T w[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) w[u] = sm.u.lu.ust[par][k][u];
#pragma unroll
        for (int a = 0; a < RPT; ++a)
#pragma unroll
          for (int u = 0; u < UC; ++u) cur[a][u] -= v[a][k] * w[u];
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        gptr<T> dc = D + unsigned((cc + u <= n ? cc + u : n + 1) * ld);
#pragma unroll
        for (int a = 0; a < RPT; ++a) dc[unsigned(rowd[a])] = cur[a][u];
      }
#pragma unroll
      for (int a = 0; a < RPT; ++a)
#pragma unroll
        for (int u = 0; u < UC; ++u) cur[a][u] = nxt[a][u];
      par ^= 1;
    }
    __syncthreads();  // this panel's stores are read by the next one
  }

  // back substitution U y = c, blocks of up to 64 rows from the bottom: the
  // diagonal block is staged in LDS and solved by wave 0, then every thread
  // updates the rows above it
  auto urow = [&](int i) -> gcptr<T> { return ((i / PB) & 1 ? B1 : B0) + unsigned(i); };
  for (int i = tid; i < n; i += NT) y[i] = urow(i)[unsigned(n * ld)];
  T* ub = sm.u.ub;  // [i + j * 64]
  for (int r1 = n; r1 > 0; r1 -= 64) {
    const int r0 = max(0, r1 - 64), nb = r1 - r0;
    // the block's upper triangle, FP32: four loads in flight at a time
    // (clamped addresses); FP64 one at a time, since more live registers
    // cost its variants the second wave per SIMD
    constexpr int PER = 64 * 64 / NT, GRP = sizeof(T) == 4 ? 4 : 1;
#pragma unroll 1
    for (int q0 = 0; q0 < PER; q0 += GRP) {
      T u[GRP];
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        const int e = tid + NT * (q0 + q), i = e % 64, j = e / 64;
        u[q] = urow(r0 + min(i, nb - 1))[unsigned((r0 + min(j, nb - 1)) * ld)];
      }
#pragma unroll
      for (int q = 0; q < GRP; ++q) {
        const int e = tid + NT * (q0 + q), i = e % 64, j = e / 64;
        if (j < nb && j >= i) ub[i + j * 64] = u[q];
      }
    }
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
      gcptr<T> ur = urow(r);
      T s = y[r];
#pragma unroll 16
      for (int i = r0; i < r1; ++i) s -= ur[unsigned(i * ld)] * y[i];
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
        if constexpr (sizeof(T) == 4) {
          if (!op.trans)
            gemv_n<T, NT>(M, ld, n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst], &sm.u.red[0][0]);
          else
            gemv_t<T, NT>(M, ld, n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst]);
        } else {
          if (!op.trans)
            gemv_n_pairs<T, NT>(M, ld, n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst],
                                &sm.u.red[0][0]);
          else
            gemv_t_pairs<T, NT>(M, ld, n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst]);
        }
      } else if (op.kind == B_SOLVE) {
        batch_solve<T, PB, NT>(gcptr<T>(I->leaf[op.leaf]), int(I->ld[op.leaf]), n,
                               sm.slots[op.src], sm.slots[op.dst], W, scratch_stride / 2, sm,
                               status, idx);
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
constexpr Variant kF32[] = {{32, 256}, {64, 256}, {16, 256}};
constexpr Variant kF64[] = {{16, 256}, {8, 256}};

template <typename T, int PB, int NT>
void launch_one(int grid, const BProgram* p, const BInst* inst, const int32_t* order, int count,
                unsigned* queue, void* scratch, int64_t stride, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL((batch_kernel<T, PB, NT>), dim3(grid), dim3(NT), 0, s, p, inst, order, count,
                     queue, static_cast<T*>(scratch), stride, status);
}

}  // namespace

int batch_variant_count(int dtype) { return dtype == 0 ? 2 : 3; }

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

// Two (max_n + 1) x (max_n + 2) buffers per workgroup, each 256-byte aligned
// for FP32 and FP64.
int64_t batch_scratch_stride(int64_t max_n) {
  const int64_t e = (max_n + 1) * (max_n + 2);
  return 2 * ((e + 63) & ~int64_t(63));
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
      case 0: HEXLA_BATCH_CASE(double, 16, 256); break;
      default: HEXLA_BATCH_CASE(double, 8, 256); break;
    }
  } else {
    switch (cfg.variant) {
      case 0: HEXLA_BATCH_CASE(float, 32, 256); break;
      case 1: HEXLA_BATCH_CASE(float, 64, 256); break;
      default: HEXLA_BATCH_CASE(float, 16, 256); break;
    }
  }
#undef HEXLA_BATCH_CASE
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
