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
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace hexla {
namespace k {

namespace {

constexpr int kStatusSingular = 5;

template <typename T>
__device__ __forceinline__ T bexp(T x);
template <>
__device__ __forceinline__ float bexp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double bexp<double>(double x) { return exp(x); }

template <typename T, int PB, int NT>
struct Smem {
  T slots[kBMaxSlots][kBMaxN];
  T panel[kBMaxN * PB];  // LU panel; reused as the GEMV reduction buffer
  T ustage[PB * 64];     // A12 chunk of the trailing update [column][k]; L11^-1
  int piv[kBMaxN];
  double red_v[NT / 64];
  int red_i[NT / 64];
  int q;
  int swapped;
};

template <typename T>
__device__ __forceinline__ T operand(uint8_t a, const BInst* I, T (*slots)[kBMaxN], int i) {
  if (a & kBSlotBit) return slots[a & 0x7f][i];
  return static_cast<const T*>(I->leaf[a])[i];
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

// y = alpha * M x, M n x n (ld). Wave w takes columns w, w + NW, ...; lane l
// rows l + 64 r; the per-wave partial sums are added through LDS.
template <typename T, int NT>
__device__ void gemv_n(const T* __restrict__ M, int64_t ld, int n, T alpha, const T* x, T* y,
                       T* red) {
  constexpr int NW = NT / 64;
  constexpr int R = kBMaxN / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = T(0);
  for (int j = wave; j < n; j += NW) {
    const T xj = x[j];
    const T* col = M + int64_t(j) * ld;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      if (i < n) acc[r] += col[i] * xj;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
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

// y = alpha * M^T x: one wave per output entry, lanes over the column.
template <typename T, int NT>
__device__ void gemv_t(const T* __restrict__ M, int64_t ld, int n, T alpha, const T* x, T* y) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = wave; j < n; j += NW) {
    const T* col = M + int64_t(j) * ld;
    T acc = 0;
    for (int i = lane; i < n; i += 64) acc += col[i] * x[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) y[j] = alpha * acc;
  }
}

// Solves S y = x for one instance by Gaussian elimination with partial
// pivoting on the augmented matrix [S | x] (n x (n+1) in W, ld n): the right-
// hand side rides along as column n, so the multipliers L are never stored
// outside the panel. Panels of PB columns are factored in LDS (pivot = first
// largest |value| of the column, as in GEPP); the panel's row interchanges
// are applied to the columns on its right, and one rank-PB update with the
// panel rewritten as G = [I - L11^-1 ; L21 L11^-1] turns the rows k0.. of
// those columns into U12 = L11^-1 A12 and A22 - L21 U12 (no separate
// triangular solve). Then back substitution U y = c. y may be x.
template <typename T, int PB, int NT>
__device__ void batch_solve(const T* __restrict__ S, int64_t lds, int n, const T* x, T* y,
                            T* __restrict__ W, Smem<T, PB, NT>& sm, int32_t* status,
                            int instance) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ldw = n;
  const int ncol = n + 1;
  T* panel = sm.panel;
  for (int j = 0; j < n; ++j)
    for (int i = tid; i < n; i += NT) W[i + j * ldw] = S[i + j * lds];
  for (int i = tid; i < n; i += NT) W[i + int64_t(n) * ldw] = x[i];
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += PB) {
    const int jb = min(PB, n - k0), m = n - k0;
    for (int c = 0; c < jb; ++c)
      for (int r = tid; r < m; r += NT) panel[r + c * m] = W[(k0 + r) + int64_t(k0 + c) * ldw];
    if (tid == 0) sm.swapped = 0;
    __syncthreads();
    for (int j = 0; j < jb; ++j) {
      double bv = -1.0;
      int bi = 1 << 30;
      for (int r = j + tid; r < m; r += NT) {
        const double a = fabs(double(panel[r + j * m]));
        if (a > bv) {  // a thread visits its rows in increasing order
          bv = a;
          bi = r;
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double v2 = __shfl_xor(bv, off, 64);
        const int i2 = __shfl_xor(bi, off, 64);
        if (v2 > bv || (v2 == bv && i2 < bi)) {
          bv = v2;
          bi = i2;
        }
      }
      if (lane == 0) {
        sm.red_v[wave] = bv;
        sm.red_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double v = sm.red_v[0];
        int i = sm.red_i[0];
        for (int w = 1; w < NW; ++w)
          if (sm.red_v[w] > v || (sm.red_v[w] == v && sm.red_i[w] < i)) {
            v = sm.red_v[w];
            i = sm.red_i[w];
          }
        if (i >= m) i = j;  // no candidate compared (NaN column): keep the row
        sm.piv[k0 + j] = k0 + i;
        if (i != j) sm.swapped = 1;
        if (!(v > 0.0) && atomicCAS(status, 0, kStatusSingular) == 0) status[2] = instance;
      }
      __syncthreads();
      const int p = sm.piv[k0 + j] - k0;
      if (p != j)
        for (int c = tid; c < jb; c += NT) {
          const T t = panel[j + c * m];
          panel[j + c * m] = panel[p + c * m];
          panel[p + c * m] = t;
        }
      __syncthreads();
      const T piv = panel[j + j * m];
      if (piv != T(0))
        for (int r = j + 1 + tid; r < m; r += NT) {
          const T l = panel[r + j * m] / piv;
          panel[r + j * m] = l;
          for (int c = j + 1; c < jb; ++c) panel[r + c * m] -= l * panel[j + c * m];
        }
      __syncthreads();
    }
    // U11 back to W (L11 below its diagonal is not needed there)
    for (int c = 0; c < jb; ++c)
      for (int r = tid; r <= min(c, jb - 1); r += NT)
        W[(k0 + r) + int64_t(k0 + c) * ldw] = panel[r + c * m];
    const int c0 = k0 + jb;
    if (c0 < ncol) {
      // the panel's row interchanges on the columns to its right
      if (sm.swapped)
        for (int c = c0 + tid; c < ncol; c += NT) {
          T* col = W + int64_t(c) * ldw;
          for (int j = 0; j < jb; ++j) {
            const int pr = sm.piv[k0 + j];
            if (pr != k0 + j) {
              const T t = col[k0 + j];
              col[k0 + j] = col[pr];
              col[pr] = t;
            }
          }
        }
      // Linv = L11^-1 (unit lower), one thread per column, into ustage
      T* linv = sm.ustage;  // [i + c * PB], reused below after a barrier
      if (tid < jb) {
        const int c = tid;
        for (int i = 0; i < jb; ++i) {
          T s = i == c ? T(1) : T(0);
          if (i > c)
            for (int l = c; l < i; ++l) s -= panel[i + l * m] * linv[l + c * PB];
          linv[i + c * PB] = s;
        }
      }
      __syncthreads();
      // G = [I - Linv ; L21 Linv] overwrites the panel, so that one update
      // A(k0.., right) -= G A12 gives U12 = Linv A12 in the top jb rows and
      // A22 - L21 U12 below them. Row r of L21 Linv is built in place in
      // increasing column order (column c reads L21(r, l) for l >= c only).
      for (int r = jb + tid; r < m; r += NT)
        for (int c = 0; c < jb; ++c) {
          T s = 0;
          for (int l = c; l < jb; ++l) s += panel[r + l * m] * linv[l + c * PB];
          panel[r + c * m] = s;
        }
      for (int e = tid; e < jb * jb; e += NT) {
        const int i = e % jb, c = e / jb;
        panel[i + c * m] = (i == c ? T(1) : T(0)) - (i >= c ? linv[i + c * PB] : T(0));
      }
      __syncthreads();
      // A(k0.., c0..) -= G A12 in chunks of 64 columns. A wave's tile: rows
      // lane + 64 a (a < 4) of a 256-row block by 4 adjacent columns, so the
      // G reads are consecutive across lanes and the A12 reads broadcast.
      for (int cc = c0; cc < ncol; cc += 64) {
        const int nc = min(64, ncol - cc);
        for (int e = tid; e < PB * 64; e += NT) {
          const int kk = e % PB, c = e / PB;
          sm.ustage[kk + c * PB] =
              (kk < jb && c < nc) ? W[(k0 + kk) + int64_t(cc + c) * ldw] : T(0);
        }
        __syncthreads();
        const int ncg = (nc + 3) >> 2, nrb = (m + 255) >> 8;
        for (int t = wave; t < nrb * ncg; t += NW) {
          const int rb = t / ncg, cg = t - rb * ncg;
          T acc[4][4];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
          const T* lp = panel + rb * 256 + lane;
          const T* up = sm.ustage + cg * 4 * PB;
          for (int kk = 0; kk < jb; ++kk) {
            T av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
              av[a] = (rb * 256 + lane + 64 * a < m) ? lp[64 * a + kk * m] : T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = up[kk + b * PB];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
          }
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if (cg * 4 + b >= nc) continue;
            T* col = W + int64_t(cc + cg * 4 + b) * ldw + k0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int r = rb * 256 + lane + 64 * a;
              if (r < m) col[r] -= acc[a][b];
            }
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
  // back substitution U y = c (column n), blocks of up to 64 rows from the
  // bottom: wave 0 solves the diagonal block, then every thread updates the
  // rows above it
  const T* rhs = W + int64_t(n) * ldw;
  for (int i = tid; i < n; i += NT) y[i] = rhs[i];
  __syncthreads();
  for (int r1 = n; r1 > 0; r1 -= 64) {
    const int r0 = max(0, r1 - 64);
    if (wave == 0) {
      T yi = (r0 + lane < r1) ? y[r0 + lane] : T(0);
      for (int i = r1 - 1; i >= r0; --i) {
        T xi = __shfl(yi, i - r0, 64);
        xi = xi / W[i + int64_t(i) * ldw];
        if (lane == i - r0) yi = xi;
        if (lane < i - r0) yi -= W[(r0 + lane) + int64_t(i) * ldw] * xi;
      }
      if (r0 + lane < r1) y[r0 + lane] = yi;
    }
    __syncthreads();
    for (int r = tid; r < r0; r += NT) {
      T s = y[r];
      for (int i = r0; i < r1; ++i) s -= W[r + int64_t(i) * ldw] * y[i];
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
  T* W = scratch + int64_t(blockIdx.x) * scratch_stride;
  for (;;) {
    if (tid == 0) sm.q = int(atomicAdd(queue, 1u));
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(sm.q);
    __syncthreads();
    if (q >= count) break;
    const int idx = order[q];
    const BInst* I = inst + idx;
    const int n = int(I->n);
    for (int o = 0; o < p.n_ops; ++o) {
      const BOp& op = p.ops[o];
      if (op.kind == B_LOAD) {
        const T* src = static_cast<const T*>(I->leaf[op.leaf]);
        for (int i = tid; i < n; i += NT) sm.slots[op.dst][i] = src[i];
      } else if (op.kind == B_GEMV) {
        const T* M = static_cast<const T*>(I->leaf[op.leaf]);
        if (!op.trans)
          gemv_n<T, NT>(M, I->ld[op.leaf], n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst],
                        sm.panel);
        else
          gemv_t<T, NT>(M, I->ld[op.leaf], n, T(op.alpha), sm.slots[op.src], sm.slots[op.dst]);
      } else if (op.kind == B_SOLVE) {
        batch_solve<T, PB, NT>(static_cast<const T*>(I->leaf[op.leaf]), I->ld[op.leaf], n,
                               sm.slots[op.src], sm.slots[op.dst], W, sm, status, idx);
      } else {  // B_EW
        T* out = op.dst == kBOut ? static_cast<T*>(I->out) : sm.slots[op.dst];
        for (int i = tid; i < n; i += NT) {
          const T v = ew_batch<T>(p, op, I, sm.slots, i);
          out[i] = v;
        }
      }
      __syncthreads();
    }
    if (p.out_slot != kBOut)
      for (int i = tid; i < n; i += NT) static_cast<T*>(I->out)[i] = sm.slots[p.out_slot][i];
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
