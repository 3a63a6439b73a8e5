// Device-side interpreter of an element-wise program (used by the fused
// element-wise kernel and by the GEMV epilogue).
//
// All control flow depends only on the program, which is identical for every
// lane, so branches are scalar and the value stack lives in registers. V is
// the number of consecutive elements a lane evaluates at once.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace hexla {
namespace k {

template <typename T, int V>
struct Pack {
  T v[V];
};

template <typename T>
__device__ __forceinline__ T ew_exp(T x);
template <>
__device__ __forceinline__ float ew_exp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double ew_exp<double>(double x) { return exp(x); }

// The loaded leaves of one lane: kEwMaxLeaf packs of V values in one register
// vector. Selecting leaf `a` (uniform) is a dynamic extract from registers,
// not an index into private memory.
template <typename T, int V>
struct LeafRegs {
  typedef T type __attribute__((ext_vector_type(kEwMaxLeaf * V)));
};

template <typename T, int V>
__device__ __forceinline__ Pack<T, V> ew_pick(int a, const typename LeafRegs<T, V>::type& L) {
  Pack<T, V> x;
#pragma unroll
  for (int e = 0; e < V; ++e) x.v[e] = L[a * V + e];
  return x;
}

// Evaluates the program on V elements whose leaves are already loaded in L.
// `extra` is the producer's value (GEMV epilogue), ident the identity-matrix
// values of the V elements (only read by EW_IDENT).
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> ew_eval(const EwProgram& p,
                                              const typename LeafRegs<T, V>::type& L,
                                              const Pack<T, V>& extra,
                                              const Pack<T, V>& ident) {
  Pack<T, V> s0, s1, s2, s3;
#pragma unroll
  for (int e = 0; e < V; ++e) s0.v[e] = s1.v[e] = s2.v[e] = s3.v[e] = T(0);
  for (int pc = 0; pc < p.n_instr; ++pc) {
    const int op = p.op[pc];
    const int a = p.arg[pc];
    if (op <= EW_IDENT) {
      Pack<T, V> x;
      if (op == EW_LEAF) {
        x = ew_pick<T, V>(a, L);
      } else if (op == EW_EXTRA) {
        x = extra;
      } else if (op == EW_CONST) {
        const T c = T(p.cst[a]);
#pragma unroll
        for (int e = 0; e < V; ++e) x.v[e] = c;
      } else {
        x = ident;
      }
      s3 = s2;
      s2 = s1;
      s1 = s0;
      s0 = x;
    } else if (op <= EW_RDIV) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T lhs = s1.v[e], rhs = s0.v[e];
        T r;
        switch (op) {
          case EW_ADD: r = lhs + rhs; break;
          case EW_SUB: r = lhs - rhs; break;
          case EW_MUL: r = lhs * rhs; break;
          case EW_DIV: r = lhs / rhs; break;
          case EW_RSUB: r = rhs - lhs; break;
          default: r = rhs / lhs; break;
        }
        s0.v[e] = r;
      }
      s1 = s2;
      s2 = s3;
    } else {
      switch (op) {
        case EW_NEG:
#pragma unroll
          for (int e = 0; e < V; ++e) s0.v[e] = -s0.v[e];
          break;
        case EW_EXP:
#pragma unroll
          for (int e = 0; e < V; ++e) s0.v[e] = ew_exp<T>(s0.v[e]);
          break;
        case EW_SCALE: {
          const T c = T(p.cst[a]);
#pragma unroll
          for (int e = 0; e < V; ++e) s0.v[e] = s0.v[e] * c;
        } break;
        case EW_ADDC: {
          const T c = T(p.cst[a]);
#pragma unroll
          for (int e = 0; e < V; ++e) s0.v[e] = s0.v[e] + c;
        } break;
        case EW_LEAFMUL: {
          const Pack<T, V> x = ew_pick<T, V>(a, L);
#pragma unroll
          for (int e = 0; e < V; ++e) s0.v[e] = s0.v[e] * x.v[e];
        } break;
        default: {  // EW_LEAFADD
          const Pack<T, V> x = ew_pick<T, V>(a, L);
#pragma unroll
          for (int e = 0; e < V; ++e) s0.v[e] = s0.v[e] + x.v[e];
        } break;
      }
    }
  }
  return s0;
}

// Scalar evaluation at flat index idx of a rows x cols view through the
// leaves' strides (any layout, transposed views included).
template <typename T>
__device__ __forceinline__ T ew_eval_at(const EwProgram& p, int64_t idx, T extra) {
  const int64_t i = idx % p.rows;
  const int64_t j = idx / p.rows;
  typename LeafRegs<T, 1>::type L;
#pragma unroll
  for (int l = 0; l < kEwMaxLeaf; ++l) {
    L[l] = T(0);
    if (l < p.n_leaf) {
      const T* ptr = static_cast<const T*>(p.leaf[l].ptr);
      L[l] = ptr[i * p.leaf[l].si + j * p.leaf[l].sj];
    }
  }
  Pack<T, 1> x, id;
  x.v[0] = extra;
  id.v[0] = (i == j) ? T(1) : T(0);
  return ew_eval<T, 1>(p, L, x, id).v[0];
}

// V elements of column j at rows i0, i0 + S, ..., i0 + (V - 1) S of a
// rows x cols view through the leaves' strides: the row and column come
// from the caller's tiling (no division per element), every leaf load is
// issued before the program runs (rows past the view clamped to the last
// row; their values are not used).
template <typename T, int V, int S>
__device__ __forceinline__ Pack<T, V> ew_eval_col(const EwProgram& p, int64_t i0, int64_t j) {
  typename LeafRegs<T, V>::type L;
  Pack<T, V> zero, id;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int64_t i = i0 + int64_t(e) * S;
    zero.v[e] = T(0);
    id.v[e] = (i == j) ? T(1) : T(0);
  }
#pragma unroll
  for (int l = 0; l < kEwMaxLeaf; ++l) {
#pragma unroll
    for (int e = 0; e < V; ++e) L[l * V + e] = T(0);
    if (l < p.n_leaf) {
      const T* ptr = static_cast<const T*>(p.leaf[l].ptr) + j * p.leaf[l].sj;
      const int64_t si = p.leaf[l].si;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int64_t i = std::min<int64_t>(i0 + int64_t(e) * S, p.rows - 1);
        L[l * V + e] = ptr[i * si];
      }
    }
  }
  return ew_eval<T, V>(p, L, zero, id);
}

}  // namespace k
}  // namespace hexla
