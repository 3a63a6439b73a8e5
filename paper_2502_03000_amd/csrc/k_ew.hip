// Fused element-wise kernel: one pass over the elements evaluates the whole
// element-wise expression, reading each operand once and writing the result
// once (the single loop with no temporaries of Sec. II; expression (1) of
// Sec. III). HBM-bound: per element it moves (leaves + 1) * sizeof(T) bytes.
#include <hip/hip_runtime.h>

#include "ew_device.h"

namespace hexla {
namespace k {

namespace {

constexpr int kThreads = 256;

template <typename T, int V>
struct Native;
template <>
struct Native<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Native<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename T, int V>
__device__ __forceinline__ typename Native<T, V>::type load_native(const void* base, int64_t q) {
  using N = typename Native<T, V>::type;
  return __builtin_nontemporal_load(reinterpret_cast<const N*>(base) + q);
}

template <typename T, int V>
__device__ __forceinline__ void store_pack(void* base, int64_t q, const Pack<T, V>& r) {
  using N = typename Native<T, V>::type;
  N x;
#pragma unroll
  for (int e = 0; e < V; ++e) x[e] = r.v[e];
  __builtin_nontemporal_store(x, reinterpret_cast<N*>(base) + q);
}

// Contiguous path: every leaf and the output are dense in flat column-major
// order and 16-byte aligned. Each lane handles U packs of V elements per
// iteration so that U * n_leaf 16-byte loads are in flight before any use.
template <typename T, int V, int U>
__global__ __launch_bounds__(kThreads) void ew_contig_kernel(EwProgram p, T* __restrict__ out,
                                                             int64_t n_pack, int64_t n_total) {
  using P = Pack<T, V>;
  const int64_t stride = int64_t(gridDim.x) * kThreads * U;
  P zero;
#pragma unroll
  for (int e = 0; e < V; ++e) zero.v[e] = T(0);
  for (int64_t base = int64_t(blockIdx.x) * kThreads * U + threadIdx.x; base < n_pack;
       base += stride) {
    typename LeafRegs<T, V>::type L[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = base + int64_t(u) * kThreads;
#pragma unroll
      for (int l = 0; l < kEwMaxLeaf; ++l) {
        typename Native<T, V>::type x = {};
        if (l < p.n_leaf && q < n_pack) x = load_native<T, V>(p.leaf[l].ptr, q);
#pragma unroll
        for (int e = 0; e < V; ++e) L[u][l * V + e] = x[e];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = base + int64_t(u) * kThreads;
      if (q < n_pack) {
        const P r = ew_eval<T, V>(p, L[u], zero, zero);
        store_pack<T, V>(out, q, r);
      }
    }
  }
  // ragged tail (n_total not a multiple of V): first lanes of block 0
  if (blockIdx.x == 0) {
    const int64_t t = n_pack * V + threadIdx.x;
    if (t < n_total) out[t] = ew_eval_at<T>(p, t, T(0));
  }
}

// General path: any strides (transposed views, leading dimensions, identity).
template <typename T>
__global__ __launch_bounds__(kThreads) void ew_general_kernel(EwProgram p, T* __restrict__ out,
                                                              int64_t osi, int64_t osj,
                                                              int64_t n_total) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x; t < n_total; t += stride) {
    const int64_t i = t % p.rows;
    const int64_t j = t / p.rows;
    out[i * osi + j * osj] = ew_eval_at<T>(p, t, T(0));
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <typename T>
hipError_t launch_typed(const EwProgram& p, void* out, int64_t osi, int64_t osj, hipStream_t s) {
  const int64_t n_total = p.rows * p.cols;
  if (n_total == 0) return hipSuccess;
  bool contig = p.contiguous && !p.uses_ident && aligned16(out) && osi == 1 &&
                (p.cols == 1 || osj == p.rows);
  for (int l = 0; l < p.n_leaf && contig; ++l) contig = aligned16(p.leaf[l].ptr);
  constexpr int V = 16 / sizeof(T);
  if (contig && n_total >= V) {
    constexpr int U = 2;
    const int64_t n_pack = n_total / V;
    int64_t blocks = (n_pack + int64_t(kThreads) * U - 1) / (int64_t(kThreads) * U);
    const int64_t cap = 256 * 16;  // 16 workgroups per CU on a 256-CU part
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((ew_contig_kernel<T, V, U>), dim3(unsigned(blocks)), dim3(kThreads), 0, s,
                       p, static_cast<T*>(out), n_pack, n_total);
  } else {
    int64_t blocks = (n_total + kThreads - 1) / kThreads;
    if (blocks > 256 * 32) blocks = 256 * 32;
    hipLaunchKernelGGL((ew_general_kernel<T>), dim3(unsigned(blocks)), dim3(kThreads), 0, s, p,
                       static_cast<T*>(out), osi, osj, n_total);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t ew_launch(int dtype, const EwProgram& p, void* out, int64_t osi, int64_t osj,
                     hipStream_t s) {
  return dtype == 0 ? launch_typed<double>(p, out, osi, osj, s)
                    : launch_typed<float>(p, out, osi, osj, s);
}

namespace {
__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t value) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = value;
}
}  // namespace

hipError_t fill_i32_launch(int32_t* p, int64_t count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
