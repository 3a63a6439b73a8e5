// Fused element-wise kernel: one pass over the elements evaluates the whole
// element-wise expression, reading each operand once and writing the result
// once (the single loop with no temporaries of Sec. II; expression (1) of
// Sec. III). HBM-bound: per element it moves (leaves + 1) * sizeof(T) bytes.
#include <hip/hip_runtime.h>

#include <algorithm>

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
// order and 16-byte aligned. One-shot grid: each lane loads one 16-byte pack
// of every operand, evaluates it and stores it (no grid-stride loop, which
// measured slower on this part); the last lanes take the ragged tail.
template <typename T, int V>
__global__ __launch_bounds__(kThreads) void ew_contig_kernel(EwProgram p, T* __restrict__ out,
                                                             int64_t n_pack, int64_t n_total) {
  using P = Pack<T, V>;
  const int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (q < n_pack) {
    typename LeafRegs<T, V>::type L;
#pragma unroll
    for (int l = 0; l < kEwMaxLeaf; ++l) {
      typename Native<T, V>::type x = {};
      if (l < p.n_leaf) x = load_native<T, V>(p.leaf[l].ptr, q);
#pragma unroll
      for (int e = 0; e < V; ++e) L[l * V + e] = x[e];
    }
    P zero;
#pragma unroll
    for (int e = 0; e < V; ++e) zero.v[e] = T(0);
    store_pack<T, V>(out, q, ew_eval<T, V>(p, L, zero, zero));
  } else {
    const int64_t t = n_pack * V + (q - n_pack);
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

// General path for views of at least kColRows rows: tiles of kThreads x
// kColV rows of one column, the tile's row and column found once per tile,
// kColV elements per lane (as many as a 16-byte pack: the interpreter's
// register vector of leaves stays in registers) with all their loads in
// flight together.
template <typename T>
constexpr int kColV = 16 / int(sizeof(T));
constexpr int64_t kColRows = 64;
template <typename T>
__global__ __launch_bounds__(kThreads) void ew_columns_kernel(EwProgram p, T* __restrict__ out,
                                                              int64_t osi, int64_t osj,
                                                              int64_t tiles_per_col,
                                                              int64_t tiles) {
  for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
    const int64_t j = b / tiles_per_col;
    const int64_t i0 = (b - j * tiles_per_col) * (kThreads * kColV<T>) + threadIdx.x;
    const Pack<T, kColV<T>> r = ew_eval_col<T, kColV<T>, kThreads>(p, i0, j);
#pragma unroll
    for (int e = 0; e < kColV<T>; ++e) {
      const int64_t i = i0 + int64_t(e) * kThreads;
      if (i < p.rows) out[i * osi + j * osj] = r.v[e];
    }
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
  if (contig) {
    const int64_t n_pack = n_total / V;
    const int64_t threads = n_pack + (n_total - n_pack * V);
    const int64_t blocks = (threads + kThreads - 1) / kThreads;
    hipLaunchKernelGGL((ew_contig_kernel<T, V>), dim3(unsigned(blocks)), dim3(kThreads), 0, s, p,
                       static_cast<T*>(out), n_pack, n_total);
  } else if (p.rows >= kColRows) {
    const int64_t per_col = (p.rows + kThreads * kColV<T> - 1) / (kThreads * kColV<T>);
    const int64_t tiles = per_col * p.cols;
    const int64_t blocks = std::min<int64_t>(tiles, 256 * 32);
    hipLaunchKernelGGL((ew_columns_kernel<T>), dim3(unsigned(blocks)), dim3(kThreads), 0, s, p,
                       static_cast<T*>(out), osi, osj, per_col, tiles);
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
