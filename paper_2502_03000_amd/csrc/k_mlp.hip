// The learned cost model's kernels: a fully connected ReLU network
// F -> 64 -> 64 -> 64 -> 1 in FP32 (inference, MSE gradient, Adam).
//
// One workgroup handles a block of 64 samples with the weights, inputs and
// pre-activations in LDS: the forward pass keeps z_l, the backward pass
// forms delta_l and the weight gradients of its block, which go to a
// per-block slot (fixed-order reduction afterwards: deterministic).
//   z_l = W_l h_{l-1} + b_l, h_l = max(z_l, 0), y = z_4
//   delta_4 = 2 (y - t) / N,  dW_l = sum_s delta_l h_{l-1}^T,
//   delta_{l-1} = (W_l^T delta_l) * [z_{l-1} > 0]
// Parameter layout (flat, FP32): W1 (64 x F, row-major), b1, W2 (64 x 64),
// b2, W3, b3, W4 (1 x 64), b4.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace hexla {
namespace k {

namespace {

constexpr int F = kMlpFeatures;
constexpr int H = kMlpHidden;
constexpr int NB = 64;   // samples per workgroup
constexpr int NT = 256;  // threads per workgroup
constexpr int NW = NT / 64;
constexpr int S1 = F + 1, S2 = H + 1;  // padded LDS row strides of W1, W2/W3

// offsets into the flat parameter vector
constexpr int oW1 = 0, ob1 = oW1 + H * F, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H,
              ob3 = oW3 + H * H, oW4 = ob3 + H, ob4 = oW4 + H, kP = ob4 + 1;
static_assert(kP == kMlpParams, "parameter count");

struct MlpSmem {
  float w1[H * S1], w2[H * S2], w3[H * S2], w4[H], b1[H], b2[H], b3[H], b4;
  float x[NB][F];
  float z1[NB][H], z2[NB][H], z3[NB][H];
  float d0[NB][H], d1[NB][H];
  float y[NB], dy[NB];
};

__device__ void load_params(MlpSmem& s, const float* __restrict__ p) {
  for (int e = threadIdx.x; e < H * F; e += NT) s.w1[(e / F) * S1 + e % F] = p[oW1 + e];
  for (int e = threadIdx.x; e < H * H; e += NT) {
    s.w2[(e / H) * S2 + e % H] = p[oW2 + e];
    s.w3[(e / H) * S2 + e % H] = p[oW3 + e];
  }
  for (int e = threadIdx.x; e < H; e += NT) {
    s.w4[e] = p[oW4 + e];
    s.b1[e] = p[ob1 + e];
    s.b2[e] = p[ob2 + e];
    s.b3[e] = p[ob3 + e];
  }
  if (threadIdx.x == 0) s.b4 = p[ob4];
}

// z[s][o] = b[o] + sum_i W[o][i] act(in[s][i]); lane = o, wave w takes
// samples w, w + NW, ... (the input row is a broadcast, W a padded row).
template <int IN, int STRIDE, bool RELU_IN>
__device__ void dense(const float* w, const float* b, const float (*in)[IN], float (*z)[H]) {
  const int o = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float acc[NB / NW];
#pragma unroll
  for (int j = 0; j < NB / NW; ++j) acc[j] = b[o];
  for (int i = 0; i < IN; ++i) {
    const float wi = w[o * STRIDE + i];
#pragma unroll
    for (int j = 0; j < NB / NW; ++j) {
      float h = in[wv + NW * j][i];
      if (RELU_IN) h = fmaxf(h, 0.f);
      acc[j] += wi * h;
    }
  }
#pragma unroll
  for (int j = 0; j < NB / NW; ++j) z[wv + NW * j][o] = acc[j];
}

// forward pass of the block's samples (rows beyond `valid` are zero inputs)
__device__ void forward(MlpSmem& s, const float* __restrict__ x, const int32_t* __restrict__ idx,
                        int64_t base, int valid) {
  for (int e = threadIdx.x; e < NB * F; e += NT) {
    const int r = e / F, c = e % F;
    float v = 0.f;
    if (r < valid) {
      const int64_t row = idx ? idx[base + r] : base + r;
      v = x[row * F + c];
    }
    s.x[r][c] = v;
  }
  __syncthreads();
  dense<F, S1, false>(s.w1, s.b1, s.x, s.z1);
  __syncthreads();
  dense<H, S2, true>(s.w2, s.b2, s.z1, s.z2);
  __syncthreads();
  dense<H, S2, true>(s.w3, s.b3, s.z2, s.z3);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r = wv; r < NB; r += NW) {
    float v = s.w4[lane] * fmaxf(s.z3[r][lane], 0.f);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) s.y[r] = v + s.b4;
  }
  __syncthreads();
}

// dW[o][i] = sum_s d[s][o] act(h[s][i]) written to g (row-major, IN columns),
// db[o] = sum_s d[s][o]; lane = o, wave w takes i = w, w + NW, ...
template <int IN, bool RELU_IN>
__device__ void weight_grad(const float (*d)[H], const float (*h)[IN], float* gw, float* gb) {
  const int o = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = wv; i < IN; i += NW) {
    float acc = 0.f;
    for (int r = 0; r < NB; ++r) {
      float hv = h[r][i];
      if (RELU_IN) hv = fmaxf(hv, 0.f);
      acc += d[r][o] * hv;
    }
    gw[o * IN + i] = acc;
  }
  if (wv == 0) {
    float acc = 0.f;
    for (int r = 0; r < NB; ++r) acc += d[r][o];
    gb[o] = acc;
  }
}

// dprev[s][i] = sum_o d[s][o] W[o][i] * [z[s][i] > 0]; lane = i, wave w
// takes samples w, w + NW, ...
__device__ void back_delta(const float* w, const float (*d)[H], const float (*z)[H],
                           float (*dprev)[H]) {
  const int i = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r = wv; r < NB; r += NW) {
    float acc = 0.f;
    for (int o = 0; o < H; ++o) acc += d[r][o] * w[o * S2 + i];
    dprev[r][i] = z[r][i] > 0.f ? acc : 0.f;
  }
}

__global__ __launch_bounds__(NT) void mlp_grad_kernel(const float* __restrict__ params,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ t,
                                                       const int32_t* __restrict__ idx,
                                                       int64_t count, float inv_n,
                                                       float* __restrict__ partial,
                                                       float* __restrict__ loss_partial) {
  __shared__ MlpSmem s;
  const int64_t base = int64_t(blockIdx.x) * NB;
  const int valid = int(min(int64_t(NB), count - base));
  load_params(s, params);
  forward(s, x, idx, base, valid);
  const int tid = threadIdx.x;
  if (tid < NB) {
    float d = 0.f;
    if (tid < valid) {
      const int64_t row = idx ? idx[base + tid] : base + tid;
      d = s.y[tid] - t[row];
    }
    s.dy[tid] = 2.f * d * inv_n;
    float sq = d * d;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (tid == 0) loss_partial[blockIdx.x] = sq;
  }
  __syncthreads();
  float* g = partial + int64_t(blockIdx.x) * kP;
  // output layer: dW4[i] = sum_s dy[s] h3[s][i], db4 = sum_s dy[s]
  if (tid < H) {
    float acc = 0.f;
    for (int r = 0; r < NB; ++r) acc += s.dy[r] * fmaxf(s.z3[r][tid], 0.f);
    g[oW4 + tid] = acc;
  }
  if (tid == H) {
    float acc = 0.f;
    for (int r = 0; r < NB; ++r) acc += s.dy[r];
    g[ob4] = acc;
  }
  // delta3[s][i] = dy[s] W4[i] [z3 > 0]
  for (int e = tid; e < NB * H; e += NT) {
    const int r = e / H, i = e % H;
    s.d0[r][i] = s.z3[r][i] > 0.f ? s.dy[r] * s.w4[i] : 0.f;
  }
  __syncthreads();
  weight_grad<H, true>(s.d0, s.z2, g + oW3, g + ob3);
  back_delta(s.w3, s.d0, s.z2, s.d1);
  __syncthreads();
  weight_grad<H, true>(s.d1, s.z1, g + oW2, g + ob2);
  back_delta(s.w2, s.d1, s.z1, s.d0);
  __syncthreads();
  weight_grad<F, false>(s.d0, s.x, g + oW1, g + ob1);
}

__global__ __launch_bounds__(NT) void mlp_predict_kernel(const float* __restrict__ params,
                                                          const float* __restrict__ x,
                                                          int64_t count, float scale, float shift,
                                                          float* __restrict__ y) {
  __shared__ MlpSmem s;
  const int64_t base = int64_t(blockIdx.x) * NB;
  const int valid = int(min(int64_t(NB), count - base));
  load_params(s, params);
  forward(s, x, nullptr, base, valid);
  if (threadIdx.x < valid) y[base + threadIdx.x] = shift + scale * s.y[threadIdx.x];
}

// g[p] = sum over blocks (fixed order); optionally one Adam step on params.
__global__ void mlp_reduce_kernel(const float* __restrict__ partial, int nblocks,
                                  float* __restrict__ grad, float* __restrict__ params,
                                  float* __restrict__ m, float* __restrict__ v, float lr,
                                  float beta1, float beta2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kP) return;
  float g = 0.f;
  for (int b = 0; b < nblocks; ++b) g += partial[int64_t(b) * kP + p];
  if (grad) grad[p] = g;
  if (params) {
    const float mp = beta1 * m[p] + (1.f - beta1) * g;
    const float vp = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mp;
    v[p] = vp;
    const float mhat = mp / bc1, vhat = vp / bc2;
    params[p] -= lr * mhat / (sqrtf(vhat) + eps);
  }
}

}  // namespace

int64_t mlp_blocks(int64_t count) { return (count + NB - 1) / NB; }

hipError_t mlp_grad_launch(const float* params, const float* x, const float* t,
                           const int32_t* idx, int64_t count, float* partial,
                           float* loss_partial, hipStream_t s) {
  const int64_t nb = mlp_blocks(count);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(unsigned(nb)), dim3(NT), 0, s, params, x, t, idx, count,
                     1.0f / float(count), partial, loss_partial);
  return hipGetLastError();
}

hipError_t mlp_reduce_launch(const float* partial, int64_t nblocks, float* grad, float* params,
                             float* m, float* v, float lr, float beta1, float beta2, float eps,
                             int64_t step, hipStream_t s) {
  const float bc1 = 1.f - powf(beta1, float(step)), bc2 = 1.f - powf(beta2, float(step));
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kP + 255) / 256), dim3(256), 0, s, partial,
                     int(nblocks), grad, params, m, v, lr, beta1, beta2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t mlp_predict_launch(const float* params, const float* x, int64_t count, float scale,
                              float shift, float* y, hipStream_t s) {
  const int64_t nb = mlp_blocks(count);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_predict_kernel, dim3(unsigned(nb)), dim3(NT), 0, s, params, x, count,
                     scale, shift, y);
  return hipGetLastError();
}

}  // namespace k
}  // namespace hexla
