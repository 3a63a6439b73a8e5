// The learned cost model: a small FP32 network that predicts the log of a
// matrix product's run time from its shape and launch configuration,
// trained on timings the evaluator measures itself (the autotuner's timing
// log). Training, gradients and inference run in the kernels of k_mlp.hip;
// this file holds the features, the host side of training and the planner's
// batched inference call.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <numeric>
#include <random>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace k = hexla::k;
using hexla::set_err;

struct hexla_model {
  hexla_ctx* ctx = nullptr;
  float* params = nullptr;  // device: kMlpParams
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  int64_t step = 0;
  float y_mean = 0.f, y_std = 1.f;  // target standardisation (log microseconds)
  // inference buffers, kPredictCap samples, allocated with the model: on
  // the device, and pinned host staging for the copies
  float* x_buf = nullptr;
  float* y_buf = nullptr;
  float* x_host = nullptr;
  float* y_host = nullptr;
  ~hexla_model() {
    for (float* p : {params, m, v, x_buf, y_buf})
      if (p) (void)hipFree(p);
    for (float* p : {x_host, y_host})
      if (p) (void)hipHostFree(p);
  }
};

namespace hexla {

namespace {

// Candidates predicted per inference launch (a chain of eight factors with
// every tile and split-K candidate needs a few thousand).
constexpr int64_t kPredictCap = 16384;

constexpr int F = k::kMlpFeatures;
constexpr int P = k::kMlpParams;

float lg(double x) { return float(std::log2(std::max(x, 1.0))); }

hexla_status dev_err(const hexla_ctx* ctx, hipError_t e, const char* what) {
  return set_err(ctx, HEXLA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Scratch of one gradient evaluation over `count` samples.
struct GradBufs {
  float* partial = nullptr;
  float* loss = nullptr;
  float* grad = nullptr;
  ~GradBufs() {
    for (float* p : {partial, loss, grad})
      if (p) (void)hipFree(p);
  }
  hipError_t alloc(int64_t count) {
    const int64_t nb = std::max<int64_t>(1, k::mlp_blocks(count));
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&partial), size_t(nb) * P * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&loss), size_t(nb) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&grad), size_t(P) * sizeof(float));
    return e;
  }
};

double sum_loss(const float* d_loss, int64_t nb, hipStream_t s, hipError_t* e) {
  std::vector<float> h(size_t(std::max<int64_t>(nb, 1)));
  *e = hipMemcpyAsync(h.data(), d_loss, size_t(nb) * sizeof(float), hipMemcpyDeviceToHost, s);
  if (*e == hipSuccess) *e = hipStreamSynchronize(s);
  double acc = 0.0;
  for (int64_t b = 0; b < nb; ++b) acc += h[size_t(b)];
  return acc;
}

}  // namespace

void product_features(int dtype, int precision, int mode, int ta, int tb, int64_t m, int64_t n,
                      int64_t kk, int tile, int split, float* f) {
  std::fill(f, f + F, 0.f);
  int bm = 64, bn = 64, bk = 16;
  if (tile >= 0) k::gemm_tile_shape(dtype, precision, tile, &bm, &bn, &bk);
  split = std::max(split, 1);
  const double es = dtype == HEXLA_F64 ? 8.0 : 4.0;
  const double M = double(m), N = double(n), K = double(kk);
  const double tm = std::ceil(M / bm), tn = std::ceil(N / bn);
  const double tiles = mode == 1 ? tn * (tn + 1) / 2 : tm * tn;
  const double wgs = tiles * split;
  const double kchunk = std::ceil(K / split);
  const double bytes = es * (M * K + K * N + M * N);
  const double flops = mode == 1 ? N * (N + 1) * K : 2.0 * M * N * K;
  f[0] = lg(M) / 13.f;
  f[1] = lg(N) / 13.f;
  f[2] = lg(K) / 13.f;
  f[3] = lg(M * N * K) / 39.f;
  f[4] = lg(kchunk) / 13.f;
  f[5] = lg(split) / 10.f;
  f[6] = dtype == HEXLA_F64 ? 1.f : 0.f;
  f[7] = dtype == HEXLA_F32 ? 1.f : 0.f;
  f[8] = mode == 1 ? 1.f : 0.f;
  f[9] = ta ? 1.f : 0.f;
  f[10] = tb ? 1.f : 0.f;
  f[11] = float(precision) / 3.f;
  if (tile >= 0 && tile < 8) f[12 + tile] = 1.f;
  f[20] = lg(bm) / 8.f;
  f[21] = lg(bn) / 8.f;
  f[22] = lg(bk) / 6.f;
  f[23] = lg(wgs) / 20.f;
  f[24] = float(std::min(wgs / 256.0, 4.0) / 4.0);
  f[25] = float((M * N) / (tm * bm * tn * bn));
  f[26] = float(K / (std::ceil(kchunk / bk) * bk * split));
  f[27] = lg(bytes) / 40.f;
  f[28] = lg(flops / bytes) / 12.f;
  f[29] = split > 1 ? 1.f : 0.f;
  f[30] = split > 1 ? lg(double(split) * M * N * es) / 36.f : 0.f;
  f[31] = lg(M * N) / 26.f;
}

// The features of one product for several configurations at once: the
// same values as product_features, with the parts that do not depend on the
// configuration computed once.
void product_features_many(int dtype, int precision, int mode, int ta, int tb, int64_t m,
                           int64_t n, int64_t kk, const k::GemmConfig* cfg, int count, float* out) {
  if (count <= 0) return;
  const double es = dtype == HEXLA_F64 ? 8.0 : 4.0;
  const double M = double(m), N = double(n), K = double(kk);
  const double bytes = es * (M * K + K * N + M * N);
  const double flops = mode == 1 ? N * (N + 1) * K : 2.0 * M * N * K;
  float base[F];
  std::fill(base, base + F, 0.f);
  base[0] = lg(M) / 13.f;
  base[1] = lg(N) / 13.f;
  base[2] = lg(K) / 13.f;
  base[3] = lg(M * N * K) / 39.f;
  base[6] = dtype == HEXLA_F64 ? 1.f : 0.f;
  base[7] = dtype == HEXLA_F32 ? 1.f : 0.f;
  base[8] = mode == 1 ? 1.f : 0.f;
  base[9] = ta ? 1.f : 0.f;
  base[10] = tb ? 1.f : 0.f;
  base[11] = float(precision) / 3.f;
  base[27] = lg(bytes) / 40.f;
  base[28] = lg(flops / bytes) / 12.f;
  base[31] = lg(M * N) / 26.f;
  int last_tile = -2, bm = 64, bn = 64, bk = 16;
  float fbm = 0.f, fbn = 0.f, fbk = 0.f;
  double tm = 0.0, tn = 0.0, tiles = 0.0;
  for (int c = 0; c < count; ++c) {
    float* f = out + size_t(c) * F;
    std::copy(base, base + F, f);
    const int tile = cfg[c].tile;
    if (tile != last_tile) {
      bm = 64, bn = 64, bk = 16;
      if (tile >= 0) k::gemm_tile_shape(dtype, precision, tile, &bm, &bn, &bk);
      fbm = lg(bm) / 8.f;
      fbn = lg(bn) / 8.f;
      fbk = lg(bk) / 6.f;
      tm = std::ceil(M / bm);
      tn = std::ceil(N / bn);
      tiles = mode == 1 ? tn * (tn + 1) / 2 : tm * tn;
      last_tile = tile;
    }
    const int split = std::max(cfg[c].split, 1);
    const double wgs = tiles * split;
    const double kchunk = std::ceil(K / split);
    f[4] = lg(kchunk) / 13.f;
    f[5] = lg(split) / 10.f;
    if (tile >= 0 && tile < 8) f[12 + tile] = 1.f;
    f[20] = fbm;
    f[21] = fbn;
    f[22] = fbk;
    f[23] = lg(wgs) / 20.f;
    f[24] = float(std::min(wgs / 256.0, 4.0) / 4.0);
    f[25] = float((M * N) / (tm * bm * tn * bn));
    f[26] = float(K / (std::ceil(kchunk / bk) * bk * split));
    f[29] = split > 1 ? 1.f : 0.f;
    f[30] = split > 1 ? lg(double(split) * M * N * es) / 36.f : 0.f;
  }
}

bool model_predict_us(hexla_model* md, const std::vector<float>& x, std::vector<float>& us,
                      std::string* err) {
  const int64_t count = int64_t(x.size()) / F;
  us.assign(size_t(count), 0.f);
  if (count == 0) return true;
  hipStream_t s = md->ctx->stream;
  hipError_t e = enter_device(md->ctx->device);
  // The inference buffers were sized when the model was created: planning
  // allocates no device memory; a long candidate list runs in chunks.
  for (int64_t at = 0; at < count && e == hipSuccess; at += kPredictCap) {
    const int64_t c = std::min<int64_t>(kPredictCap, count - at);
    std::memcpy(md->x_host, x.data() + size_t(at) * F, size_t(c) * F * sizeof(float));
    e = hipMemcpyAsync(md->x_buf, md->x_host, size_t(c) * F * sizeof(float),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = k::mlp_predict_launch(md->params, md->x_buf, c, md->y_std, md->y_mean, md->y_buf, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(md->y_host, md->y_buf, size_t(c) * sizeof(float),
                         hipMemcpyDeviceToHost, s);
    // the next chunk overwrites the staging buffers: wait for this one
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) std::memcpy(us.data() + at, md->y_host, size_t(c) * sizeof(float));
  }
  if (e != hipSuccess) {
    if (err) *err = std::string("model inference: ") + hipGetErrorString(e);
    return false;
  }
  for (float& y : us) y = std::exp(y);  // the network predicts log(microseconds)
  return true;
}

void detach_model(hexla_model* md) { md->ctx = nullptr; }

}  // namespace hexla

using namespace hexla;

extern "C" {

hexla_status hexla_product_features(int32_t dtype, int32_t precision, int32_t mode, int32_t ta,
                                    int32_t tb, int64_t m, int64_t n, int64_t kk, int32_t tile,
                                    int32_t split, float* out) {
  if (!out || m < 1 || n < 1 || kk < 1 || (dtype != HEXLA_F64 && dtype != HEXLA_F32) ||
      tile < 0 || tile >= k::gemm_tile_count(dtype) || split < 1)
    return HEXLA_E_INVALID_ARG;
  product_features(dtype, precision, mode, ta, tb, m, n, kk, tile, split, out);
  return HEXLA_OK;
}

hexla_status hexla_model_create(hexla_ctx* ctx, uint64_t seed, hexla_model** out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  *out = nullptr;
  if (ctx->device < 0) return set_err(ctx, HEXLA_E_UNSUPPORTED, "model: dry-run context");
  auto md = std::make_unique<hexla_model>();
  md->ctx = ctx;
  // He-normal weights, zero biases
  std::vector<float> h(P, 0.f);
  std::mt19937_64 g(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  const int widths[5] = {F, k::kMlpHidden, k::kMlpHidden, k::kMlpHidden, 1};
  size_t off = 0;
  for (int l = 0; l < 4; ++l) {
    const int in = widths[l], outw = widths[l + 1];
    const double sd = std::sqrt(2.0 / in);
    for (int e = 0; e < in * outw; ++e) h[off + e] = float(nd(g) * sd);
    off += size_t(in) * outw + outw;
  }
  hipError_t e = enter_device(ctx->device);
  for (float** p : {&md->params, &md->m, &md->v})
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(p), P * sizeof(float));
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&md->x_buf), size_t(kPredictCap) * F * sizeof(float));
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&md->y_buf), size_t(kPredictCap) * sizeof(float));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&md->x_host), size_t(kPredictCap) * F * sizeof(float),
                      hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&md->y_host), size_t(kPredictCap) * sizeof(float),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpy(md->params, h.data(), P * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(md->m, 0, P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(md->v, 0, P * sizeof(float));
  if (e != hipSuccess) return dev_err(ctx, e, "model_create");
  ctx->models.insert(md.get());
  *out = md.release();
  return HEXLA_OK;
}

hexla_status hexla_model_destroy(hexla_model* md) {
  if (!md) return HEXLA_E_INVALID_ARG;
  if (md->ctx) {
    if (md->ctx->model == md) md->ctx->model = nullptr;
    md->ctx->models.erase(md);
    (void)hipSetDevice(md->ctx->device);
  }
  delete md;
  return HEXLA_OK;
}

hexla_status hexla_model_param_count(int64_t* n) {
  if (!n) return HEXLA_E_INVALID_ARG;
  *n = P;
  return HEXLA_OK;
}

hexla_status hexla_model_get_params(hexla_model* md, float* host, int64_t n, float* y_mean,
                                    float* y_std) {
  if (!md || !md->ctx || !host || n != P) return HEXLA_E_INVALID_ARG;
  hipError_t e = enter_device(md->ctx->device);
  if (e == hipSuccess) e = hipStreamSynchronize(md->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(host, md->params, P * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_get_params");
  if (y_mean) *y_mean = md->y_mean;
  if (y_std) *y_std = md->y_std;
  return HEXLA_OK;
}

hexla_status hexla_model_set_params(hexla_model* md, const float* host, int64_t n, float y_mean,
                                    float y_std) {
  if (!md || !md->ctx || !host || n != P || !(y_std > 0.f)) return HEXLA_E_INVALID_ARG;
  hipError_t e = enter_device(md->ctx->device);
  if (e == hipSuccess) e = hipStreamSynchronize(md->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(md->params, host, P * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(md->m, 0, P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(md->v, 0, P * sizeof(float));
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_set_params");
  md->step = 0;
  md->y_mean = y_mean;
  md->y_std = y_std;
  return HEXLA_OK;
}

hexla_status hexla_model_grad(hexla_model* md, const float* x, const float* t, int64_t count,
                              float* grad_host, double* loss) {
  if (!md || !md->ctx || !x || !t || count < 1 || !grad_host) return HEXLA_E_INVALID_ARG;
  hipStream_t s = md->ctx->stream;
  GradBufs b;
  hipError_t e = enter_device(md->ctx->device);
  if (e == hipSuccess) e = b.alloc(count);
  if (e == hipSuccess) e = k::mlp_grad_launch(md->params, x, t, nullptr, count, b.partial, b.loss, s);
  if (e == hipSuccess)
    e = k::mlp_reduce_launch(b.partial, k::mlp_blocks(count), b.grad, nullptr, nullptr, nullptr,
                             0.f, 0.f, 0.f, 0.f, 1, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad_host, b.grad, P * sizeof(float), hipMemcpyDeviceToHost, s);
  double l = 0.0;
  if (e == hipSuccess) l = sum_loss(b.loss, k::mlp_blocks(count), s, &e);
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_grad");
  if (loss) *loss = l / double(count);
  return HEXLA_OK;
}

hexla_status hexla_model_step(hexla_model* md, const float* x, const float* t, int64_t count,
                              float lr, double* loss) {
  if (!md || !md->ctx || !x || !t || count < 1 || !(lr > 0.f)) return HEXLA_E_INVALID_ARG;
  hipStream_t s = md->ctx->stream;
  GradBufs b;
  hipError_t e = enter_device(md->ctx->device);
  if (e == hipSuccess) e = b.alloc(count);
  if (e == hipSuccess) e = k::mlp_grad_launch(md->params, x, t, nullptr, count, b.partial, b.loss, s);
  if (e == hipSuccess)
    e = k::mlp_reduce_launch(b.partial, k::mlp_blocks(count), nullptr, md->params, md->m, md->v,
                             lr, 0.9f, 0.999f, 1e-8f, md->step + 1, s);
  double l = 0.0;
  if (e == hipSuccess) l = sum_loss(b.loss, k::mlp_blocks(count), s, &e);
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_step");
  ++md->step;
  if (loss) *loss = l / double(count);
  return HEXLA_OK;
}

hexla_status hexla_model_train(hexla_model* md, const float* x, const float* t, int64_t count,
                               const hexla_train_opts* opts, double* final_loss) {
  if (!md || !md->ctx || !x || !t || count < 1) return HEXLA_E_INVALID_ARG;
  hexla_train_opts o{};
  o.epochs = 200;
  o.batch = 256;
  o.lr = 1e-3f;
  o.seed = 1;
  if (opts) o = *opts;
  if (o.epochs < 1 || o.batch < 1 || !(o.lr > 0.f))
    return set_err(md->ctx, HEXLA_E_INVALID_ARG, "model_train: bad options");
  hipStream_t s = md->ctx->stream;
  hipError_t e = enter_device(md->ctx->device);
  // standardised targets
  std::vector<float> th(static_cast<size_t>(count));
  if (e == hipSuccess) e = hipMemcpy(th.data(), t, size_t(count) * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_train");
  double mean = 0.0, var = 0.0;
  for (float v : th) mean += v;
  mean /= double(count);
  for (float v : th) var += (v - mean) * (v - mean);
  const double sd = std::sqrt(var / double(count)) > 1e-6 ? std::sqrt(var / double(count)) : 1.0;
  for (float& v : th) v = float((v - mean) / sd);
  md->y_mean = float(mean);
  md->y_std = float(sd);
  md->step = 0;
  float* t_std = nullptr;
  int32_t* idx = nullptr;
  GradBufs b;
  e = hipMalloc(reinterpret_cast<void**>(&t_std), size_t(count) * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&idx), size_t(count) * sizeof(int32_t));
  if (e == hipSuccess) e = b.alloc(std::max<int64_t>(o.batch, count));
  if (e == hipSuccess) e = hipMemcpy(t_std, th.data(), size_t(count) * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(md->m, 0, P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(md->v, 0, P * sizeof(float));
  std::vector<int32_t> perm(static_cast<size_t>(count));
  std::iota(perm.begin(), perm.end(), 0);
  std::mt19937_64 g(o.seed);
  for (int ep = 0; ep < o.epochs && e == hipSuccess; ++ep) {
    for (int64_t i = count - 1; i > 0; --i) {  // Fisher-Yates
      const int64_t j = int64_t(g() % uint64_t(i + 1));
      std::swap(perm[size_t(i)], perm[size_t(j)]);
    }
    e = hipMemcpyAsync(idx, perm.data(), size_t(count) * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // perm is rewritten next epoch
    for (int64_t st = 0; st < count && e == hipSuccess; st += o.batch) {
      const int64_t nb = std::min<int64_t>(o.batch, count - st);
      e = k::mlp_grad_launch(md->params, x, t_std, idx + st, nb, b.partial, b.loss, s);
      if (e == hipSuccess)
        e = k::mlp_reduce_launch(b.partial, k::mlp_blocks(nb), nullptr, md->params, md->m, md->v,
                                 o.lr, 0.9f, 0.999f, 1e-8f, md->step + 1, s);
      ++md->step;
    }
  }
  double l = 0.0;
  if (e == hipSuccess) e = k::mlp_grad_launch(md->params, x, t_std, nullptr, count, b.partial, b.loss, s);
  if (e == hipSuccess) l = sum_loss(b.loss, k::mlp_blocks(count), s, &e);
  if (t_std) (void)hipFree(t_std);
  if (idx) (void)hipFree(idx);
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_train");
  if (final_loss) *final_loss = l / double(count);
  return HEXLA_OK;
}

hexla_status hexla_model_predict(hexla_model* md, const float* x, int64_t count, float* y) {
  if (!md || !md->ctx || (count > 0 && (!x || !y)) || count < 0) return HEXLA_E_INVALID_ARG;
  hipError_t e = enter_device(md->ctx->device);
  if (e == hipSuccess)
    e = k::mlp_predict_launch(md->params, x, count, md->y_std, md->y_mean, y, md->ctx->stream);
  if (e != hipSuccess) return dev_err(md->ctx, e, "model_predict");
  return HEXLA_OK;
}

hexla_status hexla_model_save(hexla_model* md, const char* path) {
  if (!md || !md->ctx || !path) return HEXLA_E_INVALID_ARG;
  std::vector<float> h(P);
  hexla_status st = hexla_model_get_params(md, h.data(), P, nullptr, nullptr);
  if (st != HEXLA_OK) return st;
  std::ofstream f(path);
  if (!f) return set_err(md->ctx, HEXLA_E_INVALID_ARG, std::string("cannot write ") + path);
  char buf[64];
  f << "hexla-mlp 1 gfx950 " << F << " " << P << "\n";
  std::snprintf(buf, sizeof(buf), "%.9g %.9g\n", md->y_mean, md->y_std);
  f << buf;
  for (float v : h) {
    std::snprintf(buf, sizeof(buf), "%.9g\n", v);
    f << buf;
  }
  return f ? HEXLA_OK : set_err(md->ctx, HEXLA_E_INVALID_ARG, "model_save: write failed");
}

hexla_status hexla_model_load(hexla_ctx* ctx, const char* path, hexla_model** out) {
  if (!ctx || !path || !out) return HEXLA_E_INVALID_ARG;
  *out = nullptr;
  std::ifstream f(path);
  if (!f) return set_err(ctx, HEXLA_E_INVALID_ARG, std::string("cannot read ") + path);
  std::string magic, target;
  int ver = 0, nf = 0, np = 0;
  float mean = 0.f, sd = 1.f;
  if (!(f >> magic >> ver >> target >> nf >> np >> mean >> sd) || magic != "hexla-mlp" ||
      ver != 1 || nf != F || np != P)
    return set_err(ctx, HEXLA_E_INVALID_ARG, "model_load: not a model file of this layout");
  if (target != "gfx950")
    return set_err(ctx, HEXLA_E_INVALID_ARG, "model_load: model is for " + target);
  std::vector<float> h(P);
  for (float& v : h)
    if (!(f >> v)) return set_err(ctx, HEXLA_E_INVALID_ARG, "model_load: truncated file");
  hexla_model* md = nullptr;
  hexla_status st = hexla_model_create(ctx, 0, &md);
  if (st != HEXLA_OK) return st;
  st = hexla_model_set_params(md, h.data(), P, mean, sd);
  if (st != HEXLA_OK) {
    (void)hexla_model_destroy(md);
    return st;
  }
  *out = md;
  return HEXLA_OK;
}

hexla_status hexla_ctx_set_model(hexla_ctx* ctx, hexla_model* md) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  if (md && md->ctx != ctx) return set_err(ctx, HEXLA_E_INVALID_ARG, "model belongs to another context");
  ctx->model = md;
  return HEXLA_OK;
}

hexla_status hexla_timing_log(hexla_ctx* ctx, const char* path) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  ctx->timing_log = path ? std::string(path) : std::string();
  if (path) {
    std::ofstream f(path, std::ios::app);
    if (!f) {
      ctx->timing_log.clear();
      return set_err(ctx, HEXLA_E_INVALID_ARG, std::string("cannot write ") + path);
    }
  }
  return HEXLA_OK;
}

}  // extern "C"
