// Autotuning of the matrix products' tile and split-K configuration, the
// tuning table, the timing log the learned cost model trains on, and
// HIP-graph capture of a plan.
//
// The autotuner times every candidate configuration of each product on the
// caller's buffers (HIP events on the context's stream) and keeps the
// fastest in the plan and in the context's table; plans made later look the
// table up by (type, precision, mode, transposes, m, n, k). The table can be
// saved to and loaded from a text file, one entry per line, stamped with
// the target ("gfx950"); entries for another target are rejected.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <iomanip>
#include <fstream>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace hexla {

namespace {
constexpr const char* kTarget = "gfx950";
constexpr size_t kMaxCandidatePartial = size_t(512) << 20;  // bytes of split-K partials
}  // namespace

std::string tune_key(const Step& s, int ta, int tb) {
  std::ostringstream o;
  o << "d" << s.dtype << "p" << s.precision << "m" << s.mode << "a" << ta << "b" << tb << "_" << s.m
    << "x" << s.n << "x" << s.kk;
  return o.str();
}

// Candidate configurations of a product: every valid tile, each with a
// few split-K counts (target workgroups x minimum K steps per workgroup).
std::vector<k::GemmConfig> gemm_candidates(const Step& s) {
  std::vector<k::GemmConfig> out;
  std::set<std::pair<int, int>> seen;
  auto add = [&](k::GemmConfig c) {
    if (!seen.insert({c.tile, c.split}).second) return;
    if (k::gemm_partial_bytes(s.dtype, c, s.m, s.n) > kMaxCandidatePartial) return;
    out.push_back(c);
  };
  add(k::gemm_choose(s.dtype, s.precision, s.mode, s.m, s.n, s.kk));
  if (s.precision != 0) {  // the split-BF16 / FP16 family has one tile: split-K counts
    for (int split : {1, 2, 4, 8, 16}) add(k::GemmConfig{0, split});
    const int64_t tiles = k::gemm_tiles_for(s.dtype, 0, s.mode, s.m, s.n);  // 128 x 128 tiles
    for (int64_t slots : {512, 1024, 2048})
      if (slots / tiles >= 2 && slots / tiles <= 64) add(k::GemmConfig{0, int(slots / tiles)});
    return out;
  }
  for (int t = 0; t < k::gemm_tile_count(s.dtype); ++t) {
    if (!k::gemm_tile_valid(s.dtype, t, s.mode)) continue;
    add(k::GemmConfig{t, 1});
    for (int64_t target : {128, 256, 512, 1024})
      for (int64_t steps : {1, 2, 4, 8, 16})
        add(k::GemmConfig{t, k::gemm_split_for(s.dtype, t, s.mode, s.m, s.n, s.kk, target, steps)});
    // the largest split whose workgroups fit 512, 1024 or 2048 slots (2, 4 or
    // 8 per CU): whole rounds of workgroups, no short last round
    const int64_t tiles = k::gemm_tiles_for(s.dtype, t, s.mode, s.m, s.n);
    for (int64_t slots : {512, 1024, 2048}) {
      const int64_t split = slots / tiles;
      if (split >= 2)
        add(k::GemmConfig{t, k::gemm_split_for(s.dtype, t, s.mode, s.m, s.n, s.kk, split * tiles, 1)});
    }
  }
  return out;
}

std::vector<k::GemmConfig> learned_candidates(const Step& s) {
  std::vector<k::GemmConfig> out;
  out.reserve(48);
  auto add = [&](k::GemmConfig c) {
    for (const k::GemmConfig& q : out)
      if (q.tile == c.tile && q.split == c.split) return;
    if (k::gemm_partial_bytes(s.dtype, c, s.m, s.n) > kMaxCandidatePartial) return;
    out.push_back(c);
  };
  add(k::gemm_choose(s.dtype, s.precision, s.mode, s.m, s.n, s.kk));
  if (s.precision != 0) {
    for (int split : {1, 2, 4, 8, 16}) add(k::GemmConfig{0, split});
    return out;
  }
  for (int t = 0; t < k::gemm_tile_count(s.dtype); ++t) {
    if (!k::gemm_tile_valid(s.dtype, t, s.mode)) continue;
    add(k::GemmConfig{t, 1});
    const int64_t tiles = k::gemm_tiles_for(s.dtype, t, s.mode, s.m, s.n);
    for (int64_t slots : {512, 1024, 2048}) {
      const int64_t split = slots / tiles;
      if (split >= 2)
        add(k::GemmConfig{t, k::gemm_split_for(s.dtype, t, s.mode, s.m, s.n, s.kk, split * tiles, 1)});
    }
  }
  return out;
}

size_t gemm_max_partial(const Step& s) {
  size_t b = 0;
  for (const k::GemmConfig& c : gemm_candidates(s))
    b = std::max(b, k::gemm_partial_bytes(s.dtype, c, s.m, s.n));
  return b;
}

}  // namespace hexla

hexla_plan::~hexla_plan() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
}

using namespace hexla;

extern "C" {

hexla_status hexla_plan_autotune(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                                 size_t workspace_bytes, int32_t reps) {
  hexla_status st = check_buffers(plan, out, ld_out, workspace, workspace_bytes);
  if (st != HEXLA_OK) return st;
  hexla_ctx* ctx = plan->ctx;
  if (reps <= 0) reps = 5;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = enter_device(ctx->device);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::ofstream log;
  if (!ctx->timing_log.empty()) log.open(ctx->timing_log, std::ios::app);
  for (Step& s : plan->steps) {
    if (e != hipSuccess) break;
    if (s.kind != StepKind::Gemm) continue;
    const GemmBind gb = bind_gemm(s, out, ld_out, workspace);
    float best_ms = 1e30f;
    k::GemmConfig best = s.cfg;
    for (const k::GemmConfig& c : gemm_candidates(s)) {
      if (k::gemm_partial_bytes(s.dtype, c, s.m, s.n) > size_t(s.partial_cap)) continue;
      e = launch_gemm_step(s, gb, c, ctx->stream);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_gemm_step(s, gb, c, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      if (log.is_open())
        log << "{\"dtype\":" << s.dtype << ",\"precision\":" << s.precision
            << ",\"mode\":" << s.mode << ",\"ta\":" << gb.ta << ",\"tb\":" << gb.tb
            << ",\"m\":" << s.m << ",\"n\":" << s.n << ",\"k\":" << s.kk
            << ",\"tile\":" << c.tile << ",\"split\":" << c.split << ",\"us\":"
            << std::setprecision(6) << double(ms) * 1e3 / reps << "}\n";
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    s.cfg = best;
    ctx->tuned[tune_key(s, gb.ta, gb.tb)] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_err(ctx, HEXLA_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  if (plan->graph_exec) {  // a captured graph holds the old configurations
    (void)hipGraphExecDestroy(plan->graph_exec);
    (void)hipGraphDestroy(plan->graph);
    plan->graph_exec = nullptr;
    plan->graph = nullptr;
  }
  return HEXLA_OK;
}

hexla_status hexla_tune_save(const hexla_ctx* ctx, const char* path) {
  if (!ctx || !path) return HEXLA_E_INVALID_ARG;
  std::ofstream f(path);
  if (!f) return set_err(ctx, HEXLA_E_INVALID_ARG, std::string("cannot write ") + path);
  for (const auto& kv : ctx->tuned)
    f << kTarget << " " << kv.first << " " << kv.second.tile << " " << kv.second.split << "\n";
  return HEXLA_OK;
}

hexla_status hexla_tune_load(hexla_ctx* ctx, const char* path) {
  if (!ctx || !path) return HEXLA_E_INVALID_ARG;
  std::ifstream f(path);
  if (!f) return set_err(ctx, HEXLA_E_INVALID_ARG, std::string("cannot read ") + path);
  std::string target, key;
  int tile = 0, split = 0;
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    if (!(is >> target >> key >> tile >> split)) continue;
    if (target != kTarget) return set_err(ctx, HEXLA_E_INVALID_ARG, "tuning table is for " + target);
    if (split < 1 || split > 1024 || tile < 0) continue;
    ctx->tuned[key] = k::GemmConfig{tile, split};
  }
  return HEXLA_OK;
}

hexla_status hexla_plan_capture(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                                size_t workspace_bytes) {
  hexla_status st = check_buffers(plan, out, ld_out, workspace, workspace_bytes);
  if (st != HEXLA_OK) return st;
  hexla_ctx* ctx = plan->ctx;
  for (const Step& s : plan->steps)
    if (s.kind == StepKind::IrSolve)
      return set_err(ctx, HEXLA_E_UNSUPPORTED, "capture: a refined solve reads status on the host");
    else if (s.kind == StepKind::StructSolve)
      return set_err(ctx, HEXLA_E_UNSUPPORTED,
                     "capture: a structure-aware solve reads the matrix's structure on the host "
                     "(plan with solve_structure = 1 to capture an LU solve)");
  hipError_t e = enter_device(ctx->device);
  hipStream_t cs = nullptr;  // capture needs a stream other than the null stream
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    if (cs) (void)hipStreamDestroy(cs);
    return set_err(ctx, HEXLA_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
  }
  st = run_steps(plan, out, ld_out, workspace, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (st != HEXLA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  hipGraphExec_t x = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return set_err(ctx, HEXLA_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
  }
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  plan->graph = g;
  plan->graph_exec = x;
  return HEXLA_OK;
}

hexla_status hexla_plan_replay(hexla_plan* plan) {
  if (!plan || !plan->ctx) return HEXLA_E_INVALID_ARG;
  if (!plan->graph_exec) return set_err(plan->ctx, HEXLA_E_INVALID_ARG, "replay: nothing captured");
  hipError_t e = enter_device(plan->ctx->device);
  if (e == hipSuccess) e = hipGraphLaunch(plan->graph_exec, plan->ctx->stream);
  if (e != hipSuccess) return set_err(plan->ctx, HEXLA_E_DEVICE, std::string("replay: ") + hipGetErrorString(e));
  return HEXLA_OK;
}

}  // extern "C"
