// Host-side structures shared by the builder, the planner and the evaluator.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "hexla.h"
#include "kernels.h"

namespace hexla {

enum NodeKind : uint8_t { NK_LEAF = 0, NK_SCALAR = 1, NK_UNARY = 2, NK_BINARY = 3 };

// One marker of the delayed expression (the Op/Glue objects of Sec. II): a
// leaf borrows a matrix, a scalar is copied, operators refer to children.
struct Node {
  uint8_t kind = NK_LEAF;
  int op = 0;
  uint32_t a = 0, b = 0;
  const void* ptr = nullptr;
  int64_t ld = 1;
  int dtype = -1;  // storage type of the value (-1 for scalars)
  double value = 0.0;
  int64_t rows = 0, cols = 0;
  bool scalar = false;
  int64_t r0 = 0, c0 = 0;  // submatrix view: first row and column in the operand
};

enum class Buf : uint8_t { None, Leaf, Work, Out };

// Address of a matrix: a borrowed leaf pointer, or a byte offset into the
// caller's workspace or output buffer (bound at execute time).
struct Ref {
  Buf buf = Buf::None;
  int64_t off = 0;
  const void* ptr = nullptr;
};

// A rows x cols view; element (i, j) lives at storage (j, i) when trans.
// ld == -1 means "the leading dimension hexla_execute receives" (output).
// A strided view (a matrix's diagonal, a vector broadcast along rows or
// columns) holds element (i, j) at element offset i * str_i + j * str_j, and
// `span` elements of storage; it is read only by element-wise programs.
struct View {
  Ref ref;
  int64_t rows = 0, cols = 0, ld = 1;
  bool trans = false;
  bool is_leaf = false;       // a borrowed leaf (not a temporary)
  const void* leaf_ptr = nullptr;
  bool strided = false;
  int64_t str_i = 0, str_j = 0, span = 0;
};

// Storage range of a borrowed leaf, for the aliasing checks at execute time.
struct Range {
  const void* ptr = nullptr;
  uint64_t bytes = 0;
  int64_t ld = 0;
  bool trans = false;
};

struct EwHost {
  int32_t n_instr = 0;
  uint8_t op[k::kEwMaxInstr] = {};
  uint8_t arg[k::kEwMaxInstr] = {};
  double cst[k::kEwMaxConst] = {};
  int n_cst = 0;
  std::vector<View> leaves;
  int n_arith = 0;  // arithmetic operations per element (flop count)
  bool ident = false;
};

enum class StepKind : uint8_t { Ew, Gemv, Gemm, LuFactor, LuSolve, IrSolve, Fill, DiagProd, EwSum,
                                StructSolve };

// Workspace of a mixed-precision solve (low-precision LU + FP64 refinement).
struct IrWork {
  Ref s_low;     // n x n low-precision working copy (LU in place), ld n
  Ref rowid;     // n ints
  Ref luwork;    // panel scratch of the low-precision LU
  Ref r64;       // n x nrhs FP64 residual
  Ref r_low;     // n x nrhs residual in the low precision
  Ref d_low;     // n x nrhs correction in the low precision
  Ref scratch;   // norm partials
  Ref norms;     // 4 doubles: ||S||, ||R||, ||X||, ||D||
  Ref partial;   // split-K partials of the residual product
  k::GemmConfig res_cfg{};
  int update_precision = 0;  // k::GemmPrecision of the LU's trailing updates
  bool panel_fp64 = false;   // panels factored in FP64 (pivots on FP64 values)
  int max_iter = 30;
  double tol_scale = 0.0;    // 0: sqrt(n)
};

struct Step {
  StepKind kind = StepKind::Ew;
  int dtype = 0;
  std::string name;
  // Ew: program over `ew` written to `out`; Gemv/Gemm: C = alpha op(A) op(B) + beta C
  EwHost ew;
  bool has_epi = false;
  View out, A, B, C;
  double alpha = 1.0, beta = 0.0;
  int mode = 0;       // gemm: 0 full, 1 symmetric (SYRK)
  int precision = 0;  // gemm: k::GemmPrecision
  k::GemmConfig cfg{};
  Ref partial;
  int64_t partial_cap = 0;  // bytes reserved for split-K partials
  int64_t m = 0, n = 0, kk = 0, nrhs = 0;
  Ref rowid, luwork;
  IrWork ir;
  // DiagProd: out (a vector with element stride incd, or 1 x 1 when sum)
  // gets alpha * diag(op(A) op(B)) or its sum; m = diagonal length, kk the
  // contraction. EwSum: out (1 x 1) = alpha * the sum of `ew` over m x n.
  int64_t incd = 1;
  bool sum = false;
  // StructSolve: S (A) copied by `ew` into the working matrix `out`, the
  // solver chosen at execute time from the structure of S (or Cholesky when
  // the planner knows S = X X^T); B, C: right-hand sides and solution.
  bool spd_known = false;
  Ref coef, info;
  double flops = 0.0, bytes = 0.0;
  // Ew: kernel generated for this program (null: interpreter)
  std::string cg_src;
  hipFunction_t cg_fn = nullptr;
  std::string cg_err;
};

}  // namespace hexla

struct hexla_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  std::vector<hexla::Node> nodes;
  std::string err;
  int32_t* d_status = nullptr;  // [0] status, [1] timeout, [2] singular column, [3] ir iterations
  hexla::k::Lookahead side;     // the LU's second stream and events (made with the context)
  std::map<std::string, hexla::k::GemmConfig> tuned;  // autotuned product configurations
  int32_t host_status = 0;         // deferred status raised by host-driven loops
  int32_t host_ir_iterations = 0;  // iterations of the last refined solve
  double host_ir_berr = 0.0;       // its backward error ||R||/(||S|| ||X||), last residual
  int32_t host_solver = -1;        // solver of the last structure-aware solve (hexla_solver)
  hexla_model* model = nullptr;    // cost model of the learned planner (borrowed)
  std::string timing_log;          // autotune timings are appended here when set
  // objects made from this context; destroying the context detaches them
  std::set<hexla_plan*> plans;
  std::set<hexla_batch*> batches;
  std::set<hexla_model*> models;
};

struct hexla_plan {
  hexla_ctx* ctx = nullptr;
  hexla_plan_opts opts{};
  std::vector<hexla::Step> steps;
  int64_t rows = 0, cols = 0;
  int dtype = 0;
  uint64_t ws_bytes = 0;
  double flops = 0, bytes = 0, macs = 0;
  std::vector<hexla::Range> leaf_ranges;     // read by products, solves, epilogues
  std::vector<hexla::Range> ew_leaf_ranges;  // read by element-wise passes
  std::vector<std::string> learned_notes;     // JSON of the learned planner's decisions
  hipGraph_t graph = nullptr;                 // captured launches (hexla_plan_capture)
  hipGraphExec_t graph_exec = nullptr;
  ~hexla_plan();
};

namespace hexla {
// Makes the device current and drops an error left behind by HIP calls made
// outside the library, so that hipGetLastError after a launch reports that
// launch only.
inline hipError_t enter_device(int device) {
  const hipError_t e = hipSetDevice(device);
  (void)hipGetLastError();
  return e;
}
// A destroyed context leaves its batches and models without one: they can
// then only be destroyed.
void detach_batch(hexla_batch* b);
void detach_model(hexla_model* md);
}  // namespace hexla

namespace hexla {
struct GemmBind {
  int ta = 0, tb = 0;
  const void* A = nullptr;
  int64_t lda = 0;
  const void* B = nullptr;
  int64_t ldb = 0;
  void* C = nullptr;
  int64_t ldc = 0;
  void* partial = nullptr;
};
hexla_status check_buffers(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                           size_t workspace_bytes);
hexla_status run_steps(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                       hipStream_t st);
GemmBind bind_gemm(const Step& s, void* out, int64_t ld_out, void* workspace);
hipError_t launch_gemm_step(const Step& s, const GemmBind& gb, const k::GemmConfig& cfg,
                            hipStream_t st);
std::string tune_key(const Step& s, int ta, int tb);
size_t gemm_max_partial(const Step& s);
std::vector<k::GemmConfig> gemm_candidates(const Step& s);
// learned cost model (model.cpp)
void product_features(int dtype, int precision, int mode, int ta, int tb, int64_t m, int64_t n,
                      int64_t kk, int tile, int split, float* out);
void product_features_many(int dtype, int precision, int mode, int ta, int tb, int64_t m,
                           int64_t n, int64_t kk, const k::GemmConfig* cfg, int count, float* out);
// the configurations the learned planner prices for one product: per tile,
// no split-K and the split counts that fill whole rounds of 512, 1024 and
// 2048 workgroup slots, plus the default choice
std::vector<k::GemmConfig> learned_candidates(const Step& s);
bool model_predict_us(hexla_model* md, const std::vector<float>& x, std::vector<float>& us,
                      std::string* err);
hexla_status set_err(const hexla_ctx* ctx, hexla_status st, const std::string& msg);
size_t dtype_size(int dtype);
// generated element-wise kernels (codegen.cpp)
bool codegen_enabled();
std::string codegen_source(const EwHost& p, int dtype);
hipFunction_t codegen_get(int device, const std::string& src, std::string* err);
hipError_t codegen_launch(hipFunction_t fn, int dtype, const std::vector<const void*>& leaves,
                          void* out, int64_t n_total, hipStream_t s);
}  // namespace hexla
