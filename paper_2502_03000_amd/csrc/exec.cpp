// Evaluator: binds the caller's output and workspace to the plan and launches
// its kernels on the context's stream (the evaluation at assignment of
// Sec. II, done asynchronously on the device).
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "internal.h"

namespace hexla {
namespace {

struct Bind {
  char* out;
  int64_t ld_out;
  char* ws;
};

void* addr(const Ref& r, const Bind& b) {
  switch (r.buf) {
    case Buf::Leaf: return const_cast<void*>(r.ptr);
    case Buf::Work: return b.ws + r.off;
    case Buf::Out: return b.out + r.off;
    default: return nullptr;
  }
}

View resolve(View v, const Bind& b) {
  if (v.ld < 0) v.ld = b.ld_out;
  return v;
}

int64_t si(const View& v) { return v.strided ? v.str_i : (v.trans ? v.ld : 1); }
int64_t sj(const View& v) { return v.strided ? v.str_j : (v.trans ? 1 : v.ld); }

k::EwProgram make_prog(const EwHost& h, int64_t rows, int64_t cols, const Bind& b) {
  k::EwProgram p{};
  p.n_instr = h.n_instr;
  for (int i = 0; i < h.n_instr; ++i) {
    p.op[i] = h.op[i];
    p.arg[i] = h.arg[i];
  }
  for (int i = 0; i < h.n_cst; ++i) p.cst[i] = h.cst[i];
  p.n_leaf = int32_t(h.leaves.size());
  p.rows = rows;
  p.cols = cols;
  p.uses_ident = h.ident ? 1 : 0;
  bool contig = true;
  for (size_t i = 0; i < h.leaves.size(); ++i) {
    const View v = resolve(h.leaves[i], b);
    p.leaf[i].ptr = addr(v.ref, b);
    p.leaf[i].si = si(v);
    p.leaf[i].sj = sj(v);
    contig = contig && (rows == 1 || p.leaf[i].si == 1) && (cols == 1 || p.leaf[i].sj == rows);
  }
  p.contiguous = contig ? 1 : 0;
  return p;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return na && nb && x < y + nb && y < x + na;
}

hexla_status device_err(hexla_ctx* ctx, hipError_t e, const char* what) {
  return set_err(ctx, HEXLA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace
}  // namespace hexla

using namespace hexla;

namespace hexla {

hexla_status check_buffers(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                           size_t workspace_bytes) {
  if (!plan || !plan->ctx) return HEXLA_E_INVALID_ARG;
  hexla_ctx* ctx = plan->ctx;
  if (ctx->device < 0) return set_err(ctx, HEXLA_E_UNSUPPORTED, "dry-run context cannot execute");
  const size_t esz = dtype_size(plan->dtype);
  if (ld_out < (plan->rows > 1 ? plan->rows : 1))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: ld_out < rows");
  const uint64_t out_bytes =
      plan->rows * plan->cols > 0 ? uint64_t(((plan->cols - 1) * ld_out + plan->rows) * int64_t(esz)) : 0;
  if (out_bytes && !out) return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: null output");
  if (workspace_bytes < plan->ws_bytes || (plan->ws_bytes && !workspace))
    return set_err(ctx, HEXLA_E_INVALID_ARG,
                   "execute: workspace smaller than " + std::to_string(plan->ws_bytes) + " bytes");
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255u))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: workspace not 256-byte aligned");
  for (const Range& r : plan->leaf_ranges) {
    if (overlap(out, out_bytes, r.ptr, r.bytes))
      return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: output overlaps an operand of a product or solve");
    if (overlap(workspace, plan->ws_bytes, r.ptr, r.bytes))
      return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: workspace overlaps an operand");
  }
  for (const Range& r : plan->ew_leaf_ranges) {
    const bool in_place = r.ptr == out && r.ld == ld_out && !r.trans;
    if (!in_place && overlap(out, out_bytes, r.ptr, r.bytes))
      return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: output overlaps an operand");
    if (overlap(workspace, plan->ws_bytes, r.ptr, r.bytes))
      return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: workspace overlaps an operand");
  }
  if (overlap(workspace, plan->ws_bytes, out, out_bytes))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "execute: workspace overlaps the output");
  return HEXLA_OK;
}

hipError_t launch_gemm_step(const Step& s, const GemmBind& gb, const k::GemmConfig& cfg,
                            hipStream_t st) {
  return k::gemm_launch(s.dtype, s.precision, s.mode, gb.ta, gb.tb, s.m, s.n, s.kk, s.alpha,
                        gb.A, gb.lda, gb.B, gb.ldb, s.beta, gb.C, gb.ldc, gb.partial, cfg, st);
}

GemmBind bind_gemm(const Step& s, void* out, int64_t ld_out, void* workspace) {
  const Bind b{static_cast<char*>(out), ld_out, static_cast<char*>(workspace)};
  const View A = resolve(s.A, b), B = resolve(s.B, b), C = resolve(s.C, b);
  GemmBind g;
  g.ta = A.trans ? 1 : 0;
  g.tb = B.trans ? 1 : 0;
  g.A = addr(A.ref, b);
  g.lda = A.ld;
  g.B = addr(B.ref, b);
  g.ldb = B.ld;
  g.C = addr(C.ref, b);
  g.ldc = C.ld;
  g.partial = addr(s.partial, b);
  return g;
}

// Mixed-precision solve of an FP64 system (see hexla_solve_precision): LU in
// the low precision (FP32 storage; FP64 panels for the FP16 and split-BF16
// update forms), first solve, then FP64 residual / low-precision correction
// steps. The loop reads the norms after each step (one small device-to-host
// copy). Outcome: converged (OK); the correction grew (it is dropped) or the
// cap was reached (deferred HEXLA_E_NO_CONVERGENCE); the correction shrank
// by less than half (it is applied and the loop ends): OK when the backward
// error ||R||/(||S|| ||X||) of the last residual formed is at most n * 2^-53,
// else HEXLA_E_NO_CONVERGENCE.
hexla_status run_ir_solve(hexla_ctx* ctx, const Step& s, const Bind& b, hipStream_t st) {
  const IrWork& w = s.ir;
  const int64_t n = s.n, r = s.nrhs;
  const View S = resolve(s.A, b), B = resolve(s.B, b), X = resolve(s.C, b);
  void* s_low = addr(w.s_low, b);
  int32_t* rowid = static_cast<int32_t*>(addr(w.rowid, b));
  void* r64 = addr(w.r64, b);
  void* r_low = addr(w.r_low, b);
  void* d_low = addr(w.d_low, b);
  double* scratch = static_cast<double*>(addr(w.scratch, b));
  double* norms = static_cast<double*>(addr(w.norms, b));
  const int64_t ldn = std::max<int64_t>(n, 1);
  auto fail = [&](hipError_t e, const char* what) { return device_err(ctx, e, what); };
  hipError_t e = k::cast_launch(0, 1, n, n, addr(S.ref, b), si(S), sj(S), s_low, ldn, st);
  if (e != hipSuccess) return fail(e, "ir: cast S");
  // ||S||inf of the (rounded) copy, before it is factored in place
  e = k::norm_inf_launch(1, n, n, s_low, ldn, scratch, norms + 0, st);
  if (e != hipSuccess) return fail(e, "ir: norm S");
  e = k::lu_factor_launch(1, n, s_low, ldn, rowid, addr(w.luwork, b), ctx->d_status, st,
                          &ctx->side, w.update_precision, w.panel_fp64);
  if (e != hipSuccess) return fail(e, "ir: lu");
  // X0 = LU^-1 B in the low precision
  e = k::cast_launch(0, 1, n, r, addr(B.ref, b), si(B), sj(B), r_low, ldn, st);
  if (e == hipSuccess) e = k::lu_solve_launch(1, n, r, s_low, ldn, rowid, addr(w.luwork, b), r_low, ldn, d_low, ldn,
                                                ctx->d_status, st);
  if (e == hipSuccess) e = k::cast_launch(1, 0, n, r, d_low, 1, ldn, addr(X.ref, b), X.ld, st);
  if (e != hipSuccess) return fail(e, "ir: first solve");
  const double u = std::ldexp(1.0, -53);
  const double tol = (w.tol_scale > 0 ? w.tol_scale : 1.0) * u;
  double h[4] = {0, 0, 0, 0};
  double d_prev = -1.0, berr = 0.0;
  int it = 0;
  enum { kConverged, kCap, kDiverging, kStagnated } outcome = kCap;
  for (;; ++it) {
    // R = B - S X (FP64)
    e = k::cast_launch(0, 0, n, r, addr(B.ref, b), si(B), sj(B), r64, ldn, st);
    if (e == hipSuccess)
      e = k::gemm_launch(0, 0, 0, S.trans ? 1 : 0, 0, n, r, n, -1.0, addr(S.ref, b), S.ld,
                         addr(X.ref, b), X.ld, 1.0, r64, ldn, addr(w.partial, b), w.res_cfg, st);
    if (e == hipSuccess) e = k::norm_inf_launch(0, n, r, r64, ldn, scratch, norms + 1, st);
    if (e == hipSuccess) e = k::norm_inf_launch(0, n, r, addr(X.ref, b), X.ld, scratch, norms + 2, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, norms, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e, "ir: residual");
    const double scale = h[0] * h[2];
    berr = scale > 0.0 ? h[1] / scale : (h[1] > 0.0 ? HUGE_VAL : 0.0);
    if (h[1] <= tol * scale) {
      outcome = kConverged;
      break;
    }
    if (it >= w.max_iter) break;
    // D = LU^-1 R (low precision), stop when the correction stagnates
    e = k::cast_launch(0, 1, n, r, r64, 1, ldn, r_low, ldn, st);
    if (e == hipSuccess) e = k::lu_solve_launch(1, n, r, s_low, ldn, rowid, addr(w.luwork, b), r_low, ldn, d_low, ldn,
                                                ctx->d_status, st);
    if (e == hipSuccess) e = k::norm_inf_launch(1, n, r, d_low, ldn, scratch, norms + 3, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h + 3, norms + 3, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e, "ir: correction");
    // a growing correction is dropped; a slowly shrinking one is the last
    if (d_prev >= 0.0 && h[3] > d_prev) {
      outcome = kDiverging;
      break;
    }
    e = k::add_mixed_launch(1, n, r, static_cast<double*>(addr(X.ref, b)), X.ld, d_low, ldn, st);
    if (e != hipSuccess) return fail(e, "ir: update");
    if (d_prev >= 0.0 && h[3] > 0.5 * d_prev) {
      ++it;
      outcome = kStagnated;
      break;
    }
    d_prev = h[3];
  }
  ctx->host_ir_iterations = it;
  ctx->host_ir_berr = berr;
  const bool accepted = outcome == kConverged || (outcome == kStagnated && berr <= double(n) * u);
  if (!accepted && ctx->host_status == 0) ctx->host_status = HEXLA_E_NO_CONVERGENCE;
  return HEXLA_OK;
}

// Symmetric for the solver's purpose: S_ij and S_ji differ by at most
// n u max |S| (u the unit roundoff of the storage type), the size of the
// rounding differences between the two triangles of a product X X^T formed
// by a general GEMM; the Cholesky factorisation reads the lower triangle.
bool symmetric(const int32_t* h, int64_t n, int dtype) {
  if (!h[2]) return true;
  double amax, dmax;
  std::memcpy(&amax, h + 8, sizeof(double));
  std::memcpy(&dmax, h + 10, sizeof(double));
  const double u = std::ldexp(1.0, dtype == HEXLA_F64 ? -53 : -24);
  return dmax <= double(n) * u * amax;
}

// Structure-aware solve (see hexla_solver): copy S into the working matrix,
// read its structure (one pass and one wait for four integers) unless the
// planner knows S = X X^T, then run the solver that structure allows. A
// Cholesky whose pivot is not positive falls back to LU on a fresh copy.
hexla_status run_struct_solve(hexla_ctx* ctx, const Step& s, const Bind& b, hipStream_t st) {
  const int64_t n = s.n, r = s.nrhs;
  ctx->host_solver = -1;
  if (n == 0 || r == 0) return HEXLA_OK;
  const View B = resolve(s.B, b), X = resolve(s.C, b), W = resolve(s.out, b);
  void* wm = addr(W.ref, b);
  const int64_t ldw = std::max<int64_t>(n, 1);
  int32_t* info = static_cast<int32_t*>(addr(s.info, b));
  void* xo = addr(X.ref, b);
  const size_t esz = dtype_size(s.dtype);
  auto fail = [&](hipError_t e, const char* what) { return device_err(ctx, e, what); };
  auto copy_s = [&]() {
    const k::EwProgram p = make_prog(s.ew, n, n, b);
    return k::ew_launch(s.dtype, p, wm, 1, ldw, st);
  };
  auto copy_b = [&](void* dst, int64_t ldd) {
    return hipMemcpy2DAsync(dst, size_t(ldd) * esz, addr(B.ref, b), size_t(B.ld) * esz,
                            size_t(n) * esz, size_t(r), hipMemcpyDeviceToDevice, st);
  };
  auto read_info = [&](int32_t* h) {
    hipError_t e = hipMemcpyAsync(h, info, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  };
  auto singular = [&]() {
    if (ctx->host_status == 0) ctx->host_status = HEXLA_E_SINGULAR;
  };
  alignas(8) int32_t h[16] = {};
  hipError_t e = copy_s();
  if (e != hipSuccess) return fail(e, "solve: copy");
  int solver = HEXLA_SOLVER_CHOLESKY;
  if (!s.spd_known) {
    e = k::structure_launch(s.dtype, n, wm, ldw, info, st);
    if (e == hipSuccess) e = read_info(h);
    if (e != hipSuccess) return fail(e, "solve: structure");
    const int kl = h[0], ku = h[1];
    if (kl == 0 && ku == 0) solver = HEXLA_SOLVER_DIAGONAL;
    else if (kl == 0) solver = HEXLA_SOLVER_UPPER;
    else if (ku == 0) solver = HEXLA_SOLVER_LOWER;
    else if (kl <= 1 && ku <= 1) solver = HEXLA_SOLVER_TRIDIAGONAL;
    else if (!h[3] && symmetric(h, n, s.dtype)) solver = HEXLA_SOLVER_CHOLESKY;
    else solver = HEXLA_SOLVER_LU;
    // a triangular or diagonal matrix with a zero on its diagonal is singular
    if (solver >= HEXLA_SOLVER_LOWER && solver != HEXLA_SOLVER_TRIDIAGONAL && h[5]) singular();
  } else {
    e = k::fill_i32_launch(info, 16, 0, st);
    if (e != hipSuccess) return fail(e, "solve: clear");
  }
  if (solver == HEXLA_SOLVER_CHOLESKY) {
    e = k::chol_factor_launch(s.dtype, n, wm, ldw, info, addr(s.coef, b), st, &ctx->side);
    if (e == hipSuccess) e = read_info(h);
    if (e != hipSuccess) return fail(e, "solve: cholesky");
    if (h[4]) {  // not positive definite: LU on a fresh copy
      solver = HEXLA_SOLVER_LU;
      e = copy_s();
      if (e != hipSuccess) return fail(e, "solve: copy");
    } else {
      e = copy_b(xo, X.ld);
      if (e == hipSuccess)
        e = k::tri_solve_launch(s.dtype, 0, n, r, wm, ldw, xo, X.ld, addr(s.coef, b), true,
                                ctx->d_status, st);
      if (e != hipSuccess) return fail(e, "solve: cholesky substitution");
    }
  }
  switch (solver) {
    case HEXLA_SOLVER_DIAGONAL: {  // X = B ./ diag(S), the diagonal broadcast along rows
      k::EwProgram p{};
      p.n_instr = 3;
      p.op[0] = k::EW_LEAF;
      p.arg[0] = 0;
      p.op[1] = k::EW_LEAF;
      p.arg[1] = 1;
      p.op[2] = k::EW_DIV;
      p.n_leaf = 2;
      p.rows = n;
      p.cols = r;
      p.leaf[0].ptr = addr(B.ref, b);
      p.leaf[0].si = 1;
      p.leaf[0].sj = B.ld;
      p.leaf[1].ptr = wm;
      p.leaf[1].si = ldw + 1;
      p.leaf[1].sj = 0;
      e = k::ew_launch(s.dtype, p, xo, 1, X.ld, st);
      break;
    }
    case HEXLA_SOLVER_LOWER:
    case HEXLA_SOLVER_UPPER:
      e = copy_b(xo, X.ld);
      if (e == hipSuccess)
        e = k::tri_solve_launch(s.dtype, solver == HEXLA_SOLVER_LOWER ? 1 : 2, n, r, wm, ldw, xo,
                                X.ld, addr(s.coef, b), false, ctx->d_status, st);
      break;
    case HEXLA_SOLVER_TRIDIAGONAL:
      e = copy_b(xo, X.ld);
      if (e == hipSuccess)
        e = k::gtsv_launch(s.dtype, n, r, wm, ldw, xo, X.ld, addr(s.coef, b), info, st);
      if (e == hipSuccess) e = read_info(h);
      if (e == hipSuccess && h[5]) singular();
      break;
    case HEXLA_SOLVER_LU:
      e = k::lu_factor_launch(s.dtype, n, wm, ldw, static_cast<int32_t*>(addr(s.rowid, b)),
                              addr(s.luwork, b), ctx->d_status, st, &ctx->side);
      if (e == hipSuccess)
        e = k::lu_solve_launch(s.dtype, n, r, wm, ldw, static_cast<const int32_t*>(addr(s.rowid, b)),
                               addr(s.luwork, b), addr(B.ref, b), B.ld, xo, X.ld, ctx->d_status, st);
      break;
    default:
      break;
  }
  if (e != hipSuccess) return fail(e, "solve");
  ctx->host_solver = solver;
  return HEXLA_OK;
}

hexla_status run_steps(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                       hipStream_t st) {
  hexla_ctx* ctx = plan->ctx;
  hipError_t e = enter_device(ctx->device);
  if (e != hipSuccess) return device_err(ctx, e, "hipSetDevice");
  const Bind b{static_cast<char*>(out), ld_out, static_cast<char*>(workspace)};
  for (const Step& s : plan->steps) {
    switch (s.kind) {
      case StepKind::Ew: {
        const View o = resolve(s.out, b);
        const k::EwProgram p = make_prog(s.ew, o.rows, o.cols, b);
        void* optr = addr(o.ref, b);
        bool dense = s.cg_fn && p.contiguous && !p.uses_ident && aligned16(optr) && si(o) == 1 &&
                     (o.cols == 1 || sj(o) == o.rows);
        for (int l = 0; l < p.n_leaf && dense; ++l) dense = aligned16(p.leaf[l].ptr);
        if (dense) {
          std::vector<const void*> lv(p.n_leaf);
          for (int l = 0; l < p.n_leaf; ++l) lv[l] = p.leaf[l].ptr;
          e = codegen_launch(s.cg_fn, s.dtype, lv, optr, o.rows * o.cols, st);
        } else {
          e = k::ew_launch(s.dtype, p, optr, si(o), sj(o), st);
        }
        break;
      }
      case StepKind::Gemv: {
        const View A = resolve(s.A, b), B = resolve(s.B, b), C = resolve(s.C, b);
        const int trans = A.trans ? 1 : 0;
        const int64_t ms = trans ? A.cols : A.rows, ns = trans ? A.rows : A.cols;
        const int64_t incx = B.cols == 1 ? si(B) : sj(B);
        const int64_t incy = C.cols == 1 ? si(C) : sj(C);
        k::EwProgram p{};
        if (s.has_epi) p = make_prog(s.ew, C.rows, C.cols, b);
        e = k::gemv_launch(s.dtype, trans, ms, ns, s.alpha, addr(A.ref, b), A.ld, addr(B.ref, b),
                           incx, addr(C.ref, b), incy, s.has_epi ? &p : nullptr, st);
        break;
      }
      case StepKind::Gemm:
        e = launch_gemm_step(s, bind_gemm(s, out, ld_out, workspace), s.cfg, st);
        break;
      case StepKind::LuFactor: {
        const View A = resolve(s.A, b);
        e = k::lu_factor_launch(s.dtype, s.n, addr(A.ref, b), A.ld,
                                static_cast<int32_t*>(addr(s.rowid, b)), addr(s.luwork, b),
                                ctx->d_status, st, &ctx->side);
        break;
      }
      case StepKind::LuSolve: {
        const View A = resolve(s.A, b), B = resolve(s.B, b), C = resolve(s.C, b);
        e = k::lu_solve_launch(s.dtype, s.n, s.nrhs, addr(A.ref, b), A.ld,
                               static_cast<const int32_t*>(addr(s.rowid, b)), addr(s.luwork, b),
                               addr(B.ref, b), B.ld, addr(C.ref, b), C.ld, ctx->d_status, st);
        break;
      }
      case StepKind::IrSolve: {
        const hexla_status hs = run_ir_solve(ctx, s, b, st);
        if (hs != HEXLA_OK) return hs;
        break;
      }
      case StepKind::StructSolve: {
        const hexla_status hs = run_struct_solve(ctx, s, b, st);
        if (hs != HEXLA_OK) return hs;
        break;
      }
      case StepKind::DiagProd: {
        const View A = resolve(s.A, b), B = resolve(s.B, b), o = resolve(s.out, b);
        // incd 0: onto the diagonal of the output matrix
        const int64_t incd = s.incd ? s.incd : o.ld + 1;
        e = k::diagprod_launch(s.dtype, A.trans ? 1 : 0, B.trans ? 1 : 0, s.m, s.kk, s.alpha,
                               addr(A.ref, b), A.ld, addr(B.ref, b), B.ld, addr(o.ref, b), incd,
                               s.sum, addr(s.partial, b), st);
        break;
      }
      case StepKind::EwSum: {
        const View o = resolve(s.out, b);
        const k::EwProgram p = make_prog(s.ew, s.m, s.n, b);
        e = k::ew_sum_launch(s.dtype, p, s.alpha, addr(o.ref, b), addr(s.partial, b), st);
        break;
      }
      default:
        break;
    }
    if (e != hipSuccess) return device_err(ctx, e, s.name.c_str());
  }
  return HEXLA_OK;
}

}  // namespace hexla

extern "C" {

hexla_status hexla_execute(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                           size_t workspace_bytes) {
  const hexla_status st = check_buffers(plan, out, ld_out, workspace, workspace_bytes);
  if (st != HEXLA_OK) return st;
  return run_steps(plan, out, ld_out, workspace, plan->ctx->stream);
}

hexla_status hexla_split_bf16(hexla_ctx* ctx, const float* x, int64_t n, uint16_t* t0,
                              uint16_t* t1, uint16_t* t2, int32_t terms) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  if (ctx->device < 0) return set_err(ctx, HEXLA_E_UNSUPPORTED, "dry-run context cannot execute");
  if (n < 0 || (terms != 2 && terms != 3) || (n > 0 && (!x || !t0 || !t1 || (terms == 3 && !t2))))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "split_bf16: bad arguments");
  hipError_t e = enter_device(ctx->device);
  if (e == hipSuccess) e = k::split_bf16_launch(x, n, t0, t1, t2, terms, ctx->stream);
  if (e != hipSuccess) return device_err(ctx, e, "split_bf16");
  return HEXLA_OK;
}

hexla_status hexla_sync(hexla_ctx* ctx, hexla_report* report) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  hexla_report r{};
  r.singular_column = -1;
  r.solver = -1;
  if (ctx->device < 0) {
    if (report) *report = r;
    return HEXLA_OK;
  }
  hipError_t e = enter_device(ctx->device);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  int32_t h[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpy(h, ctx->d_status, sizeof(h), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(ctx->d_status, 0, sizeof(h));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return device_err(ctx, e, "hexla_sync");
  r.status = h[0] ? h[0] : ctx->host_status;
  r.ir_iterations = ctx->host_ir_iterations;
  r.ir_backward_error = ctx->host_ir_berr;
  r.solver = ctx->host_solver;
  ctx->host_solver = -1;
  ctx->host_status = 0;
  if (h[0] == HEXLA_E_SINGULAR) r.singular_column = h[2];
  if (h[1]) {
    r.status = HEXLA_E_DEVICE;
    set_err(ctx, HEXLA_E_DEVICE, "a device-wide barrier timed out");
  }
  if (report) *report = r;
  return HEXLA_OK;
}

}  // extern "C"
