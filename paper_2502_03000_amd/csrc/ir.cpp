// Context and expression builder: the marker objects of delayed evaluation
// (Sec. II). Building records references and scalar copies and checks sizes
// (the conformance checks of Sec. II); nothing is evaluated here.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "internal.h"

namespace hexla {

hexla_status set_err(const hexla_ctx* ctx, hexla_status st, const std::string& msg) {
  if (ctx) const_cast<hexla_ctx*>(ctx)->err = msg;
  return st;
}

size_t dtype_size(int dtype) { return dtype == HEXLA_F64 ? 8 : 4; }

namespace {

bool valid_node(const hexla_ctx* ctx, hexla_node n) { return n < ctx->nodes.size(); }

std::string shape(const Node& n) {
  return std::to_string(n.rows) + "x" + std::to_string(n.cols);
}

hexla_status push(hexla_ctx* ctx, const Node& n, hexla_node* out) {
  ctx->nodes.push_back(n);
  *out = hexla_node(ctx->nodes.size() - 1);
  return HEXLA_OK;
}

bool is_elementwise(int op) {
  return op == HEXLA_OP_PLUS || op == HEXLA_OP_MINUS || op == HEXLA_OP_SCHUR || op == HEXLA_OP_DIV;
}

}  // namespace
}  // namespace hexla

using hexla::Node;
using hexla::set_err;

extern "C" {

const char* hexla_version(void) { return "hexla 0.1 (gfx950)"; }

hexla_status hexla_ctx_create(int device, void* stream, hexla_ctx** out) {
  if (!out || device < -1) return HEXLA_E_INVALID_ARG;
  *out = nullptr;
  hexla_ctx* ctx = new hexla_ctx();
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  if (device >= 0) {
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ctx->d_status), 256);
    if (e == hipSuccess) e = hipMemset(ctx->d_status, 0, 256);
    // the LU's lookahead stream (default priority, like the caller's) and
    // events are made once here, so that executing a plan creates nothing
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->side.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->side.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->side.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      hexla_ctx_destroy(ctx);
      return HEXLA_E_DEVICE;
    }
  }
  *out = ctx;
  return HEXLA_OK;
}

hexla_status hexla_ctx_destroy(hexla_ctx* ctx) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  for (hexla_plan* p : ctx->plans) p->ctx = nullptr;
  for (hexla_batch* b : ctx->batches) hexla::detach_batch(b);
  for (hexla_model* md : ctx->models) hexla::detach_model(md);
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    if (ctx->side.s) (void)hipStreamSynchronize(ctx->side.s);
    if (ctx->side.done) (void)hipEventDestroy(ctx->side.done);
    if (ctx->side.ready) (void)hipEventDestroy(ctx->side.ready);
    if (ctx->side.s) (void)hipStreamDestroy(ctx->side.s);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
  }
  delete ctx;
  return HEXLA_OK;
}

hexla_status hexla_ctx_set_stream(hexla_ctx* ctx, void* stream) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  ctx->stream = static_cast<hipStream_t>(stream);
  return HEXLA_OK;
}

hexla_status hexla_ctx_clear_nodes(hexla_ctx* ctx) {
  if (!ctx) return HEXLA_E_INVALID_ARG;
  ctx->nodes.clear();
  return HEXLA_OK;
}

const char* hexla_last_error(const hexla_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hexla_status hexla_leaf(hexla_ctx* ctx, const void* ptr, int64_t rows, int64_t cols, int64_t ld,
                        hexla_dtype dtype, hexla_node* out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  if (rows < 0 || cols < 0)
    return set_err(ctx, HEXLA_E_INVALID_ARG, "leaf: negative size");
  if (ld < (rows > 1 ? rows : 1))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "leaf: ld < max(rows, 1)");
  if (dtype != HEXLA_F64 && dtype != HEXLA_F32)
    return set_err(ctx, HEXLA_E_INVALID_ARG, "leaf: unknown dtype");
  if (!ptr && rows * cols > 0) return set_err(ctx, HEXLA_E_INVALID_ARG, "leaf: null pointer");
  Node n;
  n.kind = hexla::NK_LEAF;
  n.ptr = ptr;
  n.rows = rows;
  n.cols = cols;
  n.ld = ld;
  n.dtype = dtype;
  return hexla::push(ctx, n, out);
}

hexla_status hexla_scalar(hexla_ctx* ctx, double value, hexla_node* out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  Node n;
  n.kind = hexla::NK_SCALAR;
  n.value = value;
  n.rows = n.cols = 1;
  n.scalar = true;
  return hexla::push(ctx, n, out);
}

hexla_status hexla_unary(hexla_ctx* ctx, hexla_op op, hexla_node a, hexla_node* out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  if (!hexla::valid_node(ctx, a)) return set_err(ctx, HEXLA_E_INVALID_ARG, "unary: bad node");
  const Node& x = ctx->nodes[a];
  Node n;
  n.kind = hexla::NK_UNARY;
  n.op = op;
  n.a = a;
  n.dtype = x.dtype;
  n.scalar = x.scalar;
  switch (op) {
    case HEXLA_OP_TRANS:
      n.rows = x.cols;
      n.cols = x.rows;
      break;
    case HEXLA_OP_NEG:
    case HEXLA_OP_EXP:
      n.rows = x.rows;
      n.cols = x.cols;
      break;
    case HEXLA_OP_INV:
      if (!x.scalar && x.rows != x.cols)
        return set_err(ctx, HEXLA_E_NOT_SQUARE, "inv: matrix is " + hexla::shape(x));
      n.rows = x.rows;
      n.cols = x.cols;
      break;
    case HEXLA_OP_DIAG:  // the main diagonal, min(m, n) x 1 (a scalar stays one)
      n.rows = x.scalar ? 1 : std::min(x.rows, x.cols);
      n.cols = 1;
      break;
    case HEXLA_OP_DIAGMAT:  // a vector spreads onto a square diagonal
      if (!x.scalar && (x.rows == 1 || x.cols == 1)) {
        n.rows = n.cols = std::max(x.rows, x.cols);
      } else {
        n.rows = x.rows;
        n.cols = x.cols;
      }
      break;
    case HEXLA_OP_TRACE:
      n.rows = n.cols = 1;
      break;
    default:
      return set_err(ctx, HEXLA_E_INVALID_ARG, "unary: unknown op");
  }
  return hexla::push(ctx, n, out);
}

hexla_status hexla_binary(hexla_ctx* ctx, hexla_op op, hexla_node a, hexla_node b,
                          hexla_node* out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  if (!hexla::valid_node(ctx, a) || !hexla::valid_node(ctx, b))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "binary: bad node");
  const Node& x = ctx->nodes[a];
  const Node& y = ctx->nodes[b];
  if (x.dtype >= 0 && y.dtype >= 0 && x.dtype != y.dtype)
    return set_err(ctx, HEXLA_E_DTYPE, "operands have different storage types");
  Node n;
  n.kind = hexla::NK_BINARY;
  n.op = op;
  n.a = a;
  n.b = b;
  n.dtype = x.dtype >= 0 ? x.dtype : y.dtype;
  n.scalar = x.scalar && y.scalar;
  if (op == HEXLA_OP_TIMES) {
    if (x.scalar) {
      n.rows = y.rows;
      n.cols = y.cols;
    } else if (y.scalar) {
      n.rows = x.rows;
      n.cols = x.cols;
    } else {
      if (x.cols != y.rows)
        return set_err(ctx, HEXLA_E_DIM,
                       "matrix product: " + hexla::shape(x) + " * " + hexla::shape(y));
      n.rows = x.rows;
      n.cols = y.cols;
    }
  } else if (hexla::is_elementwise(op)) {
    if (x.scalar) {
      n.rows = y.rows;
      n.cols = y.cols;
    } else if (y.scalar) {
      n.rows = x.rows;
      n.cols = x.cols;
    } else {
      if (x.rows != y.rows || x.cols != y.cols)
        return set_err(ctx, HEXLA_E_DIM,
                       "element-wise operation: " + hexla::shape(x) + " vs " + hexla::shape(y));
      n.rows = x.rows;
      n.cols = x.cols;
    }
  } else if (op == HEXLA_OP_SOLVE) {
    if (x.scalar || y.scalar)
      return set_err(ctx, HEXLA_E_UNSUPPORTED, "solve: scalar operand");
    if (x.rows != x.cols)
      return set_err(ctx, HEXLA_E_NOT_SQUARE, "solve: matrix is " + hexla::shape(x));
    if (x.rows != y.rows)
      return set_err(ctx, HEXLA_E_DIM, "solve: " + hexla::shape(x) + " vs " + hexla::shape(y));
    n.rows = x.cols;
    n.cols = y.cols;
  } else {
    return set_err(ctx, HEXLA_E_INVALID_ARG, "binary: unknown op");
  }
  return hexla::push(ctx, n, out);
}

hexla_status hexla_submatrix(hexla_ctx* ctx, hexla_node a, int64_t r0, int64_t c0, int64_t rows,
                             int64_t cols, hexla_node* out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  if (!hexla::valid_node(ctx, a)) return set_err(ctx, HEXLA_E_INVALID_ARG, "submatrix: bad node");
  const Node& x = ctx->nodes[a];
  if (x.scalar) return set_err(ctx, HEXLA_E_INVALID_ARG, "submatrix: scalar operand");
  if (r0 < 0 || c0 < 0 || rows < 0 || cols < 0)
    return set_err(ctx, HEXLA_E_INVALID_ARG, "submatrix: negative index or size");
  if (r0 + rows > x.rows || c0 + cols > x.cols)
    return set_err(ctx, HEXLA_E_DIM,
                   "submatrix: rows " + std::to_string(r0) + "+" + std::to_string(rows) +
                       ", columns " + std::to_string(c0) + "+" + std::to_string(cols) + " of " +
                       hexla::shape(x));
  Node n;
  n.kind = hexla::NK_UNARY;
  n.op = HEXLA_OP_SUBMAT;
  n.a = a;
  n.dtype = x.dtype;
  n.rows = rows;
  n.cols = cols;
  n.r0 = r0;
  n.c0 = c0;
  return hexla::push(ctx, n, out);
}

hexla_status hexla_node_shape(const hexla_ctx* ctx, hexla_node n, int64_t* rows, int64_t* cols,
                              int32_t* is_scalar) {
  if (!ctx || !hexla::valid_node(ctx, n)) return HEXLA_E_INVALID_ARG;
  const Node& x = ctx->nodes[n];
  if (rows) *rows = x.rows;
  if (cols) *cols = x.cols;
  if (is_scalar) *is_scalar = x.scalar ? 1 : 0;
  return HEXLA_OK;
}

hexla_status hexla_plan_opts_default(hexla_plan_opts* o) {
  if (!o) return HEXLA_E_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->planner = HEXLA_PLANNER_DP;
  o->product_precision = HEXLA_PRODUCT_PLAIN;
  o->solve_precision = HEXLA_SOLVE_PLAIN;
  o->fuse = 1;
  o->syrk = 1;
  o->ir_max_iter = 30;
  o->ir_tol_scale = 0.0;
  o->codegen = 1;
  return HEXLA_OK;
}

}  // extern "C"
