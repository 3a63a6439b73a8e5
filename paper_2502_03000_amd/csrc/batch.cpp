// Batched plans: one template expression, many small instances of uneven
// size, evaluated by one persistent launch (device side: k_batch.hip).
//
// The template is compiled into a short program over vector slots: a matrix
// chain whose last factor is a vector runs right to left as matrix-vector
// products (with square factors every other bracketing costs n^3 per pair,
// so this is the order the cost-based reordering of Sec. II picks), inv(S)*x
// and solve(S, x) become an LU solve (Sec. I, Sec. II), and element-wise
// sub-expressions become one fused program (Sec. II). Instances are ordered
// by decreasing cost so that the queue hands out the longest work first.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

using hexla::Node;
using hexla::set_err;
namespace k = hexla::k;

struct hexla_batch {
  hexla_ctx* ctx = nullptr;
  int dtype = 0;
  int64_t count = 0, max_n = 0;
  k::BProgram prog{};
  k::BatchConfig cfg{};
  int max_grid = 0;
  bool has_solve = false;
  void* table = nullptr;  // pinned host copy of [program | order | instances]
  size_t table_bytes = 0, off_order = 0, off_inst = 0;
  int64_t stride = 0;     // scratch elements per workgroup
  uint64_t ws_bytes = 0;
  double flops = 0, bytes = 0;
  std::string ops_json;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  ~hexla_batch() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (table) (void)hipHostFree(table);
  }
};

namespace hexla {
namespace {

constexpr int kGrids[] = {256, 512, 768};
constexpr size_t kQueueBytes = 256;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

class BatchCompiler {
 public:
  BatchCompiler(const hexla_ctx* ctx, std::vector<uint32_t> leaves, int64_t t)
      : ctx_(ctx), leaves_(std::move(leaves)), t_(t) {
    p.out_slot = k::kBOut;
  }

  k::BProgram p{};
  hexla_status st = HEXLA_OK;
  std::string err;
  // per-instance cost: flops = c3 n^3 + c2 n^2 + c1 n
  double c3 = 0, c2 = 0, c1 = 0;
  std::vector<bool> leaf_is_matrix;
  std::ostringstream js;

  void compile(uint32_t root) {
    leaf_is_matrix.assign(leaves_.size(), false);
    for (size_t l = 0; l < leaves_.size(); ++l) leaf_is_matrix[l] = N(leaves_[l]).cols == t_;
    if (!is_vec(root)) return fail(HEXLA_E_DIM, "batch: the template result must be t x 1");
    if (is_chain_or_solve(root) || N(root).kind == NK_LEAF) {
      const int s = materialize(root);
      if (ok()) p.out_slot = s;
    } else {
      ew_op(root, k::kBOut);
    }
  }

 private:
  const hexla_ctx* ctx_;
  std::vector<uint32_t> leaves_;
  int64_t t_;
  bool used_[k::kBMaxSlots] = {};
  int n_ew_ = 0, n_cst_ = 0;
  bool first_op_ = true;

  bool ok() const { return st == HEXLA_OK; }
  void fail(hexla_status s, const std::string& m) {
    if (st == HEXLA_OK) {
      st = s;
      err = m;
    }
  }
  const Node& N(uint32_t n) const { return ctx_->nodes[n]; }
  bool is_vec(uint32_t n) const { return !N(n).scalar && N(n).rows == t_ && N(n).cols == 1; }
  bool is_mat(uint32_t n) const { return !N(n).scalar && N(n).rows == t_ && N(n).cols == t_; }
  int leaf_index(uint32_t n) const {
    const Node& x = N(n);
    for (size_t l = 0; l < leaves_.size(); ++l) {
      const Node& y = N(leaves_[l]);
      if (leaves_[l] == n || (y.ptr == x.ptr && y.rows == x.rows && y.cols == x.cols &&
                              y.ld == x.ld && y.dtype == x.dtype))
        return int(l);
    }
    return -1;
  }

  double scalar_value(uint32_t n) const {
    const Node& x = N(n);
    if (x.kind == NK_SCALAR) return x.value;
    if (x.kind == NK_UNARY) {
      const double a = scalar_value(x.a);
      switch (x.op) {
        case HEXLA_OP_NEG: return -a;
        case HEXLA_OP_EXP: return std::exp(a);
        case HEXLA_OP_INV: return 1.0 / a;
        default: return a;
      }
    }
    const double a = scalar_value(x.a), b = scalar_value(x.b);
    switch (x.op) {
      case HEXLA_OP_PLUS: return a + b;
      case HEXLA_OP_MINUS: return a - b;
      case HEXLA_OP_DIV: return a / b;
      default: return a * b;
    }
  }

  int alloc() {
    for (int s = 0; s < k::kBMaxSlots; ++s)
      if (!used_[s]) {
        used_[s] = true;
        return s;
      }
    fail(HEXLA_E_UNSUPPORTED, "batch: more live vectors than slots");
    return 0;
  }
  void release(int s) {
    if (s >= 0 && s < k::kBMaxSlots) used_[s] = false;
  }

  void push_op(const k::BOp& op) {
    if (!ok()) return;
    if (p.n_ops >= k::kBMaxOps) return fail(HEXLA_E_UNSUPPORTED, "batch: program too long");
    p.ops[p.n_ops++] = op;
    static const char* kinds[] = {"load", "gemv", "solve", "ew"};
    js << (first_op_ ? "" : ",") << "{\"op\":\"" << kinds[op.kind] << "\",\"dst\":"
       << (op.dst == k::kBOut ? -1 : int(op.dst));
    if (op.kind != k::B_EW) js << ",\"leaf\":" << int(op.leaf);
    if (op.kind == k::B_GEMV || op.kind == k::B_SOLVE) js << ",\"src\":" << int(op.src);
    if (op.kind == k::B_GEMV) js << ",\"trans\":" << int(op.trans) << ",\"alpha\":" << op.alpha;
    if (op.kind == k::B_EW) js << ",\"instructions\":" << int(op.ew_end - op.ew_begin);
    js << "}";
    first_op_ = false;
  }

  // products (with at least one matrix factor) and solves
  void flatten(uint32_t n, std::vector<uint32_t>& f, double& alpha) const {
    const Node& x = N(n);
    if (x.scalar) {
      alpha *= scalar_value(n);
    } else if (x.kind == NK_BINARY && x.op == HEXLA_OP_TIMES) {
      flatten(x.a, f, alpha);
      flatten(x.b, f, alpha);
    } else if (x.kind == NK_UNARY && x.op == HEXLA_OP_NEG) {
      alpha = -alpha;
      flatten(x.a, f, alpha);
    } else {
      f.push_back(n);
    }
  }
  bool is_chain_or_solve(uint32_t n) const {
    const Node& x = N(n);
    if (x.kind == NK_BINARY && x.op == HEXLA_OP_SOLVE) return true;
    if (!(x.kind == NK_BINARY && x.op == HEXLA_OP_TIMES)) return false;
    std::vector<uint32_t> f;
    double alpha = 1.0;
    flatten(n, f, alpha);
    for (uint32_t g : f)
      if (is_mat(g)) return true;
    return false;
  }
  // a matrix factor: leaf (kind 0), trans(leaf) (1), inv(leaf) (2)
  int matrix_factor(uint32_t n, int& leaf) {
    const Node& x = N(n);
    bool t = false;
    uint32_t m = n;
    while (N(m).kind == NK_UNARY && N(m).op == HEXLA_OP_TRANS) {
      t = !t;
      m = N(m).a;
    }
    if (N(m).kind == NK_LEAF) {
      leaf = leaf_index(m);
      if (leaf < 0) fail(HEXLA_E_INVALID_ARG, "batch: a leaf of the template is not listed");
      return t ? 1 : 0;
    }
    if (!t && x.kind == NK_UNARY && x.op == HEXLA_OP_INV && N(x.a).kind == NK_LEAF) {
      leaf = leaf_index(x.a);
      if (leaf < 0) fail(HEXLA_E_INVALID_ARG, "batch: a leaf of the template is not listed");
      return 2;
    }
    fail(HEXLA_E_UNSUPPORTED,
         "batch: matrix factors must be leaves, trans(leaf) or inv(leaf)");
    return 0;
  }

  int materialize(uint32_t n) {
    if (!ok()) return 0;
    const Node& x = N(n);
    if (x.kind == NK_LEAF) {
      const int l = leaf_index(n);
      if (l < 0) {
        fail(HEXLA_E_INVALID_ARG, "batch: a leaf of the template is not listed");
        return 0;
      }
      const int s = alloc();
      push_op(k::BOp{k::B_LOAD, uint8_t(s), 0, uint8_t(l), 0, 0, 0, 0, 1.0});
      return s;
    }
    if (x.kind == NK_BINARY && x.op == HEXLA_OP_SOLVE) {
      if (N(x.a).kind != NK_LEAF || !is_mat(x.a)) {
        fail(HEXLA_E_UNSUPPORTED, "batch: solve() needs a matrix leaf on the left");
        return 0;
      }
      const int l = leaf_index(x.a);
      if (l < 0) {
        fail(HEXLA_E_INVALID_ARG, "batch: a leaf of the template is not listed");
        return 0;
      }
      const int s = materialize(x.b);
      push_op(k::BOp{k::B_SOLVE, uint8_t(s), uint8_t(s), uint8_t(l), 0, 0, 0, 0, 1.0});
      c3 += 2.0 / 3.0;
      c2 += 2.0;
      return s;
    }
    if (is_chain_or_solve(n)) {
      std::vector<uint32_t> f;
      double alpha = 1.0;
      flatten(n, f, alpha);
      if (f.empty() || !is_vec(f.back())) {
        fail(HEXLA_E_UNSUPPORTED, "batch: a product must end in a t x 1 vector");
        return 0;
      }
      int s = materialize(f.back());
      for (size_t i = f.size() - 1; i-- > 0 && ok();) {
        if (!is_mat(f[i])) {
          fail(HEXLA_E_UNSUPPORTED, "batch: product factors must be t x t matrices");
          return 0;
        }
        int leaf = 0;
        const int kind = matrix_factor(f[i], leaf);
        if (!ok()) return 0;
        if (kind == 2) {
          push_op(k::BOp{k::B_SOLVE, uint8_t(s), uint8_t(s), uint8_t(leaf), 0, 0, 0, 0, 1.0});
          c3 += 2.0 / 3.0;
          c2 += 2.0;
        } else {
          const int d = alloc();
          push_op(k::BOp{k::B_GEMV, uint8_t(d), uint8_t(s), uint8_t(leaf), uint8_t(kind), 0, 0, 0,
                         alpha});
          alpha = 1.0;
          c2 += 2.0;
          release(s);
          s = d;
        }
      }
      if (alpha != 1.0) {  // only solves in the chain: scale in an element-wise pass
        std::vector<uint8_t> o{k::EW_LEAF, k::EW_SCALE}, a{uint8_t(k::kBSlotBit | s), add_const(alpha)};
        append_ew(o, a, uint8_t(s), 1);
      }
      return s;
    }
    const int s = ew_op(n, 0xfe);
    return s;
  }

  uint8_t add_const(double v) {
    for (int i = 0; i < n_cst_; ++i)
      if (p.cst[i] == v) return uint8_t(i);
    if (n_cst_ >= k::kBMaxConst) {
      fail(HEXLA_E_UNSUPPORTED, "batch: too many constants");
      return 0;
    }
    p.cst[n_cst_] = v;
    return uint8_t(n_cst_++);
  }

  void append_ew(const std::vector<uint8_t>& o, const std::vector<uint8_t>& a, uint8_t dst,
                 int arith) {
    if (!ok()) return;
    if (n_ew_ + int(o.size()) > k::kBMaxEw)
      return fail(HEXLA_E_UNSUPPORTED, "batch: element-wise program too long");
    const int b = n_ew_;
    for (size_t i = 0; i < o.size(); ++i) {
      p.ew_op[n_ew_] = o[i];
      p.ew_arg[n_ew_] = a[i];
      ++n_ew_;
    }
    push_op(k::BOp{k::B_EW, dst, 0, 0, 0, uint8_t(b), uint8_t(n_ew_), 0, 1.0});
    c1 += arith;
  }

  // Element-wise program of a vector-valued node; materialised sub-results
  // enter as slot operands. dst: kBOut (the output) or 0xfe (a new slot,
  // returned).
  int ew_op(uint32_t n, uint8_t dst) {
    std::vector<uint8_t> o, a;
    std::vector<int> held;
    int depth = 0, max_depth = 0, arith = 0;
    emit(n, o, a, held, depth, max_depth, arith);
    if (!ok()) return 0;
    if (max_depth > 4) {
      fail(HEXLA_E_UNSUPPORTED, "batch: element-wise expression needs more than 4 stack entries");
      return 0;
    }
    for (int s : held) release(s);
    int s = -1;
    if (dst != k::kBOut) {
      s = alloc();
      dst = uint8_t(s);
    }
    append_ew(o, a, dst, arith);
    return s;
  }

  int need(uint32_t n) const {
    const Node& x = N(n);
    if (x.scalar || x.kind == NK_LEAF || is_chain_or_solve(n)) return 1;
    if (x.kind == NK_UNARY) return need(x.a);
    if (x.kind == NK_BINARY) {
      if (N(x.a).scalar) return need(x.b) + (x.op == HEXLA_OP_DIV ? 1 : 0);
      if (N(x.b).scalar) return need(x.a) + (x.op == HEXLA_OP_DIV ? 1 : 0);
      const int l = need(x.a), r = need(x.b);
      return l == r ? l + 1 : std::max(l, r);
    }
    return 1;
  }

  void push(std::vector<uint8_t>& o, std::vector<uint8_t>& a, uint8_t op, uint8_t arg, int& depth,
            int& max_depth, int delta) {
    o.push_back(op);
    a.push_back(arg);
    depth += delta;
    max_depth = std::max(max_depth, depth);
  }

  void emit(uint32_t n, std::vector<uint8_t>& o, std::vector<uint8_t>& a, std::vector<int>& held,
            int& depth, int& md, int& arith) {
    if (!ok()) return;
    const Node& x = N(n);
    if (x.scalar) return push(o, a, k::EW_CONST, add_const(scalar_value(n)), depth, md, 1);
    if (!is_vec(n)) return fail(HEXLA_E_UNSUPPORTED, "batch: element-wise operands must be t x 1");
    if (x.kind == NK_LEAF) {
      const int l = leaf_index(n);
      if (l < 0) return fail(HEXLA_E_INVALID_ARG, "batch: a leaf of the template is not listed");
      return push(o, a, k::EW_LEAF, uint8_t(l), depth, md, 1);
    }
    if (is_chain_or_solve(n)) {
      const int s = materialize(n);
      held.push_back(s);
      return push(o, a, k::EW_LEAF, uint8_t(k::kBSlotBit | s), depth, md, 1);
    }
    if (x.kind == NK_UNARY) {
      if (x.op == HEXLA_OP_NEG || x.op == HEXLA_OP_EXP) {
        emit(x.a, o, a, held, depth, md, arith);
        ++arith;
        return push(o, a, x.op == HEXLA_OP_NEG ? k::EW_NEG : k::EW_EXP, 0, depth, md, 0);
      }
      return fail(HEXLA_E_UNSUPPORTED, "batch: trans/inv of a vector expression");
    }
    if (x.kind != NK_BINARY) return fail(HEXLA_E_UNSUPPORTED, "batch: unknown node");
    const bool sa = N(x.a).scalar, sb = N(x.b).scalar;
    const int op = x.op;
    if (op == HEXLA_OP_SOLVE) return fail(HEXLA_E_UNSUPPORTED, "batch: solve form");
    if (sa || sb) {
      const uint32_t v = sa ? x.b : x.a;
      const double c = scalar_value(sa ? x.a : x.b);
      emit(v, o, a, held, depth, md, arith);
      ++arith;
      switch (op) {
        case HEXLA_OP_TIMES:
        case HEXLA_OP_SCHUR: return push(o, a, k::EW_SCALE, add_const(c), depth, md, 0);
        case HEXLA_OP_PLUS: return push(o, a, k::EW_ADDC, add_const(c), depth, md, 0);
        case HEXLA_OP_MINUS:
          if (sb) return push(o, a, k::EW_ADDC, add_const(-c), depth, md, 0);
          push(o, a, k::EW_NEG, 0, depth, md, 0);
          return push(o, a, k::EW_ADDC, add_const(c), depth, md, 0);
        case HEXLA_OP_DIV:
          push(o, a, k::EW_CONST, add_const(c), depth, md, 1);
          return push(o, a, sb ? k::EW_DIV : k::EW_RDIV, 0, depth, md, -1);
        default: return fail(HEXLA_E_UNSUPPORTED, "batch: operator");
      }
    }
    uint8_t code;
    switch (op) {
      case HEXLA_OP_PLUS: code = k::EW_ADD; break;
      case HEXLA_OP_MINUS: code = k::EW_SUB; break;
      case HEXLA_OP_SCHUR: code = k::EW_MUL; break;
      case HEXLA_OP_DIV: code = k::EW_DIV; break;
      default: return fail(HEXLA_E_UNSUPPORTED, "batch: operator");
    }
    const bool swap = need(x.b) > need(x.a);  // deeper operand first (Sethi-Ullman)
    emit(swap ? x.b : x.a, o, a, held, depth, md, arith);
    emit(swap ? x.a : x.b, o, a, held, depth, md, arith);
    if (swap && code == k::EW_SUB) code = k::EW_RSUB;
    if (swap && code == k::EW_DIV) code = k::EW_RDIV;
    ++arith;
    push(o, a, code, 0, depth, md, -1);
  }
};

hexla_status upload_table(hexla_batch* b, void* ws, hipStream_t s) {
  const hipError_t e = hipMemcpyAsync(static_cast<char*>(ws) + kQueueBytes, b->table,
                                      b->table_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return set_err(b->ctx, HEXLA_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
  return HEXLA_OK;
}

hipError_t launch(hexla_batch* b, const k::BatchConfig& cfg, void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  char* tab = base + kQueueBytes;
  void* scratch = b->has_solve ? base + kQueueBytes + align256(b->table_bytes) : nullptr;
  return k::batch_launch(b->dtype, cfg, reinterpret_cast<const k::BProgram*>(tab),
                         reinterpret_cast<const k::BInst*>(tab + b->off_inst),
                         reinterpret_cast<const int32_t*>(tab + b->off_order), b->count,
                         reinterpret_cast<unsigned*>(base), scratch, b->stride, b->ctx->d_status,
                         s);
}

hexla_status check_ws(hexla_batch* b, void* ws, size_t bytes) {
  if (!b || !b->ctx) return HEXLA_E_INVALID_ARG;
  if (b->ctx->device < 0) return set_err(b->ctx, HEXLA_E_UNSUPPORTED, "batch: dry-run context");
  if (!ws || bytes < b->ws_bytes || (reinterpret_cast<uintptr_t>(ws) & 255))
    return set_err(b->ctx, HEXLA_E_INVALID_ARG,
                   "batch: workspace must be 256-byte aligned and hold " +
                       std::to_string(b->ws_bytes) + " bytes");
  if (enter_device(b->ctx->device) != hipSuccess)
    return set_err(b->ctx, HEXLA_E_DEVICE, "batch: hipSetDevice");
  return HEXLA_OK;
}

// A captured graph holds the configuration it was captured with.
void drop_graph(hexla_batch* b) {
  if (!b->graph_exec) return;
  (void)hipGraphExecDestroy(b->graph_exec);
  (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

void detach_batch(hexla_batch* b) { b->ctx = nullptr; }

}  // namespace hexla

using namespace hexla;

extern "C" {

hexla_status hexla_batch_create(hexla_ctx* ctx, hexla_node root, const hexla_node* leaves,
                                int32_t n_leaves, int64_t count, const int64_t* sizes,
                                const void* const* leaf_ptrs, const int64_t* lds,
                                void* const* outs, const hexla_plan_opts* opts,
                                hexla_batch** out) {
  (void)opts;
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  *out = nullptr;
  if (root >= ctx->nodes.size()) return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: bad root");
  if (n_leaves < 1 || n_leaves > k::kBMaxLeaf || !leaves)
    return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: 1 to 8 template leaves");
  if (count < 0 || count > INT32_MAX || (count > 0 && (!sizes || !leaf_ptrs || !outs)))
    return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: bad instance arrays");
  const Node& r = ctx->nodes[root];
  const int64_t t = r.rows;
  if (r.scalar || r.cols != 1 || t < 2)
    return set_err(ctx, HEXLA_E_DIM, "batch: the template result must be t x 1 with t >= 2");
  std::vector<uint32_t> lv(leaves, leaves + n_leaves);
  int dtype = -1;
  for (int l = 0; l < n_leaves; ++l) {
    if (lv[l] >= ctx->nodes.size() || ctx->nodes[lv[l]].kind != NK_LEAF)
      return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: template leaf " + std::to_string(l));
    const Node& x = ctx->nodes[lv[l]];
    if (x.rows != t || (x.cols != t && x.cols != 1))
      return set_err(ctx, HEXLA_E_DIM, "batch: template leaves must be t x t or t x 1");
    if (dtype >= 0 && x.dtype != dtype)
      return set_err(ctx, HEXLA_E_DTYPE, "batch: leaves have different storage types");
    dtype = x.dtype;
    for (int m = 0; m < l; ++m)
      if (lv[m] == lv[l]) return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: leaf listed twice");
  }
  BatchCompiler bc(ctx, lv, t);
  bc.compile(root);
  if (bc.st != HEXLA_OK) return set_err(ctx, bc.st, bc.err);

  auto b = std::make_unique<hexla_batch>();
  b->ctx = ctx;
  b->dtype = dtype;
  b->count = count;
  b->prog = bc.p;
  b->ops_json = bc.js.str();
  for (int o = 0; o < bc.p.n_ops; ++o) b->has_solve |= bc.p.ops[o].kind == k::B_SOLVE;
  const size_t es = dtype_size(dtype);

  // instances: validation, costs, overlap check
  std::vector<k::BInst> inst(static_cast<size_t>(count));
  std::vector<double> cost(static_cast<size_t>(count));
  struct Iv {
    uintptr_t lo, hi;
    bool out;
  };
  std::vector<Iv> iv;
  iv.reserve(size_t(count) * (n_leaves + 1));
  std::vector<bool> used_leaf(n_leaves, false);
  for (int o = 0; o < bc.p.n_ops; ++o)
    if (bc.p.ops[o].kind != k::B_EW) used_leaf[bc.p.ops[o].leaf] = true;
  for (int i = 0; i < bc.p.n_ops; ++i)
    if (bc.p.ops[i].kind == k::B_EW)
      for (int pc = bc.p.ops[i].ew_begin; pc < bc.p.ops[i].ew_end; ++pc) {
        const uint8_t op = bc.p.ew_op[pc], a = bc.p.ew_arg[pc];
        if ((op == k::EW_LEAF || op == k::EW_LEAFMUL || op == k::EW_LEAFADD) &&
            !(a & k::kBSlotBit))
          used_leaf[a] = true;
      }
  double flops = 0, bytes = 0;
  int64_t max_n = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t n = sizes[i];
    if (n < 0) return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: negative size");
    if (n > k::kBMaxN)
      return set_err(ctx, HEXLA_E_UNSUPPORTED,
                     "batch: instance " + std::to_string(i) + " has n > " +
                         std::to_string(k::kBMaxN));
    max_n = std::max(max_n, n);
    k::BInst& I = inst[size_t(i)];
    std::memset(&I, 0, sizeof(I));
    I.n = n;
    I.out = outs[i];
    if (n > 0 && !I.out)
      return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: null output " + std::to_string(i));
    for (int l = 0; l < n_leaves; ++l) {
      const void* ptr = leaf_ptrs[i * n_leaves + l];
      const int64_t ld = lds ? lds[i * n_leaves + l] : std::max<int64_t>(n, 1);
      I.leaf[l] = ptr;
      I.ld[l] = ld;
      if (n == 0 || !used_leaf[l]) continue;
      if (!ptr)
        return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: null leaf pointer, instance " +
                                                     std::to_string(i));
      if (ld < n)
        return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: ld < n, instance " + std::to_string(i));
      const bool mat = bc.leaf_is_matrix[l];
      const uint64_t span = mat ? uint64_t((n - 1) * ld + n) * es : uint64_t(n) * es;
      if (span >= (uint64_t(1) << 31))  // the kernel addresses an instance with 32-bit offsets
        return set_err(ctx, HEXLA_E_UNSUPPORTED,
                       "batch: an instance matrix spans 2^31 bytes or more, instance " +
                           std::to_string(i));
      const uintptr_t lo = reinterpret_cast<uintptr_t>(ptr);
      iv.push_back({lo, lo + span, false});
      bytes += double(mat ? n * n : n) * double(es);
    }
    if (n > 0) {
      const uintptr_t lo = reinterpret_cast<uintptr_t>(I.out);
      iv.push_back({lo, lo + uint64_t(n) * es, true});
      bytes += double(n) * double(es);
    }
    const double dn = double(n);
    const double f = bc.c3 * dn * dn * dn + bc.c2 * dn * dn + bc.c1 * dn;
    flops += f;
    cost[size_t(i)] = b->has_solve ? dn * dn * dn + 8.0 * dn * dn : dn * dn;
  }
  std::sort(iv.begin(), iv.end(), [](const Iv& x, const Iv& y) { return x.lo < y.lo; });
  uintptr_t all_end = 0, out_end = 0;
  for (const Iv& x : iv) {
    if ((x.out && x.lo < all_end) || (!x.out && x.lo < out_end))
      return set_err(ctx, HEXLA_E_INVALID_ARG, "batch: an output overlaps another buffer");
    all_end = std::max(all_end, x.hi);
    if (x.out) out_end = std::max(out_end, x.hi);
  }
  std::vector<int32_t> order(static_cast<size_t>(count));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return cost[size_t(x)] > cost[size_t(y)]; });

  b->max_n = max_n;
  b->flops = flops;
  b->bytes = bytes;
  b->cfg = k::batch_default(dtype, count);
  b->max_grid = kGrids[sizeof(kGrids) / sizeof(kGrids[0]) - 1];
  b->stride = b->has_solve ? k::batch_scratch_stride(max_n) : 0;
  b->off_order = align256(sizeof(k::BProgram));
  b->off_inst = b->off_order + align256(size_t(count) * sizeof(int32_t));
  b->table_bytes = b->off_inst + size_t(count) * sizeof(k::BInst);
  b->ws_bytes = kQueueBytes + align256(b->table_bytes) +
                uint64_t(b->max_grid) * uint64_t(b->stride) * es;
  if (ctx->device >= 0) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipHostMalloc(&b->table, b->table_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      b->table = nullptr;
      return set_err(ctx, HEXLA_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
    }
    char* tab = static_cast<char*>(b->table);
    std::memcpy(tab, &b->prog, sizeof(k::BProgram));
    std::memcpy(tab + b->off_order, order.data(), order.size() * sizeof(int32_t));
    std::memcpy(tab + b->off_inst, inst.data(), inst.size() * sizeof(k::BInst));
  }
  ctx->batches.insert(b.get());
  *out = b.release();
  return HEXLA_OK;
}

hexla_status hexla_batch_get_info(const hexla_batch* b, hexla_batch_info* out) {
  if (!b || !b->ctx || !out) return HEXLA_E_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->count = b->count;
  out->max_n = b->max_n;
  out->dtype = b->dtype;
  out->n_ops = b->prog.n_ops;
  int panel = 0, threads = 0;
  k::batch_variant_shape(b->dtype, b->cfg.variant, &panel, &threads);
  out->panel = panel;
  out->threads = threads;
  out->grid = b->cfg.grid;
  out->workspace_bytes = b->ws_bytes;
  out->flops = b->flops;
  out->bytes = b->bytes;
  return HEXLA_OK;
}

hexla_status hexla_batch_describe(const hexla_batch* b, char* buf, size_t cap, size_t* needed) {
  if (!b || !b->ctx) return HEXLA_E_INVALID_ARG;
  int panel = 0, threads = 0;
  k::batch_variant_shape(b->dtype, b->cfg.variant, &panel, &threads);
  std::ostringstream js;
  js.precision(17);
  js << "{\"count\":" << b->count << ",\"max_n\":" << b->max_n << ",\"dtype\":\""
     << (b->dtype == HEXLA_F64 ? "f64" : "f32") << "\",\"ops\":[" << b->ops_json
     << "],\"out_slot\":" << (b->prog.out_slot == k::kBOut ? -1 : b->prog.out_slot)
     << ",\"panel\":" << panel << ",\"threads\":" << threads << ",\"grid\":" << b->cfg.grid
     << ",\"flops\":" << b->flops << ",\"bytes\":" << b->bytes
     << ",\"workspace_bytes\":" << b->ws_bytes << "}";
  const std::string s = js.str();
  if (needed) *needed = s.size();
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = '\0';
  }
  return HEXLA_OK;
}

hexla_status hexla_batch_execute(hexla_batch* b, void* ws, size_t bytes) {
  hexla_status st = check_ws(b, ws, bytes);
  if (st != HEXLA_OK) return st;
  st = upload_table(b, ws, b->ctx->stream);
  if (st != HEXLA_OK) return st;
  const hipError_t e = launch(b, b->cfg, ws, b->ctx->stream);
  if (e != hipSuccess)
    return set_err(b->ctx, HEXLA_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
  return HEXLA_OK;
}

hexla_status hexla_batch_autotune(hexla_batch* b, void* ws, size_t bytes, int32_t reps) {
  hexla_status st = check_ws(b, ws, bytes);
  if (st != HEXLA_OK) return st;
  if (reps <= 0) reps = 3;
  hipStream_t s = b->ctx->stream;
  st = upload_table(b, ws, s);
  if (st != HEXLA_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best_ms = 1e30f;
  k::BatchConfig best = b->cfg;
  for (int v = 0; v < k::batch_variant_count(b->dtype) && e == hipSuccess; ++v)
    for (int g : kGrids) {
      if (g > b->max_grid) continue;
      const k::BatchConfig c{v, g};
      e = launch(b, c, ws, s);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(b, c, ws, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess)
    return set_err(b->ctx, HEXLA_E_DEVICE, std::string("batch autotune: ") + hipGetErrorString(e));
  b->cfg = best;
  drop_graph(b);
  return HEXLA_OK;
}

hexla_status hexla_batch_set_config(hexla_batch* b, int32_t panel, int32_t threads, int32_t grid) {
  if (!b || !b->ctx) return HEXLA_E_INVALID_ARG;
  if (grid < 1 || grid > b->max_grid)
    return set_err(b->ctx, HEXLA_E_INVALID_ARG, "batch config: grid out of range");
  for (int v = 0; v < k::batch_variant_count(b->dtype); ++v) {
    int p = 0, t = 0;
    k::batch_variant_shape(b->dtype, v, &p, &t);
    if (p == panel && t == threads) {
      b->cfg = k::BatchConfig{v, grid};
      drop_graph(b);
      return HEXLA_OK;
    }
  }
  return set_err(b->ctx, HEXLA_E_INVALID_ARG, "batch config: no variant with this panel and threads");
}

hexla_status hexla_batch_capture(hexla_batch* b, void* ws, size_t bytes) {
  hexla_status st = check_ws(b, ws, bytes);
  if (st != HEXLA_OK) return st;
  st = upload_table(b, ws, b->ctx->stream);
  if (st != HEXLA_OK) return st;
  hipError_t e = hipStreamSynchronize(b->ctx->stream);
  hipStream_t cs = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    if (cs) (void)hipStreamDestroy(cs);
    return set_err(b->ctx, HEXLA_E_DEVICE, std::string("batch capture: ") + hipGetErrorString(e));
  }
  const hipError_t le = launch(b, b->cfg, ws, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (le != hipSuccess) e = le;
  hipGraphExec_t x = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return set_err(b->ctx, HEXLA_E_DEVICE, std::string("batch capture: ") + hipGetErrorString(e));
  }
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph = g;
  b->graph_exec = x;
  return HEXLA_OK;
}

hexla_status hexla_batch_replay(hexla_batch* b) {
  if (!b || !b->ctx) return HEXLA_E_INVALID_ARG;
  if (!b->graph_exec) return set_err(b->ctx, HEXLA_E_INVALID_ARG, "batch replay: nothing captured");
  hipError_t e = enter_device(b->ctx->device);
  if (e == hipSuccess) e = hipGraphLaunch(b->graph_exec, b->ctx->stream);
  if (e != hipSuccess)
    return set_err(b->ctx, HEXLA_E_DEVICE, std::string("batch replay: ") + hipGetErrorString(e));
  return HEXLA_OK;
}

hexla_status hexla_batch_destroy(hexla_batch* b) {
  if (!b) return HEXLA_E_INVALID_ARG;
  if (b->ctx) {
    b->ctx->batches.erase(b);
    if (b->ctx->device >= 0) (void)hipSetDevice(b->ctx->device);
  }
  delete b;
  return HEXLA_OK;
}

}  // extern "C"
