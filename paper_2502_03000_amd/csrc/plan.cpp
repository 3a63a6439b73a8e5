// Planner: turns the delayed expression into a list of kernel launches.
//
// The rewrites are the paper's (Sec. II):
//   * element-wise subtrees of any length become one fused program (no
//     temporaries), and when such a program consumes a matrix-vector product
//     it runs as that product's epilogue;
//   * inv(S) * Y becomes an LU solve with Y as right-hand side (xGESV);
//   * a product of a matrix with its own transpose (same storage) becomes a
//     symmetric rank-k update computing one triangle (xSYRK);
//   * scalars fold into the product's alpha or the element-wise program, and
//     transposes fold into kernel flags;
//   * matrix chains are bracketed by exact dynamic programming over
//     multiply-add counts (default), by the paper's rule "multiply the
//     adjacent pair with the smallest result first" (leftmost on ties), or
//     left to right (the "naive" evaluation of Sec. III, which also disables
//     the other rewrites).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace hexla {

namespace {

typedef __int128 i128;

bool is_ew_binary(int op) {
  return op == HEXLA_OP_PLUS || op == HEXLA_OP_MINUS || op == HEXLA_OP_SCHUR || op == HEXLA_OP_DIV;
}

struct Factor {
  int kind = 0;  // 0 view, 1 inverse marker (node = S), 2 expression to materialize,
                 // 3 diagonal matrix (node = diagmat's argument)
  uint32_t node = 0;
  bool trans = false;
  View v;
};

// Element-wise tree node.
struct ENode {
  int kind = 0;  // 0 op, 1 view, 2 const, 3 pending (product/solve/inverse), 4 extra,
                 // 5 identity matrix
  int op = 0;    // k::EwOp of an op node (binary or NEG/EXP)
  int a = -1, b = -1;
  View v;
  double c = 0.0;
  uint32_t node = 0;
  bool trans = false;
  bool diag = false;  // pending: its main diagonal (a column vector) is wanted
  int64_t rows = 0, cols = 0;
};

struct TNode {  // chain bracketing tree
  int leaf = -1, left = -1, right = -1;
  int lo = 0, hi = 0;
};

const char* planner_name(int p) {
  switch (p) {
    case HEXLA_PLANNER_GREEDY: return "greedy";
    case HEXLA_PLANNER_NAIVE: return "naive";
    case HEXLA_PLANNER_LEARNED: return "learned";
    case HEXLA_PLANNER_ROOFLINE: return "roofline";
    default: return "dp";
  }
}

bool same_storage(const View& a, const View& b) {
  return a.is_leaf && b.is_leaf && a.leaf_ptr == b.leaf_ptr && a.ld == b.ld &&
         (a.trans ? a.cols : a.rows) == (b.trans ? b.cols : b.rows) &&
         (a.trans ? a.rows : a.cols) == (b.trans ? b.rows : b.cols);
}

View transposed(const View& v) {
  View t = v;
  std::swap(t.rows, t.cols);
  if (v.strided) std::swap(t.str_i, t.str_j);
  else t.trans = !v.trans;
  return t;
}

// Element strides of a view whose leading dimension is known (leaves and
// temporaries; the output's is bound only at execute time).
int64_t vsi(const View& v) { return v.strided ? v.str_i : (v.trans ? v.ld : 1); }
int64_t vsj(const View& v) { return v.strided ? v.str_j : (v.trans ? 1 : v.ld); }
int64_t extent(const View& v) {
  if (v.strided) return v.span;
  const int64_t rs = v.trans ? v.cols : v.rows, cs = v.trans ? v.rows : v.cols;
  return rs * cs > 0 ? (cs - 1) * v.ld + rs : 0;
}

// The main diagonal of v as a min(rows, cols) x 1 strided view.
View diag_view(const View& v) {
  View d = v;
  d.strided = true;
  d.str_i = vsi(v) + vsj(v);
  d.str_j = 0;
  d.span = extent(v);
  d.rows = std::min(v.rows, v.cols);
  d.cols = 1;
  d.trans = false;
  return d;
}

// A column vector v (n x 1, strided or not) repeated across `cols` columns.
View bcast_cols(const View& v, int64_t cols) {
  View b = v;
  b.strided = true;
  b.str_i = vsi(v);
  b.str_j = 0;
  b.span = extent(v);
  b.cols = cols;
  b.trans = false;
  return b;
}

// The same column vector repeated down `rows` rows as a rows x n matrix
// (element (i, j) = v_j).
View bcast_rows(const View& v, int64_t rows) {
  View b = v;
  b.strided = true;
  b.str_i = 0;
  b.str_j = vsi(v);
  b.span = extent(v);
  b.cols = v.rows;
  b.rows = rows;
  b.trans = false;
  return b;
}

// Rows [r0, r0 + rows) and columns [c0, c0 + cols) of v, in place.
View sub_view(const View& v, int64_t r0, int64_t c0, int64_t rows, int64_t cols, size_t esz) {
  View s = v;
  const int64_t off = r0 * vsi(v) + c0 * vsj(v);
  if (s.ref.buf == Buf::Leaf) {
    s.ref.ptr = static_cast<const char*>(v.ref.ptr) + off * int64_t(esz);
    s.leaf_ptr = s.ref.ptr;
  } else {
    s.ref.off = v.ref.off + off * int64_t(esz);
  }
  s.rows = rows;
  s.cols = cols;
  if (v.strided) s.span = std::max<int64_t>(0, v.span - off);
  return s;
}

class Planner {
 public:
  Planner(hexla_ctx* ctx, const hexla_plan_opts& o, hexla_plan* plan)
      : ctx_(ctx), o_(o), plan_(plan) {}

  hexla_status run(hexla_node root) {
    const Node& r = N(root);
    if (r.scalar) return fail(HEXLA_E_UNSUPPORTED, "the expression is a scalar");
    dtype_ = r.dtype;
    esz_ = dtype_size(dtype_);
    plan_->rows = r.rows;
    plan_->cols = r.cols;
    plan_->dtype = dtype_;
    View out;
    out.ref.buf = Buf::Out;
    out.rows = r.rows;
    out.cols = r.cols;
    out.ld = -1;
    materialize(root, false, &out);
    if (status_ != HEXLA_OK) return status_;
    plan_->ws_bytes = uint64_t(top_);
    double fl = 0, by = 0;
    for (const Step& s : steps_) {
      fl += s.flops;
      by += s.bytes;
    }
    plan_->flops = fl;
    plan_->bytes = by;
    plan_->macs = macs_;
    plan_->learned_notes = learned_notes_;
    plan_->steps = std::move(steps_);
    return HEXLA_OK;
  }

 private:
  hexla_ctx* ctx_;
  hexla_plan_opts o_;
  hexla_plan* plan_;
  int dtype_ = 0;
  size_t esz_ = 8;
  int64_t top_ = 0;
  double macs_ = 0;
  std::vector<Step> steps_;
  std::vector<ENode> E_;
  std::map<std::string, k::GemmConfig> learned_cfg_;  // predicted-fastest configurations
  std::vector<std::string> learned_notes_;           // the learned planner's decisions
  hexla_status status_ = HEXLA_OK;
  bool diag_mode_ = false;  // build_ew builds the diagonal of its node

  const Node& N(uint32_t i) const { return ctx_->nodes[i]; }

  hexla_status fail(hexla_status st, const std::string& msg) {
    if (status_ == HEXLA_OK) {
      status_ = st;
      set_err(ctx_, st, msg);
    }
    return st;
  }

  Ref work(int64_t bytes) {
    Ref r;
    r.buf = Buf::Work;
    top_ = (top_ + 255) & ~int64_t(255);
    r.off = top_;
    top_ += std::max<int64_t>(bytes, 1);
    return r;
  }

  View temp(int64_t rows, int64_t cols) {
    View v;
    v.ref = work(rows * cols * int64_t(esz_));
    v.rows = rows;
    v.cols = cols;
    v.ld = std::max<int64_t>(rows, 1);
    return v;
  }

  View leaf_view(uint32_t n, bool t) const {
    const Node& x = N(n);
    View v;
    v.ref.buf = Buf::Leaf;
    v.ref.ptr = x.ptr;
    v.rows = t ? x.cols : x.rows;
    v.cols = t ? x.rows : x.cols;
    v.ld = x.ld;
    v.trans = t;
    v.is_leaf = true;
    v.leaf_ptr = x.ptr;
    return v;
  }

  static bool same_view(const View& a, const View& b) {
    return a.ref.buf == b.ref.buf && a.ref.off == b.ref.off && a.ref.ptr == b.ref.ptr &&
           a.rows == b.rows && a.cols == b.cols && a.ld == b.ld && a.trans == b.trans &&
           a.strided == b.strided && a.str_i == b.str_i && a.str_j == b.str_j;
  }

  // A view products and solves can read: strided views (diagonals,
  // broadcasts) are copied into a temporary first.
  View dense(const View& v) {
    if (!v.strided || status_ != HEXLA_OK) return v;
    return emit_ew(add_view(v), nullptr, v.rows, v.cols, true);
  }

  // ------------------------------------------------------------- scalars
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
      default: return a * b;  // TIMES, SCHUR
    }
  }

  // ------------------------------------------------------------ products
  void flatten(uint32_t n, bool t, std::vector<Factor>& out, double& alpha) const {
    const Node& x = N(n);
    if (x.scalar) {
      alpha *= scalar_value(n);
      return;
    }
    if (x.kind == NK_BINARY && x.op == HEXLA_OP_TIMES) {
      if (t) {
        flatten(x.b, t, out, alpha);
        flatten(x.a, t, out, alpha);
      } else {
        flatten(x.a, t, out, alpha);
        flatten(x.b, t, out, alpha);
      }
      return;
    }
    Factor f;
    f.trans = t;
    if (x.kind == NK_UNARY && x.op == HEXLA_OP_TRANS) {
      flatten(x.a, !t, out, alpha);
      return;
    }
    if (x.kind == NK_UNARY && x.op == HEXLA_OP_INV) {
      f.kind = 1;
      f.node = x.a;
      out.push_back(f);
      return;
    }
    if (x.kind == NK_UNARY && x.op == HEXLA_OP_DIAGMAT) {
      f.kind = 3;
      f.node = x.a;
      f.v.rows = t ? x.cols : x.rows;
      f.v.cols = t ? x.rows : x.cols;
      out.push_back(f);
      return;
    }
    if (x.kind == NK_LEAF) {
      f.kind = 0;
      f.node = n;
      f.v = leaf_view(n, t);
      out.push_back(f);
      return;
    }
    f.kind = 2;
    f.node = n;
    out.push_back(f);
  }

  // A product node that is a real chain (two or more matrix factors, or an
  // inverse marker), as opposed to a scaled matrix.
  bool is_chain(uint32_t n) const {
    std::vector<Factor> f;
    double alpha = 1.0;
    flatten(n, false, f, alpha);
    if (f.size() >= 2) return true;
    return f.size() == 1 && (f[0].kind == 1 || f[0].kind == 3);
  }

  // The final product of this chain is a matrix-vector product.
  bool gemv_final(uint32_t n, bool t) const {
    const Node& x = N(n);
    if (x.kind != NK_BINARY || x.op != HEXLA_OP_TIMES) return false;
    std::vector<Factor> f;
    double alpha = 1.0;
    flatten(n, t, f, alpha);
    if (f.size() < 2) return false;
    for (const Factor& q : f)
      if (q.kind == 1 || q.kind == 3) return false;
    const int64_t rows = t ? x.cols : x.rows, cols = t ? x.rows : x.cols;
    return rows == 1 || cols == 1;
  }

  // ------------------------------------------------------ materialization
  // Evaluates node (transposed when t) into dest, or into a new temporary
  // (or returns a borrowed view) when dest is null.
  View materialize(uint32_t n, bool t, const View* dest) {
    if (status_ != HEXLA_OK) return View{};
    const Node& x = N(n);
    if (x.scalar) {
      fail(HEXLA_E_UNSUPPORTED, "scalar used where a matrix is required");
      return View{};
    }
    switch (x.kind) {
      case NK_LEAF: {
        View v = leaf_view(n, t);
        if (!dest) return v;
        return emit_ew(add_view(v), dest, v.rows, v.cols);
      }
      case NK_UNARY:
        if (x.op == HEXLA_OP_TRANS) return materialize(x.a, !t, dest);
        if (x.op == HEXLA_OP_INV) {
          View s = dense(materialize(x.a, t, nullptr));
          return explicit_inverse(s, dest);
        }
        if (x.op == HEXLA_OP_SUBMAT) {
          // a view of the operand's storage (a leaf, or its evaluated value)
          View base = materialize(x.a, false, nullptr);
          if (status_ != HEXLA_OK) return View{};
          View sv = sub_view(base, x.r0, x.c0, x.rows, x.cols, esz_);
          if (t) sv = transposed(sv);
          if (!dest) return sv;
          return emit_ew(add_view(sv), dest, sv.rows, sv.cols);
        }
        if (x.op == HEXLA_OP_DIAG) {
          View d = diag_value(x.a, t ? nullptr : dest);
          if (!t) return d;
          View dt = transposed(d);
          if (!dest) return dt;
          return emit_ew(add_view(dt), dest, dt.rows, dt.cols);
        }
        if (x.op == HEXLA_OP_TRACE) return trace_value(x.a, dest);
        if (x.op == HEXLA_OP_DIAGMAT) return diagmat_value(x.a, t, dest);
        return emit_ew(build_ew(n, t), dest, t ? x.cols : x.rows, t ? x.rows : x.cols);
      default:
        break;
    }
    if (x.op == HEXLA_OP_TIMES) {
      if (is_chain(n)) return lower_chain(n, t, dest, nullptr);
      return emit_ew(build_ew(n, t), dest, t ? x.cols : x.rows, t ? x.rows : x.cols);
    }
    if (is_ew_binary(x.op))
      return emit_ew(build_ew(n, t), dest, t ? x.cols : x.rows, t ? x.rows : x.cols);
    if (x.op == HEXLA_OP_SOLVE) {
      const bool spd = gram_product(x.a);
      View s = dense(materialize(x.a, false, nullptr));
      View b = dense(materialize(x.b, false, nullptr));
      if (!t) {
        View xo = dest ? *dest : temp(s.cols, b.cols);
        solve(s, b, xo, spd);
        return xo;
      }
      View xo = temp(s.cols, b.cols);
      solve(s, b, xo, spd);
      View tv = transposed(xo);
      if (!dest) return tv;
      return emit_ew(add_view(tv), dest, tv.rows, tv.cols);
    }
    fail(HEXLA_E_UNSUPPORTED, "unknown operation");
    return View{};
  }

  // ------------------------------------------------------------- element-wise
  int add_node(const ENode& e) {
    E_.push_back(e);
    return int(E_.size()) - 1;
  }
  int add_view(const View& v) {
    ENode e;
    e.kind = 1;
    e.v = v;
    e.rows = v.rows;
    e.cols = v.cols;
    return add_node(e);
  }
  int add_const(double c) {
    ENode e;
    e.kind = 2;
    e.c = c;
    return add_node(e);
  }
  int add_op(int op, int a, int b, int64_t rows, int64_t cols) {
    ENode e;
    e.kind = 0;
    e.op = op;
    e.a = a;
    e.b = b;
    e.rows = rows;
    e.cols = cols;
    return add_node(e);
  }

  int add_ident(int64_t rows, int64_t cols) {
    ENode e;
    e.kind = 5;
    e.rows = rows;
    e.cols = cols;
    return add_node(e);
  }

  // Element-wise tree of node n (transposed when t). In diagonal mode
  // (diag_mode_) the tree computes the main diagonal of n's value as a
  // column vector: element-wise operations commute with taking the
  // diagonal, so every operand is replaced by its diagonal.
  int build_ew(uint32_t n, bool t) {
    const Node& x = N(n);
    if (x.scalar) return add_const(scalar_value(n));
    int64_t rows = t ? x.cols : x.rows, cols = t ? x.rows : x.cols;
    if (diag_mode_) {
      rows = std::min(rows, cols);
      cols = 1;
    }
    if (x.kind == NK_LEAF) {
      const View v = leaf_view(n, t);
      return add_view(diag_mode_ ? diag_view(v) : v);
    }
    auto pending = [&]() {
      ENode e;
      e.kind = 3;
      e.node = n;
      e.trans = t;
      e.diag = diag_mode_;
      e.rows = rows;
      e.cols = cols;
      return add_node(e);
    };
    if (x.kind == NK_UNARY) {
      switch (x.op) {
        case HEXLA_OP_TRANS: return build_ew(x.a, !t);
        case HEXLA_OP_NEG: return add_op(k::EW_NEG, build_ew(x.a, t), -1, rows, cols);
        case HEXLA_OP_EXP: return add_op(k::EW_EXP, build_ew(x.a, t), -1, rows, cols);
        case HEXLA_OP_DIAG:
          if (t || diag_mode_) return pending();
          return with_diag(x.a);
        case HEXLA_OP_DIAGMAT: return diagmat_ew(n, t);
        default: return pending();
      }
    }
    switch (x.op) {
      case HEXLA_OP_PLUS: return add_op(k::EW_ADD, build_ew(x.a, t), build_ew(x.b, t), rows, cols);
      case HEXLA_OP_MINUS: return add_op(k::EW_SUB, build_ew(x.a, t), build_ew(x.b, t), rows, cols);
      case HEXLA_OP_SCHUR: return add_op(k::EW_MUL, build_ew(x.a, t), build_ew(x.b, t), rows, cols);
      case HEXLA_OP_DIV: return add_op(k::EW_DIV, build_ew(x.a, t), build_ew(x.b, t), rows, cols);
      case HEXLA_OP_TIMES: {
        if (is_chain(n)) return pending();
        std::vector<Factor> f;
        double alpha = 1.0;
        flatten(n, t, f, alpha);
        const int inner = f[0].kind == 0 ? add_view(diag_mode_ ? diag_view(f[0].v) : f[0].v)
                                         : build_ew(f[0].node, f[0].trans);
        if (alpha == 1.0) return inner;
        return add_op(k::EW_MUL, inner, add_const(alpha), rows, cols);
      }
      default:
        return pending();
    }
  }

  // The diagonal of node a as an element-wise tree (a column vector).
  int with_diag(uint32_t a) {
    const bool prev = diag_mode_;
    diag_mode_ = true;
    const int r = build_ew(a, false);
    diag_mode_ = prev;
    return r;
  }
  int without_diag(uint32_t a, bool t) {
    const bool prev = diag_mode_;
    diag_mode_ = false;
    const int r = build_ew(a, t);
    diag_mode_ = prev;
    return r;
  }

  static bool is_vector(const Node& y) { return !y.scalar && (y.rows == 1 || y.cols == 1); }

  // diagmat(z) inside an element-wise tree: the identity's mask times the
  // broadcast diagonal values (a vector argument) or times the matrix.
  int diagmat_ew(uint32_t n, bool t) {
    const Node& x = N(n);
    const Node& z = N(x.a);
    if (diag_mode_) {  // diag(diagmat(v)) = v, diag(diagmat(M)) = diag(M)
      if (is_vector(z)) return without_diag(x.a, z.rows == 1 && z.cols != 1);
      return build_ew(x.a, t);
    }
    const int64_t rows = t ? x.cols : x.rows, cols = t ? x.rows : x.cols;
    if (is_vector(z)) {
      const View dv = diag_vector(x.a);
      return add_op(k::EW_MUL, add_ident(rows, cols), add_view(bcast_cols(dv, cols)), rows, cols);
    }
    return add_op(k::EW_MUL, add_ident(rows, cols), build_ew(x.a, t), rows, cols);
  }

  void collect(int e, int kind, std::vector<int>& out) const {
    if (e < 0) return;
    if (E_[e].kind == kind) out.push_back(e);
    if (E_[e].kind == 0) {
      collect(E_[e].a, kind, out);
      collect(E_[e].b, kind, out);
    }
  }

  View out_or_temp(const View* dest, int64_t rows, int64_t cols) {
    return dest ? *dest : temp(rows, cols);
  }

  // The value of a pending subtree (its diagonal when marked so).
  View pending_value(int p) {
    const ENode& e = E_[p];
    if (!e.diag) return materialize(e.node, e.trans, nullptr);
    return diag_value(e.node, nullptr);
  }

  // A column read with a stride and repeated across many columns (the
  // diagonal of a matrix in diagmat(A) * B, a row vector scaling columns)
  // would be gathered again for every column, one cache line per element;
  // on large passes it is first copied into a contiguous column.
  void gather_broadcasts(int e) {
    if (e < 0 || status_ != HEXLA_OK) return;
    if (E_[e].kind == 0) {
      gather_broadcasts(E_[e].a);
      gather_broadcasts(E_[e].b);
      return;
    }
    if (E_[e].kind != 1) return;
    const View v = E_[e].v;
    if (!v.strided || v.str_j != 0 || v.str_i == 1 || v.str_i == 0 || v.cols < 8 || v.rows < 64 ||
        v.rows * v.cols < (int64_t(1) << 20))
      return;
    View col = v;
    col.cols = 1;
    EwHost p;
    if (!compile(add_view(col), p, false)) return;
    View t = temp(v.rows, 1);
    push_ew(p, t);
    E_[e].v = bcast_cols(t, v.cols);
  }

  // copy: a lone view is copied into a temporary (or dest) instead of
  // being returned as it is.
  View emit_ew(int root, const View* dest, int64_t rows, int64_t cols, bool copy = false) {
    if (status_ != HEXLA_OK) return View{};
    if (E_[root].kind == 1 && !dest && !copy) return E_[root].v;
    if (E_[root].kind == 3 && !E_[root].diag) return materialize(E_[root].node, E_[root].trans, dest);
    std::vector<int> pend;
    collect(root, 3, pend);
    int epi = -1;
    if (o_.fuse && o_.planner != HEXLA_PLANNER_NAIVE && E_[root].kind == 0) {
      for (int p : pend)
        if (!E_[p].diag && gemv_final(E_[p].node, E_[p].trans)) {
          epi = p;
          break;
        }
    }
    for (int p : pend) {
      if (p == epi) continue;
      View v = pending_value(p);
      E_[p].kind = 1;
      E_[p].v = v;
    }
    if (status_ != HEXLA_OK) return View{};
    if (E_[root].kind == 1 && !dest && !copy) return E_[root].v;
    if (!o_.fuse || o_.planner == HEXLA_PLANNER_NAIVE) {
      if (E_[root].kind == 1 && !dest) {  // copy a lone view
        EwHost p;
        if (!compile(root, p, false)) return View{};
        View o = temp(rows, cols);
        push_ew(p, o);
        return o;
      }
      return emit_unfused(root, dest);
    }
    gather_broadcasts(root);
    if (epi >= 0) {
      E_[epi].kind = 4;
      EwHost prog;
      if (!compile(root, prog, true)) return View{};
      return lower_chain(E_[epi].node, E_[epi].trans, dest, &prog);
    }
    EwHost prog;
    if (!compile(root, prog, false)) return View{};
    View o = out_or_temp(dest, rows, cols);
    push_ew(prog, o);
    return o;
  }

  // One pass that multiplies and sums: dest (1 x 1) = alpha * the sum of
  // the program `root` over its rows x cols elements.
  View emit_sum(int root, int64_t rows, int64_t cols, double alpha, const View* dest) {
    if (status_ != HEXLA_OK) return View{};
    std::vector<int> pend;
    collect(root, 3, pend);
    for (int p : pend) {
      View v = pending_value(p);
      E_[p].kind = 1;
      E_[p].v = v;
    }
    gather_broadcasts(root);
    EwHost prog;
    if (status_ != HEXLA_OK || !compile(root, prog, false)) return View{};
    Step st;
    st.kind = StepKind::EwSum;
    st.dtype = dtype_;
    st.name = "sum";
    st.ew = prog;
    st.m = rows;
    st.n = cols;
    st.alpha = alpha;
    st.sum = true;
    st.out = out_or_temp(dest, 1, 1);
    const size_t pb = k::ew_sum_partial_bytes(dtype_, rows * cols);
    if (pb) st.partial = work(int64_t(pb));
    const double elems = double(rows) * double(cols);
    st.flops = elems * (prog.n_arith + 1);
    st.bytes = elems * double(esz_) * double(prog.leaves.size()) + double(esz_);
    steps_.push_back(st);
    return st.out;
  }

  // --------------------------------------------------------- diagonals
  // Only the diagonal of a product (expressions (4), (5) of Sec. III):
  // d_i = sum_k L_ik R_ki with L, R the chain's factors on either side of
  // the split with the fewest multiply-adds (sub-chains by the DP), and
  // with `sum` its trace. diag_of_dest: write d onto the diagonal of dest
  // (stride ld + 1) instead of into a vector.
  static bool plain_chain(const std::vector<Factor>& f) {
    if (f.size() < 2) return false;
    for (const Factor& q : f)
      if (q.kind == 1 || q.kind == 3) return false;
    return true;
  }

  View diag_product(std::vector<Factor> f, double alpha, const View* dest, bool sum,
                    bool diag_of_dest = false) {
    for (Factor& q : f)
      if (q.kind == 2) {
        q.v = materialize(q.node, q.trans, nullptr);
        q.kind = 0;
      }
    if (status_ != HEXLA_OK) return View{};
    const int L = int(f.size());
    std::vector<int64_t> d(L + 1);
    d[0] = f[0].v.rows;
    for (int i = 0; i < L; ++i) d[i + 1] = f[i].v.cols;
    const int64_t nd = std::min(d[0], d[L]);
    const std::vector<char> sym(L, 0);
    const auto cost = dp_table(d, sym);
    int best = 1;
    i128 bc = -1;
    for (int p = 1; p < L; ++p) {
      const i128 c = cost[0][p - 1] + cost[p][L - 1] + i128(nd) * d[p];
      if (bc < 0 || c < bc) {
        bc = c;
        best = p;
      }
    }
    std::vector<Factor> lf(f.begin(), f.begin() + best), rf(f.begin() + best, f.end());
    View left = best == 1 ? lf[0].v : chain_views(lf, 1.0, nullptr, nullptr);
    View right = best == L - 1 ? rf[0].v : chain_views(rf, 1.0, nullptr, nullptr);
    left = dense(left);
    right = dense(right);
    if (status_ != HEXLA_OK) return View{};
    macs_ += double(nd) * double(d[best]);
    Step st;
    st.kind = StepKind::DiagProd;
    st.dtype = dtype_;
    st.name = sum ? "trace_product" : "diag_product";
    st.A = left;
    st.B = right;
    st.m = nd;
    st.kk = d[best];
    st.alpha = alpha;
    st.sum = sum;
    st.out = dest ? *dest : temp(sum ? 1 : nd, 1);
    st.incd = diag_of_dest ? 0 : 1;
    const size_t pb = k::diagprod_partial_bytes(dtype_, nd, d[best], sum);
    if (pb) st.partial = work(int64_t(pb));
    st.flops = 2.0 * double(nd) * double(d[best]);
    st.bytes = (2.0 * double(nd) * double(d[best]) + (sum ? 1.0 : double(nd))) * double(esz_);
    steps_.push_back(st);
    return st.out;
  }

  // The main diagonal of node a's value, as a column vector (a view when
  // it can be one).
  View diag_value(uint32_t a, const View* dest) {
    const Node& y = N(a);
    const int64_t nd = y.scalar ? 1 : std::min(y.rows, y.cols);
    const bool naive = o_.planner == HEXLA_PLANNER_NAIVE;
    if (!y.scalar && !naive && is_chain(a)) {
      std::vector<Factor> f;
      double alpha = 1.0;
      flatten(a, false, f, alpha);
      if (plain_chain(f)) return diag_product(f, alpha, dest, false);
    }
    if (!y.scalar && (naive || is_chain(a))) {
      // the full value, then its diagonal (the naive evaluation)
      const View d = diag_view(materialize(a, false, nullptr));
      if (!dest) return d;
      return emit_ew(add_view(d), dest, nd, 1);
    }
    return emit_ew(with_diag(a), dest, nd, 1);
  }

  // trace(a): a product's trace by the diagonal product; otherwise one pass
  // summing the diagonal of the (element-wise) value.
  View trace_value(uint32_t a, const View* dest) {
    const Node& y = N(a);
    const bool naive = o_.planner == HEXLA_PLANNER_NAIVE;
    if (!y.scalar && !naive && is_chain(a)) {
      std::vector<Factor> f;
      double alpha = 1.0;
      flatten(a, false, f, alpha);
      if (plain_chain(f)) return diag_product(f, alpha, dest, true);
    }
    const int64_t nd = y.scalar ? 1 : std::min(y.rows, y.cols);
    int r;
    if (y.scalar) r = add_const(scalar_value(a));
    else if (naive || is_chain(a)) r = add_view(diag_view(materialize(a, false, nullptr)));
    else r = with_diag(a);
    return emit_sum(r, nd, 1, 1.0, dest);
  }

  // The diagonal values of diagmat(z) as an n x 1 view: the vector itself,
  // or the diagonal of the matrix.
  View diag_vector(uint32_t z) {
    const Node& y = N(z);
    if (is_vector(y)) {
      const int r = without_diag(z, y.rows == 1 && y.cols != 1);
      return emit_ew(r, nullptr, std::max(y.rows, y.cols), 1);
    }
    return diag_value(z, nullptr);
  }

  // diagmat(a) as a value: expression (4) (the diagonal of a product written
  // onto zeros) or one element-wise pass.
  View diagmat_value(uint32_t a, bool t, const View* dest) {
    const Node& y = N(a);
    const bool vec = is_vector(y);
    const int64_t n = std::max(y.rows, y.cols);
    const int64_t rows = vec ? n : (t ? y.cols : y.rows), cols = vec ? n : (t ? y.rows : y.cols);
    if (!vec && !y.scalar && o_.planner != HEXLA_PLANNER_NAIVE && is_chain(a)) {
      std::vector<Factor> f;
      double alpha = 1.0;
      flatten(a, false, f, alpha);
      if (plain_chain(f)) {
        View o = out_or_temp(dest, rows, cols);
        EwHost zero;
        if (!compile(add_const(0.0), zero, false)) return View{};
        push_ew(zero, o);
        diag_product(f, alpha, &o, false, true);
        return o;
      }
    }
    int r;
    if (vec) {
      const View dv = diag_vector(a);
      r = add_op(k::EW_MUL, add_ident(rows, cols), add_view(bcast_cols(dv, cols)), rows, cols);
    } else {
      r = add_op(k::EW_MUL, add_ident(rows, cols), without_diag(a, t), rows, cols);
    }
    return emit_ew(r, dest, rows, cols);
  }

  // One kernel and one temporary per operation (the eager evaluation the
  // paper contrasts with fusion, Sec. II).
  View emit_unfused(int e, const View* dest) {
    const ENode node = E_[e];
    if (node.kind == 1) {
      if (!dest) return node.v;
      EwHost p;
      compile(e, p, false);
      push_ew(p, *dest);
      return *dest;
    }
    if (node.kind != 0) {
      fail(HEXLA_E_UNSUPPORTED, "internal: unexpected element-wise node");
      return View{};
    }
    int a = node.a, b = node.b;
    if (E_[a].kind == 0) a = add_view(emit_unfused(a, nullptr));
    if (b >= 0 && E_[b].kind == 0) b = add_view(emit_unfused(b, nullptr));
    const int single = add_op(node.op, a, b, node.rows, node.cols);
    EwHost p;
    compile(single, p, false);
    View o = out_or_temp(dest, node.rows, node.cols);
    push_ew(p, o);
    return o;
  }

  int need(int e) const {
    const ENode& n = E_[e];
    if (n.kind != 0) return 1;
    if (n.b < 0) return need(n.a);
    const ENode& a = E_[n.a];
    const ENode& b = E_[n.b];
    const bool comm = n.op == k::EW_ADD || n.op == k::EW_MUL;
    if (b.kind == 2 && (comm || n.op == k::EW_SUB)) return need(n.a);
    if (a.kind == 2 && comm) return need(n.b);
    if (comm && b.kind == 1) return need(n.a);
    if (comm && a.kind == 1) return need(n.b);
    const int na = need(n.a), nb = need(n.b);
    return na == nb ? na + 1 : std::max(na, nb);
  }

  struct Gen {
    EwHost* p;
    bool ok = true;
    std::string why;
  };

  int leaf_slot(Gen& g, const View& v) {
    for (size_t i = 0; i < g.p->leaves.size(); ++i)
      if (same_view(g.p->leaves[i], v)) return int(i);
    if (int(g.p->leaves.size()) >= k::kEwMaxLeaf) {
      g.ok = false;
      g.why = "leaves";
      return 0;
    }
    g.p->leaves.push_back(v);
    return int(g.p->leaves.size()) - 1;
  }
  int const_slot(Gen& g, double c) {
    for (int i = 0; i < g.p->n_cst; ++i)
      if (g.p->cst[i] == c) return i;
    if (g.p->n_cst >= k::kEwMaxConst) {
      g.ok = false;
      g.why = "constants";
      return 0;
    }
    g.p->cst[g.p->n_cst] = c;
    return g.p->n_cst++;
  }
  void emit(Gen& g, int op, int arg) {
    if (g.p->n_instr >= k::kEwMaxInstr) {
      g.ok = false;
      g.why = "length";
      return;
    }
    g.p->op[g.p->n_instr] = uint8_t(op);
    g.p->arg[g.p->n_instr] = uint8_t(arg);
    g.p->n_instr++;
    if (op >= k::EW_ADD) g.p->n_arith++;
  }

  void gen(Gen& g, int e) {
    if (!g.ok) return;
    const ENode& n = E_[e];
    if (n.kind == 1) return emit(g, k::EW_LEAF, leaf_slot(g, n.v));
    if (n.kind == 2) return emit(g, k::EW_CONST, const_slot(g, n.c));
    if (n.kind == 4) return emit(g, k::EW_EXTRA, 0);
    if (n.kind == 5) return emit(g, k::EW_IDENT, 0);
    if (n.b < 0) {
      gen(g, n.a);
      return emit(g, n.op, 0);
    }
    const ENode& a = E_[n.a];
    const ENode& b = E_[n.b];
    const bool comm = n.op == k::EW_ADD || n.op == k::EW_MUL;
    if (b.kind == 2 && (comm || n.op == k::EW_SUB)) {
      gen(g, n.a);
      if (n.op == k::EW_MUL) return emit(g, k::EW_SCALE, const_slot(g, b.c));
      return emit(g, k::EW_ADDC, const_slot(g, n.op == k::EW_SUB ? -b.c : b.c));
    }
    if (a.kind == 2 && comm) {
      gen(g, n.b);
      return emit(g, n.op == k::EW_MUL ? k::EW_SCALE : k::EW_ADDC, const_slot(g, a.c));
    }
    if (comm && b.kind == 1) {
      gen(g, n.a);
      return emit(g, n.op == k::EW_MUL ? k::EW_LEAFMUL : k::EW_LEAFADD, leaf_slot(g, b.v));
    }
    if (comm && a.kind == 1) {
      gen(g, n.b);
      return emit(g, n.op == k::EW_MUL ? k::EW_LEAFMUL : k::EW_LEAFADD, leaf_slot(g, a.v));
    }
    if (need(n.b) > need(n.a)) {
      gen(g, n.b);
      gen(g, n.a);
      int op = n.op;
      if (op == k::EW_SUB) op = k::EW_RSUB;
      else if (op == k::EW_DIV) op = k::EW_RDIV;
      return emit(g, op, 0);
    }
    gen(g, n.a);
    gen(g, n.b);
    emit(g, n.op, 0);
  }

  // The deepest operation child of e (to split off when a program is too big).
  int deepest_op(int e) const {
    const ENode& n = E_[e];
    int best = -1, bn = 0;
    for (int c : {n.a, n.b}) {
      if (c < 0 || E_[c].kind != 0) continue;
      const int v = need(c) * 64 + size(c);
      if (v > bn) {
        bn = v;
        best = c;
      }
    }
    return best;
  }
  int size(int e) const {
    const ENode& n = E_[e];
    if (n.kind != 0) return 1;
    return 1 + size(n.a) + (n.b >= 0 ? size(n.b) : 0);
  }

  bool compile(int root, EwHost& out, bool allow_extra) {
    for (int attempt = 0; attempt < 64; ++attempt) {
      EwHost p;
      Gen g;
      g.p = &p;
      if (need(root) <= k::kEwMaxDepth) gen(g, root);
      else {
        g.ok = false;
        g.why = "depth";
      }
      if (g.ok) {
        for (int i = 0; i < p.n_instr; ++i)
          if (p.op[i] == k::EW_IDENT) p.ident = true;
        out = p;
        return true;
      }
      // split the deepest operation subtree into its own pass and retry
      int victim = -1;
      for (int e = root; e >= 0;) {
        const int d = deepest_op(e);
        if (d < 0) break;
        victim = d;
        if (need(d) <= k::kEwMaxDepth && size(d) <= k::kEwMaxInstr / 2) break;
        e = d;
      }
      if (victim < 0) {
        fail(HEXLA_E_UNSUPPORTED, "element-wise program cannot be split (" + g.why + ")");
        return false;
      }
      (void)allow_extra;
      View v = emit_ew(victim, nullptr, E_[victim].rows, E_[victim].cols);
      E_[victim].kind = 1;
      E_[victim].v = v;
      E_[victim].a = E_[victim].b = -1;
    }
    fail(HEXLA_E_UNSUPPORTED, "element-wise program too large");
    return false;
  }

  void push_ew(const EwHost& p, const View& o) {
    Step s;
    s.kind = StepKind::Ew;
    s.dtype = dtype_;
    s.name = "elementwise";
    s.ew = p;
    s.out = o;
    const double elems = double(o.rows) * double(o.cols);
    s.flops = elems * p.n_arith;
    s.bytes = elems * double(esz_) * double(p.leaves.size() + 1);
    if (o_.codegen && codegen_enabled()) s.cg_src = codegen_source(p, dtype_);
    steps_.push_back(s);
  }

  // ----------------------------------------------------------------- chains
  View lower_chain(uint32_t n, bool t, const View* dest, const EwHost* epi) {
    std::vector<Factor> f;
    double alpha = 1.0;
    flatten(n, t, f, alpha);
    bool diag = false;
    for (const Factor& q : f) diag = diag || q.kind == 3;
    if (diag) return chain_with_diagonals(f, alpha, dest);
    for (Factor& q : f)
      if (q.kind == 2) {
        q.v = dense(materialize(q.node, q.trans, nullptr));
        q.kind = 0;
      }
    if (status_ != HEXLA_OK) return View{};
    return chain_views(f, alpha, dest, epi);
  }

  // A chain with diagonal factors diagmat(z) (expressions (3) and (7) of
  // Sec. III). Only z's diagonal values are read:
  //   * a row vector, diagonal factors and a column vector: one pass that
  //     multiplies and sums, x^T diag(d1) ... y = sum_i x_i d1_i ... y_i;
  //   * otherwise each square diagonal factor scales the rows of the factor
  //     on its right (or the columns of the one on its left, at the end), as
  //     one element-wise pass; a chain left with one factor is that pass,
  //     written to the destination.
  // The naive planner builds each diagonal matrix instead (the paper's naive
  // evaluation, a temporary dense matrix and a general product).
  View chain_with_diagonals(std::vector<Factor> f, double alpha, const View* dest) {
    const bool naive = o_.planner == HEXLA_PLANNER_NAIVE;
    bool inverse = false;
    for (const Factor& q : f) inverse = inverse || q.kind == 1;
    for (Factor& q : f)
      if (q.kind == 3 && (naive || inverse || q.v.rows != q.v.cols)) {
        q.v = diagmat_value(q.node, q.trans, nullptr);
        q.kind = 0;
      }
    for (Factor& q : f)
      if (q.kind == 2) {
        q.v = dense(materialize(q.node, q.trans, nullptr));
        q.kind = 0;
      }
    if (status_ != HEXLA_OK) return View{};
    bool any = false;
    for (const Factor& q : f) any = any || q.kind == 3;
    if (!any) return chain_views(f, alpha, dest, nullptr);
    const int L = int(f.size());
    // x^T diag(d1) ... diag(dk) y
    bool dot = L >= 3 && f[0].kind == 0 && f[L - 1].kind == 0 && f[0].v.rows == 1 &&
               f[L - 1].v.cols == 1;
    for (int i = 1; i + 1 < L && dot; ++i) dot = f[i].kind == 3;
    if (dot) {
      const int64_t n = f[0].v.cols;
      int r = add_view(transposed(f[0].v));
      for (int i = 1; i + 1 < L; ++i)
        r = add_op(k::EW_MUL, r, add_view(diag_vector(f[i].node)), n, 1);
      r = add_op(k::EW_MUL, r, add_view(f[L - 1].v), n, 1);
      return emit_sum(r, n, 1, alpha, dest);
    }
    // fold the diagonals into their neighbours
    std::vector<int> roots;         // element-wise tree of each remaining factor
    std::vector<Factor> g;
    std::vector<View> pend;         // diagonal vectors waiting for a right neighbour
    for (const Factor& q : f) {
      if (q.kind == 3) {
        pend.push_back(diag_vector(q.node));
        continue;
      }
      int r = add_view(q.v);
      for (const View& d : pend)
        r = add_op(k::EW_MUL, add_view(bcast_cols(d, q.v.cols)), r, q.v.rows, q.v.cols);
      pend.clear();
      roots.push_back(r);
      g.push_back(q);
    }
    if (status_ != HEXLA_OK) return View{};
    if (g.empty()) {  // only diagonal factors: diagmat of the product of their diagonals
      const int64_t n = f[0].v.rows;
      int r = add_ident(n, n);
      for (const View& d : pend) r = add_op(k::EW_MUL, r, add_view(bcast_cols(d, n)), n, n);
      if (alpha != 1.0) r = add_op(k::EW_MUL, r, add_const(alpha), n, n);
      return emit_ew(r, dest, n, n);
    }
    for (const View& d : pend) {  // diagonals at the end scale the last factor's columns
      const View& v = g.back().v;
      roots.back() = add_op(k::EW_MUL, roots.back(), add_view(bcast_rows(d, v.rows)), v.rows, v.cols);
    }
    if (g.size() == 1) {
      int r = roots[0];
      if (alpha != 1.0) r = add_op(k::EW_MUL, r, add_const(alpha), g[0].v.rows, g[0].v.cols);
      return emit_ew(r, dest, g[0].v.rows, g[0].v.cols);
    }
    for (size_t i = 0; i < g.size(); ++i)
      if (E_[roots[i]].kind != 1) g[i].v = emit_ew(roots[i], nullptr, g[i].v.rows, g[i].v.cols);
    if (status_ != HEXLA_OK) return View{};
    return chain_views(g, alpha, dest, nullptr);
  }

  View chain_views(std::vector<Factor> f, double alpha, const View* dest, const EwHost* epi) {
    const bool naive = o_.planner == HEXLA_PLANNER_NAIVE;
    for (size_t p = 0; p < f.size(); ++p) {
      if (f[p].kind != 1) continue;
      View s = dense(materialize(f[p].node, f[p].trans, nullptr));
      if (status_ != HEXLA_OK) return View{};
      if (naive || p + 1 == f.size()) {
        f[p].v = explicit_inverse(s, nullptr);
        f[p].kind = 0;
        continue;
      }
      std::vector<Factor> rest(f.begin() + p + 1, f.end());
      double ra = 1.0;
      if (p == 0) std::swap(ra, alpha);
      View rhs = chain_views(rest, ra, nullptr, nullptr);
      if (status_ != HEXLA_OK) return View{};
      const bool direct = p == 0 && dest && !epi;
      View xo = direct ? *dest : temp(s.cols, rhs.cols);
      solve(s, dense(rhs), xo, gram_product(f[p].node));
      f.resize(p);
      Factor q;
      q.kind = 0;
      q.v = xo;
      f.push_back(q);
      break;
    }
    if (status_ != HEXLA_OK) return View{};
    if (f.size() == 1) {
      const View v = f[0].v;
      if (epi) {
        fail(HEXLA_E_UNSUPPORTED, "internal: epilogue without a product");
        return View{};
      }
      if (alpha == 1.0 && (!dest || same_view(v, *dest))) return v;
      const int leaf = add_view(v);
      const int root = alpha == 1.0 ? leaf : add_op(k::EW_MUL, leaf, add_const(alpha), v.rows, v.cols);
      EwHost prog;
      if (!compile(root, prog, false)) return View{};
      View o = out_or_temp(dest, v.rows, v.cols);
      push_ew(prog, o);
      return o;
    }
    const int L = int(f.size());
    std::vector<int64_t> dims(L + 1);
    dims[0] = f[0].v.rows;
    for (int i = 0; i < L; ++i) dims[i + 1] = f[i].v.cols;
    std::vector<char> sym(L, 0);
    if (o_.syrk && !naive)
      for (int i = 0; i + 1 < L; ++i)
        sym[i] = same_storage(f[i].v, f[i + 1].v) && f[i].v.trans != f[i + 1].v.trans;
    std::vector<TNode> tree;
    int root;
    if (o_.planner == HEXLA_PLANNER_GREEDY) root = order_greedy(dims, tree);
    else if (naive) root = order_left(L, tree);
    else if (o_.planner == HEXLA_PLANNER_LEARNED && ctx_->model) root = order_learned(dims, sym, f, tree);
    else if (o_.planner == HEXLA_PLANNER_ROOFLINE) root = order_roofline(dims, sym, tree);
    else root = order_dp(dims, sym, tree);
    if (status_ != HEXLA_OK) return View{};
    macs_ += double(tree_cost(root, tree, dims, sym));
    return emit_tree(root, tree, f, sym, true, dest, alpha, epi);
  }

  i128 pair_cost(const std::vector<int64_t>& d, int lo, int split, int hi,
                 const std::vector<char>& sym) const {
    if (hi == lo + 1 && sym[lo]) return i128(d[lo]) * (d[lo] + 1) / 2 * d[lo + 1];
    return i128(d[lo]) * d[split + 1] * d[hi + 1];
  }

  i128 tree_cost(int t, const std::vector<TNode>& tree, const std::vector<int64_t>& d,
                 const std::vector<char>& sym) const {
    const TNode& n = tree[t];
    if (n.leaf >= 0) return 0;
    const int split = tree[n.left].hi;
    return pair_cost(d, n.lo, split, n.hi, sym) + tree_cost(n.left, tree, d, sym) +
           tree_cost(n.right, tree, d, sym);
  }

  int mk_leaf(std::vector<TNode>& tree, int i) {
    TNode n;
    n.leaf = i;
    n.lo = n.hi = i;
    tree.push_back(n);
    return int(tree.size()) - 1;
  }
  int mk_pair(std::vector<TNode>& tree, int l, int r) {
    TNode n;
    n.left = l;
    n.right = r;
    n.lo = tree[l].lo;
    n.hi = tree[r].hi;
    tree.push_back(n);
    return int(tree.size()) - 1;
  }

  int order_left(int L, std::vector<TNode>& tree) {
    int t = mk_leaf(tree, 0);
    for (int i = 1; i < L; ++i) t = mk_pair(tree, t, mk_leaf(tree, i));
    return t;
  }

  // Minimum multiply-adds of every sub-chain lo..hi (O(L^3)).
  std::vector<std::vector<i128>> dp_table(const std::vector<int64_t>& d,
                                          const std::vector<char>& sym) const {
    const int L = int(d.size()) - 1;
    std::vector<std::vector<i128>> cost(L, std::vector<i128>(L, 0));
    for (int len = 2; len <= L; ++len)
      for (int lo = 0; lo + len - 1 < L; ++lo) {
        const int hi = lo + len - 1;
        i128 best = -1;
        for (int s = lo; s < hi; ++s) {
          const i128 c = cost[lo][s] + cost[s + 1][hi] + pair_cost(d, lo, s, hi, sym);
          if (best < 0 || c < best) best = c;
        }
        cost[lo][hi] = best;
      }
    return cost;
  }

  // Roofline time of one product: the longer of its flops at the MFMA peak
  // of the product precision and its bytes (operands read once, result
  // written once) at 8 TB/s; a symmetric pair reads its operand once.
  double pair_time(const std::vector<int64_t>& d, int lo, int split, int hi,
                   const std::vector<char>& sym) const {
    double peak = dtype_ == HEXLA_F64 ? 78.6e12 : 157.3e12;
    if (dtype_ == HEXLA_F32 && o_.product_precision == HEXLA_PRODUCT_BF16X3) peak = 2.5e15 / 3.0;
    if (dtype_ == HEXLA_F32 && o_.product_precision == HEXLA_PRODUCT_BF16X6) peak = 2.5e15 / 6.0;
    const double r = double(d[lo]), k = double(d[split + 1]), c = double(d[hi + 1]);
    double flops, elems;
    if (hi == lo + 1 && sym[lo]) {
      flops = r * (r + 1.0) * k;
      elems = r * k + r * c;
    } else {
      flops = 2.0 * r * k * c;
      elems = r * k + k * c + r * c;
    }
    return std::max(flops / peak, elems * double(esz_) / 8e12);
  }

  // Exact minimum of the summed roofline times over all bracketings;
  // ties keep the first split.
  int order_roofline(const std::vector<int64_t>& d, const std::vector<char>& sym,
                     std::vector<TNode>& tree) {
    const int L = int(d.size()) - 1;
    std::vector<std::vector<double>> cost(L, std::vector<double>(L, 0.0));
    std::vector<std::vector<int>> arg(L, std::vector<int>(L, -1));
    for (int len = 2; len <= L; ++len)
      for (int lo = 0; lo + len - 1 < L; ++lo) {
        const int hi = lo + len - 1;
        double best = -1.0;
        for (int s = lo; s < hi; ++s) {
          const double c = cost[lo][s] + cost[s + 1][hi] + pair_time(d, lo, s, hi, sym);
          if (best < 0.0 || c < best) {
            best = c;
            arg[lo][hi] = s;
          }
        }
        cost[lo][hi] = best;
      }
    std::function<int(int, int)> build = [&](int lo, int hi) -> int {
      if (lo == hi) return mk_leaf(tree, lo);
      const int s = arg[lo][hi];
      const int l = build(lo, s);
      const int r = build(s + 1, hi);
      return mk_pair(tree, l, r);
    };
    return build(0, L - 1);
  }

  // Exact minimum over all bracketings (O(L^3)); ties keep the first split.
  int order_dp(const std::vector<int64_t>& d, const std::vector<char>& sym,
               std::vector<TNode>& tree) {
    const int L = int(d.size()) - 1;
    std::vector<std::vector<i128>> cost(L, std::vector<i128>(L, 0));
    std::vector<std::vector<int>> arg(L, std::vector<int>(L, -1));
    for (int len = 2; len <= L; ++len)
      for (int lo = 0; lo + len - 1 < L; ++lo) {
        const int hi = lo + len - 1;
        i128 best = -1;
        for (int s = lo; s < hi; ++s) {
          const i128 c = cost[lo][s] + cost[s + 1][hi] + pair_cost(d, lo, s, hi, sym);
          if (best < 0 || c < best) {
            best = c;
            arg[lo][hi] = s;
          }
        }
        cost[lo][hi] = best;
      }
    std::function<int(int, int)> build = [&](int lo, int hi) -> int {
      if (lo == hi) return mk_leaf(tree, lo);
      const int s = arg[lo][hi];
      const int l = build(lo, s);
      const int r = build(s + 1, hi);
      return mk_pair(tree, l, r);
    };
    return build(0, L - 1);
  }

  // The learned planner: every product (lo, s, hi) a bracketing of the chain
  // can contain is priced at its predicted-fastest configuration (one
  // inference launch for all of them), a DP minimises the predicted time,
  // and the multiply-add DP decides: its order is used unless the learned
  // order costs at most twice its multiply-adds and is predicted faster.
  // The chosen configurations are kept for product().
  int order_learned(const std::vector<int64_t>& d, const std::vector<char>& sym,
                    const std::vector<Factor>& f, std::vector<TNode>& tree) {
    const int L = int(d.size()) - 1;
    struct Prod {
      Step st;
      int ta = 0, tb = 0;
      size_t first = 0, count = 0;
      std::vector<k::GemmConfig> cands;
      double us = 0.0;
      k::GemmConfig best{};
    };
    auto at = [L](int lo, int s, int hi) { return (size_t(lo) * L + s) * L + hi; };
    std::vector<int> index(size_t(L) * L * L, -1);
    std::vector<Prod> prods;
    std::vector<float> feats;
    // a product no bracketing within twice the fewest multiply-adds can
    // contain (its own and its operands' cheapest costs exceed that) is
    // never kept by the check below: it is not priced
    const auto macs = dp_table(d, sym);
    const i128 limit = 2 * macs[0][L - 1];
    for (int lo = 0; lo < L; ++lo)
      for (int hi = lo + 1; hi < L; ++hi)
        for (int s = lo; s < hi; ++s) {
          Prod p;
          if (macs[lo][s] + macs[s + 1][hi] + pair_cost(d, lo, s, hi, sym) > limit) {
            p.us = 1e30;
            index[at(lo, s, hi)] = int(prods.size());
            prods.push_back(std::move(p));
            continue;
          }
          p.st.dtype = dtype_;
          p.st.precision = dtype_ == HEXLA_F32 ? o_.product_precision : 0;
          p.st.mode = (hi == lo + 1 && sym[lo] && o_.syrk) ? 1 : 0;
          p.st.m = d[lo];
          p.st.kk = d[s + 1];
          p.st.n = d[hi + 1];
          p.ta = s == lo && f[lo].v.trans ? 1 : 0;
          p.tb = s + 1 == hi && f[hi].v.trans ? 1 : 0;
          if (p.st.m == 1 || p.st.n == 1) {  // matrix-vector: memory-bound estimate
            const double bytes = double(esz_) * (double(p.st.m) * p.st.kk +
                                                 double(p.st.kk) * p.st.n + double(p.st.m) * p.st.n);
            p.us = 4.0 + bytes / 4.0e6;
          } else {
            p.cands = learned_candidates(p.st);
            p.first = feats.size() / k::kMlpFeatures;
            p.count = p.cands.size();
            feats.resize(feats.size() + p.count * k::kMlpFeatures);
            product_features_many(dtype_, p.st.precision, p.st.mode, p.ta, p.tb, p.st.m, p.st.n,
                                  p.st.kk, p.cands.data(), int(p.count),
                                  &feats[p.first * k::kMlpFeatures]);
          }
          index[at(lo, s, hi)] = int(prods.size());
          prods.push_back(std::move(p));
        }
    std::vector<float> us;
    std::string err;
    if (!model_predict_us(ctx_->model, feats, us, &err)) {
      fail(HEXLA_E_DEVICE, err);
      return 0;
    }
    for (Prod& p : prods) {
      if (p.count == 0) continue;
      size_t bi = 0;
      for (size_t c = 1; c < p.count; ++c)
        if (us[p.first + c] < us[p.first + bi]) bi = c;
      p.us = us[p.first + bi];
      p.best = p.cands[bi];
      learned_cfg_[tune_key(p.st, p.ta, p.tb)] = p.best;
    }
    // DP over predicted microseconds
    std::vector<std::vector<double>> cost(L, std::vector<double>(L, 0.0));
    std::vector<std::vector<int>> arg(L, std::vector<int>(L, -1));
    for (int len = 2; len <= L; ++len)
      for (int lo = 0; lo + len - 1 < L; ++lo) {
        const int hi = lo + len - 1;
        double best = -1.0;
        for (int s = lo; s < hi; ++s) {
          const double c = cost[lo][s] + cost[s + 1][hi] + prods[size_t(index[at(lo, s, hi)])].us;
          if (best < 0 || c < best) {
            best = c;
            arg[lo][hi] = s;
          }
        }
        cost[lo][hi] = best;
      }
    std::function<int(int, int)> build = [&](int lo, int hi) -> int {
      if (lo == hi) return mk_leaf(tree, lo);
      const int s = arg[lo][hi];
      const int l = build(lo, s);
      const int r = build(s + 1, hi);
      return mk_pair(tree, l, r);
    };
    const int learned = build(0, L - 1);
    const int dp = order_dp(d, sym, tree);
    std::function<double(int)> pred = [&](int t) -> double {
      const TNode& n = tree[t];
      if (n.leaf >= 0) return 0.0;
      const int s = tree[n.left].hi;
      return prods[size_t(index[at(n.lo, s, n.hi)])].us + pred(n.left) + pred(n.right);
    };
    const double pl = pred(learned), pd = pred(dp);
    const i128 ml = tree_cost(learned, tree, d, sym), md = tree_cost(dp, tree, d, sym);
    const bool keep = ml <= 2 * md && pl < pd;
    std::ostringstream js;
    js << "{\"chain\":" << L << ",\"pred_us_learned\":" << pl << ",\"pred_us_dp\":" << pd
       << ",\"macs_learned\":" << double(ml) << ",\"macs_dp\":" << double(md)
       << ",\"chosen\":\"" << (keep ? "learned" : "dp") << "\"}";
    learned_notes_.push_back(js.str());
    return keep ? learned : dp;
  }

  // The paper's rule (Sec. II): multiply the adjacent pair whose product has
  // the fewest elements, leftmost on ties, and repeat.
  int order_greedy(const std::vector<int64_t>& d, std::vector<TNode>& tree) {
    struct Item {
      int t;
      int64_t rows, cols;
    };
    std::vector<Item> items;
    for (int i = 0; i + 1 < int(d.size()); ++i) items.push_back({mk_leaf(tree, i), d[i], d[i + 1]});
    while (items.size() > 1) {
      size_t best = 0;
      i128 bs = -1;
      for (size_t j = 0; j + 1 < items.size(); ++j) {
        const i128 sz = i128(items[j].rows) * items[j + 1].cols;
        if (bs < 0 || sz < bs) {
          bs = sz;
          best = j;
        }
      }
      Item merged{mk_pair(tree, items[best].t, items[best + 1].t), items[best].rows,
                  items[best + 1].cols};
      items.erase(items.begin() + best, items.begin() + best + 2);
      items.insert(items.begin() + best, merged);
    }
    return items[0].t;
  }

  View emit_tree(int t, const std::vector<TNode>& tree, const std::vector<Factor>& f,
                 const std::vector<char>& sym, bool is_root, const View* dest, double alpha,
                 const EwHost* epi) {
    const TNode n = tree[t];
    if (n.leaf >= 0) return f[n.leaf].v;
    View a = emit_tree(n.left, tree, f, sym, false, nullptr, 1.0, nullptr);
    View b = emit_tree(n.right, tree, f, sym, false, nullptr, 1.0, nullptr);
    if (status_ != HEXLA_OK) return View{};
    const bool syrk = tree[n.left].leaf >= 0 && tree[n.right].leaf >= 0 && sym[n.lo] != 0;
    View c = (is_root && dest) ? *dest : temp(a.rows, b.cols);
    product(a, b, c, is_root ? alpha : 1.0, syrk, is_root ? epi : nullptr);
    return c;
  }

  void product(const View& a, const View& b, const View& c, double alpha, bool syrk,
               const EwHost* epi) {
    const int64_t m = a.rows, kk = a.cols, n = b.cols;
    Step s;
    s.dtype = dtype_;
    s.alpha = alpha;
    s.C = c;
    s.m = m;
    s.n = n;
    s.kk = kk;
    if (n == 1 || m == 1) {
      s.kind = StepKind::Gemv;
      if (n == 1) {
        s.A = a;
        s.B = b;
      } else {  // C^T = B^T A^T
        s.A = transposed(b);
        s.B = transposed(a);
        s.m = n;
        s.n = 1;
      }
      s.name = s.A.trans ? "gemv_t" : "gemv_n";
      s.flops = 2.0 * double(m) * double(n) * double(kk);
      s.bytes = double(esz_) * (double(m) * kk + double(kk) * n + double(m) * n);
      if (epi) {
        s.has_epi = true;
        s.ew = *epi;
        s.flops += double(m) * n * epi->n_arith;
        s.bytes += double(esz_) * double(m) * n * double(epi->leaves.size());
      }
    } else {
      if (epi) {
        fail(HEXLA_E_UNSUPPORTED, "internal: epilogue on a matrix product");
        return;
      }
      s.kind = StepKind::Gemm;
      s.A = a;
      s.B = b;
      s.mode = syrk ? 1 : 0;
      s.precision = (dtype_ == HEXLA_F32) ? o_.product_precision : 0;
      s.cfg = k::gemm_choose(dtype_, s.precision, s.mode, m, n, kk);
      const auto learned = learned_cfg_.find(tune_key(s, a.trans ? 1 : 0, b.trans ? 1 : 0));
      if (learned != learned_cfg_.end()) s.cfg = learned->second;
      const auto tuned = ctx_->tuned.find(tune_key(s, a.trans ? 1 : 0, b.trans ? 1 : 0));
      if (tuned != ctx_->tuned.end() && k::gemm_tile_valid(dtype_, tuned->second.tile, s.mode))
        s.cfg = tuned->second;
      // room for every candidate the autotuner may pick
      const size_t pb = std::max(gemm_max_partial(s), k::gemm_partial_bytes(dtype_, s.cfg, m, n));
      if (pb) {
        s.partial = work(int64_t(pb));
        s.partial_cap = int64_t(pb);
      }
      s.name = syrk ? "syrk" : "gemm";
      if (s.precision == 1) s.name += "_bf16x3";
      if (s.precision == 2) s.name += "_bf16x6";
      if (syrk) {
        s.flops = double(n) * double(n + 1) * double(kk);
        s.bytes = double(esz_) * (double(n) * kk + double(n) * n);
      } else {
        s.flops = 2.0 * double(m) * double(n) * double(kk);
        s.bytes = double(esz_) * (double(m) * kk + double(kk) * n + double(m) * n);
      }
    }
    steps_.push_back(s);
  }

  // ------------------------------------------------------------------ solves
  // Low-precision LU (FP32 storage; FP32, FP16-MFMA or split-BF16 trailing
  // updates) and FP64 iterative refinement of an FP64 system.
  void refined_solve(const View& s, const View& b, const View& x) {
    const int64_t n = s.rows, r = b.cols;
    if (b.trans || x.trans) {
      fail(HEXLA_E_UNSUPPORTED, "internal: transposed solve operand");
      return;
    }
    Step q;
    q.kind = StepKind::IrSolve;
    q.dtype = dtype_;
    q.A = s;
    q.B = b;
    q.C = x;
    q.n = n;
    q.nrhs = r;
    IrWork& w = q.ir;
    w.s_low = work(n * n * 4);
    w.rowid = work(n * 4);
    w.luwork = work(int64_t(k::lu_workspace_bytes(HEXLA_F32, n, r)));
    w.r64 = work(n * r * 8);
    w.r_low = work(n * r * 4);
    w.d_low = work(n * r * 4);
    w.scratch = work(int64_t(k::norm_scratch_elems(n)) * 8);
    w.norms = work(4 * 8);
    w.res_cfg = k::gemm_choose(HEXLA_F64, 0, 0, n, r, n);
    // the residual's product has an n x nrhs result: about four workgroups
    // per CU of K splits instead of one (8192^2 x 64: 287 -> 200 us)
    w.res_cfg.split = k::gemm_split_for(HEXLA_F64, w.res_cfg.tile, 0, n, r, n, 1024, 8);
    const size_t pb = k::gemm_partial_bytes(HEXLA_F64, w.res_cfg, n, r);
    if (pb) w.partial = work(int64_t(pb));
    w.update_precision = o_.solve_precision == HEXLA_SOLVE_IR_FP16     ? k::GEMM_F16
                         : o_.solve_precision == HEXLA_SOLVE_IR_BF16X3 ? k::GEMM_BF16X3
                         : o_.solve_precision == HEXLA_SOLVE_IR_BF16X6 ? k::GEMM_BF16X6
                                                                       : k::GEMM_PLAIN;
    w.panel_fp64 = o_.solve_precision != HEXLA_SOLVE_IR_FP32;
    w.max_iter = o_.ir_max_iter;
    w.tol_scale = o_.ir_tol_scale;
    q.name = o_.solve_precision == HEXLA_SOLVE_IR_FP16     ? "lu_solve_ir_fp16"
             : o_.solve_precision == HEXLA_SOLVE_IR_BF16X3 ? "lu_solve_ir_bf16x3"
             : o_.solve_precision == HEXLA_SOLVE_IR_BF16X6 ? "lu_solve_ir_bf16x6"
                                                           : "lu_solve_ir_fp32";
    // LU + first solve; each refinement step adds a residual and a solve
    q.flops = 2.0 / 3.0 * double(n) * n * n + 2.0 * double(n) * n * r;
    q.bytes = double(n) * n * (8 + 2 * 4) + double(n) * r * 8 * 2;
    steps_.push_back(q);
  }

  // A product X X^T or X^T X of one stored matrix (the symmetric rank-k
  // update of Sec. II) with a positive scale: symmetric positive
  // semidefinite by construction (definite when X has full rank).
  bool gram_product(uint32_t n) const {
    if (!o_.syrk) return false;
    const Node& x = N(n);
    if (x.scalar || x.kind != NK_BINARY || x.op != HEXLA_OP_TIMES) return false;
    std::vector<Factor> f;
    double alpha = 1.0;
    flatten(n, false, f, alpha);
    return f.size() == 2 && f[0].kind == 0 && f[1].kind == 0 && alpha > 0.0 &&
           same_storage(f[0].v, f[1].v) && f[0].v.trans != f[1].v.trans;
  }

  void solve(const View& s, const View& b, const View& x, bool spd = false) {
    if (s.rows > k::kLuMaxN)
      return (void)fail(HEXLA_E_UNSUPPORTED,
                        "solve: n > " + std::to_string(k::kLuMaxN) + " is not supported");
    if (dtype_ == HEXLA_F64 && o_.solve_precision != HEXLA_SOLVE_PLAIN) return refined_solve(s, b, x);
    const int64_t n = s.rows, r = b.cols;
    if (b.trans || x.trans) {
      fail(HEXLA_E_UNSUPPORTED, "internal: transposed solve operand");
      return;
    }
    View lu = temp(n, n);
    EwHost copy;
    if (!compile(add_view(s), copy, false)) return;
    if (o_.solve_structure == 0 && o_.planner != HEXLA_PLANNER_NAIVE) {
      // the solver is chosen when the plan runs, from the matrix itself
      Step q;
      q.kind = StepKind::StructSolve;
      q.dtype = dtype_;
      q.name = spd ? "solve_spd" : "solve_structured";
      q.A = s;
      q.out = lu;
      q.ew = copy;
      q.B = b;
      q.C = x;
      q.n = n;
      q.nrhs = r;
      q.spd_known = spd;
      q.rowid = work(n * 4);
      q.luwork = work(int64_t(k::lu_workspace_bytes(dtype_, n, r)));
      // the tridiagonal solver's rows, or the triangular solves' inverted
      // diagonal blocks and second buffer
      q.coef = work(std::max<int64_t>(6 * n * int64_t(esz_),
                                      int64_t(k::tri_solve_workspace_bytes(dtype_, n, r))));
      q.info = work(16 * 4);
      // the general case's work (LU and substitution); the structured
      // solvers do less
      q.flops = 2.0 / 3.0 * double(n) * n * n + 2.0 * double(n) * n * r;
      q.bytes = double(esz_) * (3.0 * double(n) * n + 2.0 * double(n) * r);
      steps_.push_back(q);
      return;
    }
    push_ew(copy, lu);
    Step f;
    f.kind = StepKind::LuFactor;
    f.dtype = dtype_;
    f.name = "lu_factor";
    f.A = lu;
    f.n = n;
    f.rowid = work(n * 4);
    f.luwork = work(int64_t(k::lu_workspace_bytes(dtype_, n, r)));
    f.flops = 2.0 / 3.0 * double(n) * n * n;
    f.bytes = 2.0 * double(esz_) * double(n) * n;
    steps_.push_back(f);
    Step q;
    q.kind = StepKind::LuSolve;
    q.dtype = dtype_;
    q.name = "lu_solve";
    q.A = lu;
    q.B = b;
    q.C = x;
    q.n = n;
    q.nrhs = r;
    q.rowid = f.rowid;
    q.luwork = f.luwork;  // the inverses of the diagonal blocks
    q.flops = 2.0 * double(n) * n * r;
    q.bytes = double(esz_) * (double(n) * n + 2.0 * double(n) * r);
    steps_.push_back(q);
  }

  View explicit_inverse(const View& s, const View* dest) {
    const int64_t n = s.rows;
    View id = temp(n, n);
    EwHost p;
    p.op[0] = k::EW_IDENT;
    p.n_instr = 1;
    p.ident = true;
    push_ew(p, id);
    View x = dest ? *dest : temp(n, n);
    solve(s, id, x);
    return x;
  }
};

// FNV-1a of a generated kernel's source: identifies the kernel a profile
// was taken on.
std::string source_hash(const std::string& src) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : src) {
    h ^= c;
    h *= 1099511628211ull;
  }
  char buf[17];
  std::snprintf(buf, sizeof buf, "%016llx", static_cast<unsigned long long>(h));
  return buf;
}

void json_view(std::ostringstream& js, const char* name, const View& v) {
  js << "\"" << name << "\":{\"rows\":" << v.rows << ",\"cols\":" << v.cols
     << ",\"trans\":" << (v.trans ? "true" : "false") << ",\"buf\":\""
     << (v.ref.buf == Buf::Leaf ? "leaf" : v.ref.buf == Buf::Work ? "work" : "out") << "\"";
  if (v.strided) js << ",\"strides\":[" << v.str_i << "," << v.str_j << "]";
  js << "}";
}

}  // namespace

std::string describe(const hexla_plan* p) {
  std::ostringstream js;
  js.precision(17);
  js << "{\"rows\":" << p->rows << ",\"cols\":" << p->cols << ",\"dtype\":\""
     << (p->dtype == HEXLA_F64 ? "f64" : "f32") << "\",\"planner\":\""
     << planner_name(p->opts.planner) << "\",\"workspace_bytes\":" << p->ws_bytes
     << ",\"flops\":" << p->flops << ",\"bytes\":" << p->bytes << ",\"chain_macs\":" << p->macs
     << ",\"steps\":[";
  for (size_t i = 0; i < p->steps.size(); ++i) {
    const Step& s = p->steps[i];
    if (i) js << ",";
    js << "{\"kernel\":\"" << s.name << "\",\"flops\":" << s.flops << ",\"bytes\":" << s.bytes;
    switch (s.kind) {
      case StepKind::Ew:
        js << ",\"instructions\":" << s.ew.n_instr << ",\"leaves\":" << s.ew.leaves.size()
           << ",\"generated\":" << (s.cg_fn ? "true" : "false") << ",\"source_hash\":\""
           << source_hash(s.cg_src) << "\",";
        json_view(js, "out", s.out);
        break;
      case StepKind::Gemv:
      case StepKind::Gemm:
        js << ",\"m\":" << s.m << ",\"n\":" << s.n << ",\"k\":" << s.kk << ",\"alpha\":" << s.alpha
           << ",\"epilogue\":" << (s.has_epi ? "true" : "false");
        if (s.kind == StepKind::Gemm)
          js << ",\"tile\":" << s.cfg.tile << ",\"split\":" << s.cfg.split;
        js << ",";
        json_view(js, "A", s.A);
        js << ",";
        json_view(js, "B", s.B);
        js << ",";
        json_view(js, "C", s.C);
        break;
      case StepKind::LuFactor:
        js << ",\"n\":" << s.n;
        break;
      case StepKind::LuSolve:
        js << ",\"n\":" << s.n << ",\"nrhs\":" << s.nrhs;
        break;
      case StepKind::DiagProd:
        js << ",\"n\":" << s.m << ",\"k\":" << s.kk << ",\"alpha\":" << s.alpha << ",";
        json_view(js, "A", s.A);
        js << ",";
        json_view(js, "B", s.B);
        break;
      case StepKind::EwSum:
        js << ",\"elements\":" << s.m * s.n << ",\"leaves\":" << s.ew.leaves.size()
           << ",\"alpha\":" << s.alpha;
        break;
      default:
        break;
    }
    js << "}";
  }
  js << "]";
  if (!p->learned_notes.empty()) {
    js << ",\"learned\":[";
    for (size_t i = 0; i < p->learned_notes.size(); ++i) js << (i ? "," : "") << p->learned_notes[i];
    js << "]";
  }
  js << "}";
  return js.str();
}

void leaf_range(const View& v, size_t esz, std::vector<Range>& out) {
  if (v.ref.buf != Buf::Leaf || !v.ref.ptr) return;
  if (v.strided) {  // a diagonal or broadcast: the storage it spans
    if (v.span <= 0) return;
    Range r;
    r.ptr = v.ref.ptr;
    r.bytes = uint64_t(v.span) * esz;
    r.ld = 0;
    out.push_back(r);
    return;
  }
  const int64_t rs = v.trans ? v.cols : v.rows, cs = v.trans ? v.rows : v.cols;
  if (rs == 0 || cs == 0) return;
  Range r;
  r.ptr = v.ref.ptr;
  r.bytes = uint64_t(((cs - 1) * v.ld + rs) * int64_t(esz));
  r.ld = v.ld;
  r.trans = v.trans;
  out.push_back(r);
}

}  // namespace hexla

using hexla::set_err;

extern "C" {

hexla_status hexla_plan_create(hexla_ctx* ctx, hexla_node root, const hexla_plan_opts* opts,
                               hexla_plan** out) {
  if (!ctx || !out) return HEXLA_E_INVALID_ARG;
  *out = nullptr;
  if (root >= ctx->nodes.size()) return set_err(ctx, HEXLA_E_INVALID_ARG, "plan: bad root node");
  hexla_plan_opts o;
  hexla_plan_opts_default(&o);
  if (opts) o = *opts;
  if (o.planner < 0 || o.planner > HEXLA_PLANNER_ROOFLINE || o.product_precision < 0 ||
      o.product_precision > HEXLA_PRODUCT_BF16X6 || o.solve_precision < 0 ||
      o.solve_precision > HEXLA_SOLVE_IR_BF16X6)
    return set_err(ctx, HEXLA_E_INVALID_ARG, "plan: bad options");
  if (o.ir_max_iter < 0) o.ir_max_iter = 30;  // 0: no refinement step
  hexla_plan* p = new hexla_plan();
  p->ctx = ctx;
  p->opts = o;
  hexla::Planner pl(ctx, o, p);
  const hexla_status st = pl.run(root);
  if (st != HEXLA_OK) {
    delete p;
    return st;
  }
  if (ctx->device >= 0) {  // plan time is the generated kernels' compile time
    (void)hipSetDevice(ctx->device);
    for (hexla::Step& s : p->steps)
      if (s.kind == hexla::StepKind::Ew && !s.cg_src.empty())
        s.cg_fn = hexla::codegen_get(ctx->device, s.cg_src, &s.cg_err);
  }
  const size_t esz = hexla::dtype_size(p->dtype);
  for (const hexla::Step& s : p->steps) {
    if (s.kind == hexla::StepKind::Ew) {
      for (const hexla::View& v : s.ew.leaves) hexla::leaf_range(v, esz, p->ew_leaf_ranges);
    } else if (s.kind == hexla::StepKind::EwSum) {
      // a sum writes one value: the output must not overlap what it reads
      for (const hexla::View& v : s.ew.leaves) hexla::leaf_range(v, esz, p->leaf_ranges);
    } else {
      hexla::leaf_range(s.A, esz, p->leaf_ranges);
      hexla::leaf_range(s.B, esz, p->leaf_ranges);
      if (s.has_epi)
        for (const hexla::View& v : s.ew.leaves) hexla::leaf_range(v, esz, p->leaf_ranges);
    }
  }
  ctx->plans.insert(p);
  *out = p;
  return HEXLA_OK;
}

hexla_status hexla_plan_get_info(const hexla_plan* p, hexla_plan_info* out) {
  if (!p || !p->ctx || !out) return HEXLA_E_INVALID_ARG;
  out->rows = p->rows;
  out->cols = p->cols;
  out->dtype = p->dtype;
  int n = 0;
  for (const hexla::Step& s : p->steps) {
    n += 1;
    if (s.kind == hexla::StepKind::Gemm && s.cfg.split > 1) n += 1;
  }
  out->n_steps = n;
  out->workspace_bytes = p->ws_bytes;
  out->flops = p->flops;
  out->bytes = p->bytes;
  out->chain_macs = p->macs;
  return HEXLA_OK;
}

hexla_status hexla_plan_describe(const hexla_plan* p, char* buf, size_t cap, size_t* needed) {
  if (!p || !p->ctx) return HEXLA_E_INVALID_ARG;
  const std::string js = hexla::describe(p);
  if (needed) *needed = js.size();
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), n);
    buf[n] = '\0';
  }
  return HEXLA_OK;
}

hexla_status hexla_plan_destroy(hexla_plan* p) {
  if (!p) return HEXLA_E_INVALID_ARG;
  if (p->ctx) p->ctx->plans.erase(p);
  delete p;
  return HEXLA_OK;
}

}  // extern "C"
