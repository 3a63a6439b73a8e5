"""Diagonal partial products, traces, diagonal matrices and submatrix views
(expressions (2)-(5) and (7) of Sec. III) through the C ABI against the FP64
oracle: normwise 1e-12 (FP64) / 1e-5 (FP32) and componentwise within K unit
roundoffs of the oracle's magnitude (K: the contraction length plus the
roundings of the pass; a trace adds the length of its sum)."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from paper_2502_03000_amd import hexla as hx
from parity import assert_close

pytestmark = pytest.mark.gpu

DT = [np.float32, np.float64]


def dev(a):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def ctx():
    return hx.Context(0)


def run(ctx, e, **opts):
    out = ctx.evaluate(e, **opts)
    torch.cuda.synchronize()
    return host(out)


def operands(g, m, k, n, ta, tb, dt):
    a = inputs.normal(g, k, m, dt) if ta else inputs.normal(g, m, k, dt)
    b = inputs.normal(g, n, k, dt) if tb else inputs.normal(g, k, n, dt)
    return a, b


def product_text(ta, tb):
    return ("trans(A)" if ta else "A") + "*" + ("trans(B)" if tb else "B")


def product_expr(ctx, a, b, ta, tb):
    ea, eb = ctx.leaf(dev(a)), ctx.leaf(dev(b))
    return (hx.trans(ea) if ta else ea) @ (hx.trans(eb) if tb else eb)


SHAPES = [(300, 500, 300), (257, 1000, 130), (1, 7, 1), (64, 64, 64), (129, 65, 200),
          (100, 20000, 100)]


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("mkn", SHAPES)
def test_diag_of_product(ctx, dt, ta, tb, mkn):
    m, k, n = mkn
    g = inputs.rng(m + 3 * k + 7 * n + 2 * ta + tb)
    a, b = operands(g, m, k, n, ta, tb, dt)
    text = "diag(" + product_text(ta, tb) + ")"
    env = {"A": a, "B": b}
    e = hx.diag(product_expr(ctx, a, b, ta, tb))
    assert [s["kernel"] for s in ctx.plan(e).describe()["steps"]] == ["diag_product"]
    got = run(ctx, e)
    assert got.shape == (min(m, n), 1)
    assert_close(got, oracle.evaluate(text, env), oracle.magnitude(text, env), dt, k + 2)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1), (0, 1)])
@pytest.mark.parametrize("mkn", SHAPES)
def test_trace_of_product(ctx, dt, ta, tb, mkn):
    m, k, n = mkn
    g = inputs.rng(11 + m + 3 * k + 7 * n + 2 * ta + tb)
    a, b = operands(g, m, k, n, ta, tb, dt)
    text = "trace(" + product_text(ta, tb) + ")"
    env = {"A": a, "B": b}
    e = hx.trace(product_expr(ctx, a, b, ta, tb))
    got = run(ctx, e)
    assert got.shape == (1, 1)
    assert_close(got, oracle.evaluate(text, env), oracle.magnitude(text, env), dt,
                 k + min(m, n) + 2)
    # the naive evaluation (full product, then the diagonal's sum) agrees
    naive = run(ctx, e, planner="naive")
    assert_close(naive, oracle.evaluate(text, env), oracle.magnitude(text, env), dt,
                 k + min(m, n) + 2)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("mkn", [(300, 400, 300), (200, 50, 170)])
def test_diagmat_of_product(ctx, dt, mkn):
    """Expression (4): zeros off the diagonal, the product's diagonal on it;
    also written into an output with a larger leading dimension."""
    m, k, n = mkn
    g = inputs.rng(21 + m + k)
    a, b = operands(g, m, k, n, 0, 0, dt)
    env = {"A": a, "B": b}
    e = hx.diagmat(product_expr(ctx, a, b, 0, 0))
    p = ctx.plan(e)
    assert [s["kernel"] for s in p.describe()["steps"]] == ["elementwise", "diag_product"]
    ref = oracle.evaluate("diagmat(A*B)", env)
    mag = oracle.magnitude("diagmat(A*B)", env)
    got = run(ctx, e)
    assert_close(got, ref, mag, dt, k + 2)
    off = got.copy()
    off[np.arange(min(m, n)), np.arange(min(m, n))] = 0.0
    assert not off.any()
    td = torch.float64 if dt == np.float64 else torch.float32
    wide = torch.full((n, m + 5), 7.0, dtype=td, device="cuda").t()  # (m + 5) x n, ld m + 5
    out = wide[:m, :]
    p.execute(out, p.workspace())
    assert ctx.sync().status == hx.OK
    assert_close(host(out), ref, mag, dt, k + 2)
    assert torch.all(wide[m:, :] == 7.0)  # the rows past the view are untouched


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("arg", ["matrix", "column", "row"])
def test_diagmat_times_matrix(ctx, dt, side, arg):
    """Expression (3): diagmat(x) * B scales B's rows (B * diagmat(x) its
    columns) in one element-wise pass reading only x's diagonal."""
    g = inputs.rng(31 + (side == "left") + 2 * len(arg))
    n, c = 333, 210
    x = {"matrix": inputs.normal(g, n, n, dt), "column": inputs.normal(g, n, 1, dt),
         "row": inputs.normal(g, 1, n, dt)}[arg]
    b = inputs.normal(g, n, c, dt) if side == "left" else inputs.normal(g, c, n, dt)
    env = {"X": x, "B": b}
    text = "diagmat(X)*B" if side == "left" else "B*diagmat(X)"
    ex, eb = ctx.leaf(dev(x)), ctx.leaf(dev(b))
    e = hx.diagmat(ex) @ eb if side == "left" else eb @ hx.diagmat(ex)
    e = 2.0 * e
    assert [s["kernel"] for s in ctx.plan(e).describe()["steps"]] == ["elementwise"]
    got = run(ctx, e)
    ref, mag = oracle.evaluate("2*" + text, env), oracle.magnitude("2*" + text, env)
    assert_close(got, ref, mag, dt, 3)
    assert_close(run(ctx, e, planner="naive"), ref, mag, dt, n + 3)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("n", [1, 100, 5000, 300000])
def test_vector_diagmat_vector(ctx, dt, n):
    """Expression (7): a^T diagmat(B) c as one multiply-and-sum pass (B a
    vector here for the large sizes; a matrix's diagonal at n <= 5000)."""
    g = inputs.rng(41 + n)
    a, c = inputs.normal(g, n, 1, dt), inputs.normal(g, n, 1, dt)
    bm = inputs.normal(g, n, n, dt) if n <= 5000 else inputs.normal(g, n, 1, dt)
    env = {"a": a, "B": bm, "c": c}
    e = hx.trans(ctx.leaf(dev(a))) @ hx.diagmat(ctx.leaf(dev(bm))) @ ctx.leaf(dev(c))
    assert [s["kernel"] for s in ctx.plan(e).describe()["steps"]] == ["sum"]
    got = run(ctx, e)
    # for a vector B the oracle takes the equivalent a^T (B % c) (pinned
    # identity), which needs no dense n x n diagonal matrix
    text = "trans(a)*diagmat(B)*c" if n <= 5000 else "trans(a)*(B % c)"
    assert_close(got, oracle.evaluate(text, env), oracle.magnitude(text, env), dt, n + 4)


@pytest.mark.parametrize("dt", DT)
def test_diagonals_of_elementwise_values(ctx, dt):
    g = inputs.rng(51)
    s, t = inputs.normal(g, 400, 400, dt), inputs.normal(g, 400, 400, dt)
    v = inputs.normal(g, 400, 1, dt)
    env = {"S": s, "T": t, "v": v}
    es, et, ev = ctx.leaf(dev(s)), ctx.leaf(dev(t)), ctx.leaf(dev(v))
    for text, e, k in [("trace(S + 2*T)", hx.trace(es + 2.0 * et), 400 + 3),
                       ("diag(S % T) + v", hx.diag(es % et) + ev, 3),
                       ("trace(exp(S/4))", hx.trace(hx.exp(es / 4.0)), 400 + 4),
                       ("diag(trans(S)) - diag(T)", hx.diag(hx.trans(es)) - hx.diag(et), 2)]:
        assert_close(run(ctx, e), oracle.evaluate(text, env), oracle.magnitude(text, env), dt, k,
                     what=text)


@pytest.mark.parametrize("dt", DT)
def test_diag_of_longer_chains(ctx, dt):
    g = inputs.rng(61)
    dims = [300, 500, 300, 20, 300]
    mats = [inputs.normal(g, dims[i], dims[i + 1], dt) for i in range(4)]
    names = ["A", "B", "C", "D"]
    env = dict(zip(names, mats))
    L = [ctx.leaf(dev(m)) for m in mats]
    for text, e in [("diag(A*B*C*D)", hx.diag(L[0] @ L[1] @ L[2] @ L[3])),
                    ("trace(A*B*C*D)", hx.trace(L[0] @ L[1] @ L[2] @ L[3])),
                    ("3*trace(C*D)", 3.0 * hx.trace(L[2] @ L[3]))]:
        assert_close(run(ctx, e), oracle.evaluate(text, env), oracle.magnitude(text, env), dt,
                     500 + 300 + 20 + 300 + 4, what=text)


@pytest.mark.parametrize("dt", DT)
def test_paper_view_expression(ctx, dt):
    """Expression (2): C = A(:,1) + B(2,:)^T, read in place (the row through
    its stride, with an implicit transpose)."""
    g = inputs.rng(71)
    a, b = inputs.normal(g, 1000, 800, dt), inputs.normal(g, 600, 1000, dt)
    env = {"A": a, "B": b}
    ea, eb = ctx.leaf(dev(a)), ctx.leaf(dev(b))
    e = ea.col(0) + hx.trans(eb.row(1))
    assert [s["kernel"] for s in ctx.plan(e).describe()["steps"]] == ["elementwise"]
    text = "col(A, 0) + trans(row(B, 1))"
    assert_close(run(ctx, e), oracle.evaluate(text, env), oracle.magnitude(text, env), dt, 1)
    # submatrices as product operands and views of evaluated values
    x = inputs.normal(g, 300, 7, dt)
    env["X"] = x
    ex = ctx.leaf(dev(x))
    for text, e, k in [("submat(A, 10, 100, 500, 300)*X", ea.submat(10, 100, 500, 300) @ ex, 302),
                       ("trans(submat(B, 3, 5, 300, 200))*submat(A, 0, 0, 300, 9)",
                        hx.trans(eb.submat(3, 5, 300, 200)) @ ea.submat(0, 0, 300, 9), 302),
                       ("col(A + A, 7) % col(A, 3)", (ea + ea).col(7) % ea.col(3), 3)]:
        assert_close(run(ctx, e), oracle.evaluate(text, env), oracle.magnitude(text, env), dt, k,
                     what=text)
