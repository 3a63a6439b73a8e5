"""Structure-aware solves (expression (10) of Sec. III; the solve of the call
trace in Sec. IV) through the C ABI: the solver the library reports for each
kind of matrix, and the solution against the FP64 oracle (GEPP): normwise
within max(1e-12 (FP64) or 1e-5 (FP32), 10 cond(S) sqrt(n) u) -- a solve's
forward error grows with the condition number, whatever the solver -- and
the FP64 backward error ||B - S X|| / (||S|| ||X||) <= n u of the storage
type."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from paper_2502_03000_amd import hexla as hx
from parity import rel

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-12, np.float32: 1e-5}
U = {np.float64: 2.0 ** -53, np.float32: 2.0 ** -24}
SIZES = [1, 63, 64, 65, 200, 513]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def ctx():
    return hx.Context(0)


def matrix(kind, g, n, dt):
    """Well-conditioned matrices of each structure."""
    d = inputs.diag_dominant(g, n)
    if kind == "diagonal":
        s = np.diag(np.diag(d))
    elif kind == "lower":
        s = np.tril(d)
    elif kind == "upper":
        s = np.triu(d)
    elif kind == "tridiagonal":  # |diagonal| < |subdiagonal|: pivoting swaps most rows
        s = np.diag(g.uniform(-0.3, 0.3, n)) + np.diag(0.2 * g.standard_normal(n - 1) + 1.0, -1) \
            + np.diag(0.2 * g.standard_normal(n - 1) - 1.0, 1)
    elif kind == "spd":
        x = g.standard_normal((n, n))
        s = x @ x.T / n + np.eye(n)
    elif kind == "symmetric_indefinite":  # positive diagonal, a negative eigenvalue
        x = g.standard_normal((n, n))
        s = (x + x.T) / 2.0
        np.fill_diagonal(s, np.abs(np.diag(s)) + 0.1)
        s = s + 0.5 * np.diag(np.abs(g.standard_normal(n)))
        if n > 1 and np.linalg.eigvalsh(s).min() > 0:
            s[0, 1] = s[1, 0] = 10.0 * (abs(s[0, 0]) + abs(s[1, 1]))
    else:  # general
        s = d
    return np.asfortranarray(s.astype(dt))


EXPECT = {"diagonal": "diagonal", "lower": "lower", "upper": "upper",
          "tridiagonal": "tridiagonal", "spd": "cholesky", "symmetric_indefinite": "lu",
          "general": "lu"}


def bound(s64, dt):
    n = s64.shape[0]
    return max(TOL[dt], 10.0 * np.linalg.cond(s64) * np.sqrt(n) * U[dt])


def check_solution(got, s, b, dt):
    ref = oracle.evaluate("solve(S,B)", {"S": s, "B": b})
    assert rel(got, ref) <= bound(s.astype(np.float64), dt)
    s64, b64 = s.astype(np.float64), b.astype(np.float64)
    berr = np.linalg.norm(b64 - s64 @ got) / (np.linalg.norm(s64) * np.linalg.norm(got))
    assert berr <= s.shape[0] * U[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("kind", list(EXPECT))
@pytest.mark.parametrize("n", SIZES)
def test_solver_chosen_by_structure(ctx, dt, kind, n):
    if kind == "symmetric_indefinite" and n < 2:
        pytest.skip("a 1 x 1 positive matrix is definite")
    g = inputs.rng(3000 + 7 * n + len(kind))
    s = matrix(kind, g, n, dt)
    b = inputs.normal(g, n, 3, dt)
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    p = ctx.plan(hx.solve(es, eb))
    assert [st["kernel"] for st in p.describe()["steps"]] == ["solve_structured"]
    out = p.output()
    p.execute(out, p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.OK
    # a 1 x 1 matrix is diagonal whatever it was drawn as
    want = "diagonal" if n == 1 else EXPECT[kind]
    assert hx.SOLVERS[rep.solver] == want, (kind, n)
    check_solution(host(out), s, b, dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("kind", ["lower", "upper", "spd"])
def test_structured_solve_many_columns(ctx, dt, kind):
    """1030 right-hand sides: the triangular solves run as two groups of
    launches (1024 + 6 columns) on one exchange; L and L^T for the SPD
    matrix, one direction for the triangular ones."""
    n, nrhs = 130, 1030
    g = inputs.rng(3100 + len(kind))
    s = matrix(kind, g, n, dt)
    b = inputs.normal(g, n, nrhs, dt)
    p = ctx.plan(hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))))
    out = p.output()
    p.execute(out, p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.OK
    assert hx.SOLVERS[rep.solver] == EXPECT[kind]
    check_solution(host(out), s, b, dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("n,nrhs", [(300, 1), (257, 70), (1000, 5)])
def test_solve_of_gram_product(ctx, dt, n, nrhs):
    """solve(A*A.t(), b): SYRK, then a Cholesky the planner chose (no
    run-time analysis); also through the inverse rewrite."""
    g = inputs.rng(3100 + n)
    a = inputs.normal(g, n, 2 * n, dt)
    b = inputs.normal(g, n, nrhs, dt)
    ea, eb = ctx.leaf(dev(a)), ctx.leaf(dev(b))
    for e in (hx.solve(ea @ hx.trans(ea), eb), hx.inv(ea @ hx.trans(ea)) @ eb):
        p = ctx.plan(e)
        assert [st["kernel"] for st in p.describe()["steps"]] == ["syrk", "solve_spd"]
        out = p.output()
        p.execute(out, p.workspace())
        rep = ctx.sync()
        assert rep.status == hx.OK and hx.SOLVERS[rep.solver] == "cholesky"
        env = {"A": a, "B": b}
        ref = oracle.evaluate("solve(A*trans(A), B)", env)
        s64 = a.astype(np.float64) @ a.astype(np.float64).T
        # the FP32 product A A^T itself is rounded: k = 2n more roundings
        lim = bound(s64, dt) * (np.sqrt(2 * n) if dt == np.float32 else 1.0)
        assert rel(host(out), ref) <= lim


def test_singular_structured_systems(ctx):
    b = np.ones((6, 1))
    z = np.eye(6)
    z[3, 3] = 0.0
    for s, solver in [(z, "diagonal"), (np.triu(np.ones((6, 6))) - np.diag([0, 0, 0, 0, 1, 0]), "upper")]:
        p = ctx.plan(hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))))
        p.execute(p.output(), p.workspace())
        rep = ctx.sync()
        assert rep.status == hx.E_SINGULAR and hx.SOLVERS[rep.solver] == solver
    # a tridiagonal matrix whose elimination meets a zero pivot (rows 0 and 1
    # are equal)
    t = np.diag([1.0, 1.0, 3.0, 4.0]) + np.diag([1.0, 1.0, 1.0], 1) + np.diag([1.0, 1.0, 1.0], -1)
    t[1, 2] = 0.0
    t[0, 1], t[1, 0], t[1, 1] = 1.0, 1.0, 1.0
    p = ctx.plan(hx.solve(ctx.leaf(dev(t)), ctx.leaf(dev(np.ones((4, 1))))))
    p.execute(p.output(), p.workspace())
    rep = ctx.sync()
    assert hx.SOLVERS[rep.solver] == "tridiagonal" and rep.status == hx.E_SINGULAR


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [3, 70])
def test_tridiagonal_rows_of_every_scale(ctx, dt, nrhs):
    """Rows scaled by powers of two across most of the storage type's range
    (2^+-100 for FP32, 2^+-500 for FP64): products of two rows' entries
    would leave that range, so the elimination must keep them apart. Row
    scaling leaves the solution alone, so the bound takes the condition
    number of the unscaled matrix."""
    n = 300
    g = inputs.rng(3300 + nrhs)
    s0 = matrix("tridiagonal", g, n, np.float64)
    b0 = inputs.normal(g, n, nrhs)
    span = 100 if dt == np.float32 else 500
    rs = 2.0 ** np.round(g.uniform(-span, span, n))
    s = np.asfortranarray((rs[:, None] * s0).astype(dt))
    b = (rs[:, None] * b0).astype(dt)
    assert np.all(np.isfinite(s)) and np.count_nonzero(s) == np.count_nonzero(s0)
    p = ctx.plan(hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))))
    out = p.output()
    p.execute(out, p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.OK and hx.SOLVERS[rep.solver] == "tridiagonal"
    ref = oracle.evaluate("solve(S,B)", {"S": s0, "B": b0})
    assert rel(host(out), ref) <= max(TOL[dt], 10.0 * np.linalg.cond(s0) * np.sqrt(n) * U[dt])


@pytest.mark.slow
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_tridiagonal_full_size(ctx, dt):
    """The structured-solve workload's tridiagonal system at its own size (n =
    8192, B 8192 x 64; |diagonal| < |off-diagonals|, so that most steps swap
    rows): 128 tiles through the three waves' four LDS buffers. Checked
    against LAPACK's banded solver in FP64 (scipy; a textbook routine, not
    the oracle, whose dense GEPP takes minutes here) within 10 cond_1(S) u,
    and by the FP64 backward error <= n u."""
    import scipy.linalg
    n, r = 8192, 64
    g = inputs.rng(3400)
    dia = g.uniform(-0.3, 0.3, n)
    sub = 0.2 * g.standard_normal(n - 1) + 1.0
    sup = 0.2 * g.standard_normal(n - 1) - 1.0
    s = np.diag(dia) + np.diag(sub, -1) + np.diag(sup, 1)
    s = np.asfortranarray(s.astype(dt))
    b = inputs.normal(g, n, r, dt)
    ab = np.zeros((3, n))
    ab[0, 1:], ab[1], ab[2, :-1] = np.diag(s, 1), np.diag(s), np.diag(s, -1)
    ref = scipy.linalg.solve_banded((1, 1), ab, b.astype(np.float64))
    inv = scipy.linalg.solve_banded((1, 1), ab, np.eye(n))
    cond1 = np.abs(s.astype(np.float64)).sum(axis=0).max() * np.abs(inv).sum(axis=0).max()
    del inv
    p = ctx.plan(hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))))
    out = p.output()
    p.execute(out, p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.OK and hx.SOLVERS[rep.solver] == "tridiagonal"
    got = host(out)
    assert rel(got, ref) <= max(TOL[dt], 10.0 * cond1 * U[dt]), (rel(got, ref), cond1)
    s64, b64 = s.astype(np.float64), b.astype(np.float64)
    berr = np.linalg.norm(b64 - s64 @ got) / (np.linalg.norm(s64) * np.linalg.norm(got))
    assert berr <= n * U[dt]


def test_structured_solve_capture_rules(ctx):
    g = inputs.rng(3200)
    s, b = inputs.diag_dominant(g, 100), inputs.normal(g, 100, 2)
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    p = ctx.plan(hx.solve(es, eb))
    with pytest.raises(hx.HexlaError) as ei:
        p.capture(p.output(), p.workspace())
    assert ei.value.status == hx.E_UNSUPPORTED
    q = ctx.plan(hx.solve(es, eb), solve_structure="general")
    out, ws = q.output(), q.workspace()
    q.capture(out, ws)
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        q.replay()
        assert ctx.sync().status == hx.OK
        assert rel(host(out), oracle.evaluate("solve(S,B)", {"S": s, "B": b})) <= 1e-12
