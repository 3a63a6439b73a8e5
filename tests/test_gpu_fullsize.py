"""Parity at the workloads' full sizes, in the configurations the bench times.

The oracle cannot evaluate these results whole in seconds, so each test
checks what it can compute exactly at any size (same tolerances as the small
cases: normwise 1e-5 / 1e-12 and componentwise K unit roundoffs of the
oracle's magnitude):

* sampled rows, columns or entries, each computed by the oracle on the
  corresponding slice of the inputs (a row of a product is that row of the
  first factor times the rest, a column of an element-wise result depends
  only on that column of the operands);
* Freivalds' check, Y r against the oracle's M1 (M2 (... (M_L r))) for
  random r;
* closed forms of the SVD-built inputs (X^T X = V S^2 V^T; S^-1 B =
  V S^-1 U^T B);
* the FP64 backward error of a solve.
"""
import numpy as np
import pytest
import torch

import inputs
import oracle
from paper_2502_03000_amd import hexla as hx
from parity import SPLIT_TERM, assert_close, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda")
    if dtype is not None:
        t = t.to(dtype)
    return t.t()


def host(t):
    return t.detach().to("cpu").numpy().astype(np.float64)


def colmajor_host(t):
    """Host copy of a column-major device matrix as a Fortran-order array."""
    return np.asfortranarray(t.t().contiguous().cpu().numpy().T)


# ------------------------------------------------- FP32 chain, 5 factors

def test_fp32_chain_full_size():
    dims = inputs.FP32_CHAIN_DIMS
    mats = inputs.fp32_chain(seed=1001, dims=dims)
    ctx = hx.Context(0)
    e = None
    for m in mats:
        x = ctx.leaf(dev(m))
        e = x if e is None else e @ x
    p = ctx.plan(e)
    out, ws = p.output(), p.workspace()
    p.autotune(out, ws, reps=2)     # the tiles the bench runs
    p.execute(out, ws)
    assert ctx.sync().status == hx.OK
    got = host(out)
    assert got.shape == (dims[0], dims[-1])
    names = [f"M{i}" for i in range(len(mats))]
    env = dict(zip(names, mats))
    k = sum(dims[1:-1]) + len(mats)
    # sampled rows: row i of the chain is row i of M0 times the other factors
    g = inputs.rng(2101)
    rows = sorted({0, dims[0] - 1, *g.choice(dims[0], 14, replace=False).tolist()})
    renv = dict(env, M0=np.asfortranarray(mats[0][rows, :]))
    text = "*".join(names)
    assert_close(got[rows], oracle.evaluate(text, renv), oracle.magnitude(text, renv),
                 np.float32, k, what="sampled rows")
    # Freivalds: Y r against M0 (M1 (... (M4 r))) for two random r
    for t in range(2):
        r = inputs.normal(g, dims[-1], 1)
        fenv = dict(env, r=r)
        ftext = text + "*r"
        assert_close(got @ r, oracle.evaluate(ftext, fenv), oracle.magnitude(ftext, fenv),
                     np.float32, k, what=f"Freivalds {t}")


# ------------------------------------------- element-wise pass, 16384^2

def test_elementwise_full_size():
    env = inputs.fp32_elementwise_device(seed=1001, n=16384)
    ctx = hx.Context(0)
    L = {k: ctx.leaf(v) for k, v in env.items()}
    p = ctx.plan(0.5 * hx.exp(-(L["A"] % L["A"])) + L["B"] / L["C"])
    out, ws = p.output(), p.workspace()
    p.execute(out, ws)
    assert ctx.sync().status == hx.OK
    g = inputs.rng(2102)
    cols = sorted({0, 16383, *g.choice(16384, 62, replace=False).tolist()})
    idx = torch.tensor(cols, device="cuda")
    sub = {k: v.index_select(1, idx).cpu().numpy().astype(np.float64) for k, v in env.items()}
    got = out.index_select(1, idx).cpu().numpy()
    assert_close(got, oracle.evaluate(inputs.ELEMENTWISE_EXPR, sub),
                 oracle.magnitude(inputs.ELEMENTWISE_EXPR, sub), np.float32, 8)


# ------------------------------------- trans(X)*X, X 65536 x 2048 (SVD-built)

@pytest.fixture(scope="module")
def gram_inputs():
    out = {}
    for cond in (1e2, 1e4, 1e6):
        x, s, v = inputs.svd_matrix_device(1003, 65536, 2048, cond)
        out[cond] = (x, s, v)
    return out


SYRK_CASES = [("fp32", 1e4), ("fp64", 1e4), ("bf16x6", 1e4),
              ("bf16x3", 1e2), ("bf16x3", 1e4), ("bf16x3", 1e6)]


@pytest.mark.parametrize("form,cond", SYRK_CASES)
def test_syrk_full_size(gram_inputs, form, cond):
    x, s, v = gram_inputs[cond]
    ctx = hx.Context(0)
    leaf = x.double() if form == "fp64" else x
    ex = ctx.leaf(leaf)
    prec = form if form.startswith("bf16") else "plain"
    p = ctx.plan(hx.trans(ex) @ ex, product_precision=prec)
    assert p.describe()["steps"][0]["kernel"] == ("syrk" if prec == "plain" else f"syrk_{prec}")
    out, ws = p.output(), p.workspace()
    p.autotune(out, ws, reps=1)
    p.execute(out, ws)
    assert ctx.sync().status == hx.OK
    got = host(out)
    assert np.array_equal(got, got.T)
    # sampled columns: C[:, J] = X^T X[:, J]
    g = inputs.rng(2103)
    cols = sorted({0, 2047, *g.choice(2048, 30, replace=False).tolist()})
    xh = colmajor_host(x).astype(np.float64)
    env = {"X": xh, "Y": np.asfortranarray(xh[:, cols])}
    dt = np.float64 if form == "fp64" else np.float32
    assert_close(got[:, cols], oracle.evaluate("trans(X)*Y", env), oracle.magnitude("trans(X)*Y", env),
                 dt, 65536 + 2, norm_tol=None if prec == "plain" else (1e-5 if prec == "bf16x3" else 2e-6),
                 extra=SPLIT_TERM.get(prec, 0.0), what=form)
    # closed form V S^2 V^T of the unrounded X: X's FP32 rounding moves it by
    # about 2^-24 relative (normwise, sampled columns)
    closed = (v * s ** 2) @ v[cols].T
    assert rel(got[:, cols], closed) <= {"bf16x3": 1e-5, "bf16x6": 2e-6}.get(prec, 1e-6)


# ---------------------------------------- solve(S, B), S 8192^2 cond 1e3

@pytest.fixture(scope="module")
def solve_inputs():
    n, nrhs = 8192, 64
    s_dev, sv, v, u = inputs.svd_matrix_device(1004, n, n, 1e3, dtype=torch.float64, return_u=True)
    bh = inputs.normal(inputs.rng(1005), n, nrhs)
    closed = (v / sv[None, :]) @ (u.T @ bh)
    return s_dev, dev(bh), bh, closed


@pytest.mark.parametrize("form", ["plain", "ir_fp32", "ir_bf16x3", "ir_bf16x6", "ir_fp16"])
def test_solve_full_size(solve_inputs, form):
    s_dev, b_dev, bh, closed = solve_inputs
    ctx = hx.Context(0)
    p = ctx.plan(hx.solve(ctx.leaf(s_dev), ctx.leaf(b_dev)), solve_precision=form)
    out, ws = p.output(), p.workspace()
    p.execute(out, ws)
    rep = ctx.sync()
    got = host(out)
    err = rel(got, closed)
    print(f"{form}: status {rep.status}, {rep.ir_iterations} iterations, "
          f"backward error {rep.ir_backward_error:.2e}, error vs closed form {err:.2e}")
    assert rep.status == hx.OK
    assert err <= 1e-12


@pytest.mark.parametrize("form", ["plain", "ir_fp32"])
def test_solve_beyond_one_xcd(form):
    """n = 8448: 33 panel workgroups, more than one XCD holds (stride-1
    placement); a general matrix, so rows are interchanged throughout. FP64
    backward error ||B - S X|| / (||S|| ||X||) <= n u."""
    n = 8448
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2104)
    s_dev = torch.randn((n, n), generator=gen, device="cuda", dtype=torch.float64).t()
    b_dev = torch.randn((3, n), generator=gen, device="cuda", dtype=torch.float64).t()
    ctx = hx.Context(0)
    p = ctx.plan(hx.solve(ctx.leaf(s_dev), ctx.leaf(b_dev)), solve_precision=form)
    out, ws = p.output(), p.workspace()
    p.execute(out, ws)
    rep = ctx.sync()
    assert rep.status == hx.OK
    sh, bh, x = colmajor_host(s_dev), colmajor_host(b_dev), host(out)
    berr = np.linalg.norm(bh - sh @ x) / (np.linalg.norm(sh) * np.linalg.norm(x))
    print(f"{form}: backward error {berr:.2e}")
    assert berr <= n * 2.0 ** -53


# ------------------------------------------------ 10,000 batched instances

def test_batched_full_size():
    insts = inputs.batched_instances(seed=1003, count=10000, dtype=np.float32)
    names = ["A", "B", "v", "S", "b", "p", "q"]
    sizes = np.array([d["A"].shape[0] for d in insts], dtype=np.int64)
    arena, ptrs = hx.pack_batch(insts, names, torch.float32)
    ctx = hx.Context(0)
    L = {nm: ctx.template_leaf(4, "matrix" if nm in "ABS" else "vector", hx.F32) for nm in names}
    root = hx.trans(L["A"]) * L["B"] * L["v"] + hx.solve(L["S"], L["b"]) + 2 * (L["p"] % L["q"])
    out, optrs, offs = hx.output_arena(sizes, torch.float32)
    bt = ctx.batch(root, [L[nm] for nm in names], sizes, ptrs, optrs)
    ws = bt.workspace()
    bt.autotune(ws, reps=1)
    bt.capture(ws)
    bt.replay()
    assert ctx.sync().status == hx.OK
    got = out.cpu().numpy()
    g = inputs.rng(2105)
    order = np.argsort(sizes, kind="stable")
    sample = sorted({*order[:4].tolist(), *order[-4:].tolist(),
                     *g.choice(len(insts), 200, replace=False).tolist()})
    for i in sample:
        ref = oracle.evaluate(inputs.BATCHED_EXPR, insts[i])
        e = rel(got[offs[i]:offs[i] + sizes[i]], ref)
        assert e <= 1e-5, f"instance {i} (n={sizes[i]}): {e:.3e}"


# --------------------------------- learned planner chains, dims up to 8192

@pytest.fixture(scope="module")
def trained_ctx(tmp_path_factory):
    from paper_2502_03000_amd import learn
    ctx = hx.Context(0)
    log = tmp_path_factory.mktemp("sweep") / "sweep.jsonl"
    learn.timing_sweep(ctx, learn.log_uniform_shapes(2005, 48, 16, 8192), str(log), reps=1)
    x, y = learn.dataset(learn.read_log(str(log)))
    model, _ = learn.train(ctx, x, y, epochs=150)
    ctx.set_model(model)
    ctx._model = model
    return ctx


def test_learned_chains_full_size(trained_ctx):
    """The held-out chains (seed 1005) with the largest operands, planned by
    the learned planner, against the oracle: sampled rows and Freivalds'
    check."""
    ctx = trained_ctx
    chains = inputs.random_chain_dims(seed=1005, count=2000)
    size = [sum(a * b for a, b in zip(d[:-1], d[1:])) for d in chains]
    pick = [chains[i] for i in np.argsort(size)[-6:]]
    g = inputs.rng(2106)
    for dims in pick:
        mats, leaves = [], []
        for a, b in zip(dims[:-1], dims[1:]):
            t = torch.randn((b, a), device="cuda").t()
            mats.append(t)
            leaves.append(ctx.leaf(t))
        e = leaves[0]
        for x in leaves[1:]:
            e = e @ x
        p = ctx.plan(e, planner="learned")
        out, ws = p.output(), p.workspace()
        p.execute(out, ws)
        assert ctx.sync().status == hx.OK
        got = host(out)
        names = [f"M{i}" for i in range(len(mats))]
        env = {nm: colmajor_host(m) for nm, m in zip(names, mats)}
        text = "*".join(names)
        k = sum(dims[1:-1]) + len(mats)
        rows = sorted({0, dims[0] - 1, *g.choice(dims[0], min(6, dims[0]), replace=False).tolist()})
        renv = dict(env, M0=np.asfortranarray(env["M0"][rows, :]))
        assert_close(got[rows], oracle.evaluate(text, renv), oracle.magnitude(text, renv),
                     np.float32, k, what=f"{dims} rows")
        r = inputs.normal(g, dims[-1], 1)
        fenv = dict(env, r=r)
        assert_close(got @ r, oracle.evaluate(text + "*r", fenv), oracle.magnitude(text + "*r", fenv),
                     np.float32, k, what=f"{dims} Freivalds")
        del p, out, ws, mats, leaves, env
        ctx.clear()
        torch.cuda.empty_cache()
