"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: normwise relative Frobenius error against the oracle, 1e-12 for
FP64 storage and 1e-5 for FP32 storage, and beside it the componentwise error
scaled by the oracle's magnitude of the computation (|op(A)| |op(B)| for a
product) within K unit roundoffs, K the roundings on the longest path (k for
a length-k sum, one per element-wise operation, two for exp and division);
bitwise equality where the arithmetic is exact (small-integer inputs) or the
result is a copy (mirrored triangle). Solves: normwise error and the backward
error.
"""
import numpy as np
import pytest
import torch

import inputs
import oracle
from oracle import gepp
from paper_2502_03000_amd import hexla as hx
from parity import assert_close

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-12, np.float32: 1e-5}


def dev(a, dtype=None):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a[:, None]
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda")
    if dtype is not None:
        t = t.to(dtype)
    return t.t()  # column-major view


def host(t):
    return t.detach().to("cpu").numpy().astype(np.float64)


def rel(got, ref):
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(np.asarray(got, np.float64) - ref)
    n = np.linalg.norm(ref)
    return d / n if n > 0 else d


@pytest.fixture(scope="module")
def ctx():
    return hx.Context(0)


def leaves(ctx, env):
    return {k: ctx.leaf(dev(v)) for k, v in env.items()}


def run(ctx, expr, **opts):
    out = ctx.evaluate(expr, **opts)
    torch.cuda.synchronize()
    return host(out)


# ------------------------------------------------------------- small chain

@pytest.mark.parametrize("planner", ["dp", "greedy", "naive", "roofline"])
def test_small_chain_expression_fp64(ctx, planner):
    env = inputs.small_chain_expr(1000)
    ref = oracle.evaluate(inputs.SMALL_CHAIN_EXPR, env)
    L = leaves(ctx, env)
    y = hx.trans(L["A"]) @ L["B"] @ L["C"] @ L["v"] + 0.5 * (L["d"] % L["e"])
    got = run(ctx, y, planner=planner)
    assert got.shape == (300, 1)
    mag = oracle.magnitude(inputs.SMALL_CHAIN_EXPR, env)
    assert_close(got, ref, mag, np.float64, 400 + 600 + 200 + 8, what=planner)


# ------------------------------------------------------------- element-wise

@pytest.mark.parametrize("codegen", [True, False])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(1000, 37), (1, 1), (4097, 3), (5, 0), (333, 257)])
def test_elementwise_expression(ctx, dt, shape, codegen):
    env = inputs.fp32_elementwise(seed=7, n=shape[0], cols=shape[1], dtype=dt)
    ref = oracle.evaluate(inputs.ELEMENTWISE_EXPR, env)
    L = leaves(ctx, env)
    e = 0.5 * hx.exp(-(L["A"] % L["A"])) + L["B"] / L["C"]
    steps = ctx.plan(e, codegen=codegen).describe()["steps"]
    assert steps[0]["generated"] is codegen
    got = run(ctx, e, codegen=codegen)
    assert got.shape == shape
    if got.size:
        assert_close(got, ref, oracle.magnitude(inputs.ELEMENTWISE_EXPR, env), dt, 8)


def test_generated_and_interpreted_kernels_agree(ctx):
    g = inputs.rng(31)
    env = {k: inputs.normal(g, 513, 129, np.float32) for k in "ABC"}
    env["C"] = np.abs(env["C"]) + 1.0
    L = leaves(ctx, env)
    e = (L["A"] - 2.0 * L["B"]) % (L["C"] + L["A"]) / L["C"] - hx.exp(L["B"] / 4.0) + 1.5
    ref = oracle.evaluate("(A - 2*B) % (C + A) / C - exp(B/4) + 1.5", env)
    a = run(ctx, e, codegen=True)
    b = run(ctx, e, codegen=False)
    mag = oracle.magnitude("(A - 2*B) % (C + A) / C - exp(B/4) + 1.5", env)
    assert_close(a, ref, mag, np.float32, 12, norm_tol=1e-6, what="generated")
    assert_close(b, ref, mag, np.float32, 12, norm_tol=1e-6, what="interpreted")
    assert np.max(np.abs(a - b)) <= 4 * np.finfo(np.float32).eps * np.max(np.abs(ref))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_elementwise_strided_and_transposed_views(ctx, dt):
    g = inputs.rng(11)
    big = inputs.normal(g, 70, 90, dt)
    x = big[3:53, 5:45]           # 50 x 40 view, ld 70
    y = inputs.normal(g, 40, 50, dt)  # used transposed
    td = torch.float64 if dt == np.float64 else torch.float32
    tbig = dev(big, td)
    tx = tbig[3:53, 5:45]
    ty_rowmajor = torch.from_numpy(np.ascontiguousarray(y.T)).to("cuda")  # (50, 40) row-major
    ex = ctx.leaf(tx)
    ey = ctx.leaf(ty_rowmajor)    # binds as trans of a 40 x 50 column-major leaf
    got = run(ctx, 0.4 * ex + 0.6 * ey - hx.trans(ctx.leaf(dev(y, td))))
    env = {"X": x, "Y": y}
    ref = oracle.evaluate("0.4*X + 0.6*trans(Y) - trans(Y)", env)
    mag = oracle.magnitude("0.4*X + 0.6*trans(Y) - trans(Y)", env)
    assert_close(got, ref, mag, dt, 5)


def test_paper_fusion_example_in_place(ctx):
    g = inputs.rng(12)
    x, yv = inputs.normal(g, 100, 100), inputs.normal(g, 100, 100)
    tx, ty = dev(x), dev(yv)
    ref = oracle.evaluate("0.4*X + 0.6*Y", {"X": x, "Y": yv})
    e = 0.4 * ctx.leaf(tx) + 0.6 * ctx.leaf(ty)
    ctx.evaluate(e, out=tx)  # Z = X written over X: element-wise, so allowed
    torch.cuda.synchronize()
    assert_close(host(tx), ref, oracle.magnitude("0.4*X + 0.6*Y", {"X": x, "Y": yv}),
                 np.float64, 3, norm_tol=1e-15)


# ----------------------------------------------------------------- products

SHAPES = [(130, 70, 50), (2, 3, 4), (64, 64, 64), (257, 129, 33), (1000, 64, 3000), (17, 900, 5)]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("mnk", SHAPES)
def test_gemm_against_oracle(ctx, dt, ta, tb, mnk):
    m, n, k = mnk
    g = inputs.rng(m * 7 + n * 3 + k + ta * 2 + tb)
    a = inputs.normal(g, k, m, dt) if ta else inputs.normal(g, m, k, dt)
    b = inputs.normal(g, n, k, dt) if tb else inputs.normal(g, k, n, dt)
    expr = ("trans(A)" if ta else "A") + "*" + ("trans(B)" if tb else "B")
    ref = oracle.evaluate(expr, {"A": a, "B": b})
    ea, eb = ctx.leaf(dev(a)), ctx.leaf(dev(b))
    got = run(ctx, (hx.trans(ea) if ta else ea) @ (hx.trans(eb) if tb else eb))
    assert got.shape == (m, n)
    assert_close(got, ref, oracle.magnitude(expr, {"A": a, "B": b}), dt, k + 2)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_small_integer_chain_is_exact(ctx, dt):
    g = inputs.rng(13)
    dims = [70, 33, 129, 65, 17, 40] if dt == np.float64 else [50, 20, 30, 10]
    mats = [inputs.small_ints(g, dims[i], dims[i + 1], -4, 4, dt) for i in range(len(dims) - 1)]
    names = [f"M{i}" for i in range(len(mats))]
    ref = oracle.evaluate("*".join(names), dict(zip(names, mats)))
    e = None
    for m in mats:
        x = ctx.leaf(dev(m))
        e = x if e is None else e @ x
    for planner in ("dp", "greedy", "naive", "roofline"):
        got = run(ctx, e, planner=planner)
        assert np.array_equal(got, ref), planner


def test_fp32_chain_scaled(ctx):
    dims = inputs.fp32_chain_dims(scale=8)
    mats = inputs.fp32_chain(seed=1001, dims=dims)
    names = [f"M{i}" for i in range(len(mats))]
    ref = oracle.evaluate("*".join(names), dict(zip(names, mats)))
    e = None
    for m in mats:
        x = ctx.leaf(dev(m))
        e = x if e is None else e @ x
    got = run(ctx, e)
    mag = oracle.magnitude("*".join(names), dict(zip(names, mats)))
    assert_close(got, ref, mag, np.float32, sum(dims[1:-1]) + len(mats))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(1000, 96), (777, 130), (300, 1)])
def test_syrk_against_oracle(ctx, dt, shape):
    g = inputs.rng(shape[0] + shape[1])
    x = inputs.normal(g, *shape, dt)
    ref = oracle.evaluate("trans(X)*X", {"X": x})
    ex = ctx.leaf(dev(x))
    p = ctx.plan(hx.trans(ex) @ ex)
    assert [s["kernel"] for s in p.describe()["steps"]] == (["syrk"] if shape[1] > 1 else ["gemv_t"])
    got = run(ctx, hx.trans(ex) @ ex)
    assert np.array_equal(got, got.T)
    assert_close(got, ref, oracle.magnitude("trans(X)*X", {"X": x}), dt, shape[0] + 2, what="X'X")
    got2 = run(ctx, ex @ hx.trans(ex))
    assert np.array_equal(got2, got2.T)
    assert_close(got2, oracle.evaluate("X*trans(X)", {"X": x}),
                 oracle.magnitude("X*trans(X)", {"X": x}), dt, shape[1] + 2, what="XX'")


def test_syrk_equals_gemm_on_integers(ctx):
    g = inputs.rng(14)
    x = inputs.small_ints(g, 513, 70, -3, 3, np.float32)
    ex = ctx.leaf(dev(x))
    a = run(ctx, hx.trans(ex) @ ex)
    b = run(ctx, hx.trans(ex) @ ex, syrk=False)
    assert np.array_equal(a, b)
    assert np.array_equal(a, x.astype(np.float64).T @ x.astype(np.float64))


# ------------------------------------------------------------------- solves

@pytest.mark.parametrize("n", [1, 7, 64, 65, 200, 513])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_solve_and_inverse_rewrite(ctx, n, nrhs):
    g = inputs.rng(n * 10 + nrhs)
    s = inputs.diag_dominant(g, n)
    b = inputs.normal(g, n, nrhs)
    ref = oracle.evaluate("solve(S,B)", {"S": s, "B": b})
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    assert rel(run(ctx, hx.solve(es, eb)), ref) <= 1e-12
    assert rel(run(ctx, hx.inv(es) @ eb), ref) <= 1e-12
    # the naive mapping (explicit inverse, then a product) agrees within
    # the inverse's error
    assert rel(run(ctx, hx.inv(es) @ eb, planner="naive"), ref) <= 1e-10


@pytest.mark.parametrize("n,nrhs", [(513, 1), (513, 3), (1200, 2), (577, 70), (130, 1030)])
def test_blocked_solve_repeats(ctx, n, nrhs):
    """The one-launch blocked triangular solves exchange solved blocks as
    tagged 64-bit words: odd panel counts (513: 9 panels, 1200: 19), several
    16-column chunks (70 columns) and two groups of launches (1030 columns:
    1024 + 6 on the same exchange), each solved four times with the deferred
    status read after every run."""
    g = inputs.rng(n + 7 * nrhs)
    s = inputs.diag_dominant(g, n)
    b = inputs.normal(g, n, nrhs)
    ref = oracle.evaluate("solve(S,B)", {"S": s, "B": b})
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    for e in (hx.solve(es, eb), hx.inv(es) @ eb, hx.solve(es, eb), hx.inv(es) @ eb):
        out = ctx.evaluate(e)
        assert ctx.sync().status == hx.OK
        assert rel(host(out), ref) <= 1e-12


def test_solve_pivots_on_general_matrix(ctx):
    g = inputs.rng(15)
    n = 300
    s = inputs.normal(g, n, n)
    b = inputs.normal(g, n, 2)
    ref = gepp.solve(s, b)
    got = run(ctx, hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))))
    cond = np.linalg.cond(s)
    assert rel(got, ref) <= 4 * cond * 2.0 ** -52 * n ** 0.5
    r = np.linalg.norm(b - s @ got) / (np.linalg.norm(s) * np.linalg.norm(got))
    assert r <= n * 2.0 ** -52


def test_solve_pivots_on_general_matrix_many_panels(ctx):
    """19 panels of 64: each trailing update beyond the next panel's columns
    runs on a second stream while that panel is factored."""
    g = inputs.rng(17)
    n = 1200
    s = inputs.normal(g, n, n)
    b = inputs.normal(g, n, 2)
    ref = gepp.solve(s, b)
    got = run(ctx, hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))))
    cond = np.linalg.cond(s)
    assert rel(got, ref) <= 4 * cond * 2.0 ** -52 * n ** 0.5
    r = np.linalg.norm(b - s @ got) / (np.linalg.norm(s) * np.linalg.norm(got))
    assert r <= n * 2.0 ** -52


def test_chain_with_inverse(ctx):
    g = inputs.rng(16)
    s = inputs.diag_dominant(g, 40)
    a = inputs.normal(g, 40, 40)
    v = inputs.normal(g, 40, 1)
    ref = oracle.evaluate("A*inv(S)*A*v", {"S": s, "A": a, "v": v})
    es, ea, ev = ctx.leaf(dev(s)), ctx.leaf(dev(a)), ctx.leaf(dev(v))
    assert rel(run(ctx, ea @ hx.inv(es) @ ea @ ev), ref) <= 1e-12


def test_explicit_inverse(ctx):
    g = inputs.rng(17)
    s = inputs.diag_dominant(g, 40)
    ref = gepp.gauss_jordan_inverse(s)
    assert rel(run(ctx, hx.inv(ctx.leaf(dev(s)))), ref) <= 1e-12


def test_singular_matrix_is_reported_at_sync(ctx):
    s = np.eye(6)
    s[:, 3] = 0.0
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(np.ones((6, 1))))
    with pytest.raises(hx.HexlaError) as ei:
        ctx.evaluate(hx.solve(es, eb))
    assert ei.value.status == hx.E_SINGULAR
    assert ctx.sync().status == hx.OK  # cleared


# ------------------------------------------------------------ error paths

def test_workspace_and_alias_checks(ctx):
    a = dev(np.ones((64, 64)))
    b = dev(np.ones((64, 64)))
    ea, eb = ctx.leaf(a), ctx.leaf(b)
    p = ctx.plan(ea @ eb + ea)
    out = p.output()
    if p.workspace_bytes:
        small = torch.empty(p.workspace_bytes // 2, dtype=torch.uint8, device="cuda")
        with pytest.raises(hx.HexlaError) as ei:
            p.execute(out, small)
        assert ei.value.status == hx.E_INVALID_ARG
    p2 = ctx.plan(ea @ eb)
    with pytest.raises(hx.HexlaError) as ei:
        p2.execute(a, p2.workspace())
    assert ei.value.status == hx.E_INVALID_ARG


# ------------------------------------------------- tuning and graph replay

def test_autotune_keeps_results_and_fills_table(ctx, tmp_path):
    dims = inputs.fp32_chain_dims(scale=16)
    mats = inputs.fp32_chain(seed=1002, dims=dims)
    names = [f"M{i}" for i in range(len(mats))]
    ref = oracle.evaluate("*".join(names), dict(zip(names, mats)))
    e = None
    for m in mats:
        x = ctx.leaf(dev(m))
        e = x if e is None else e @ x
    p = ctx.plan(e)
    out, ws = p.output(), p.workspace()
    p.autotune(out, ws, reps=2)
    p.execute(out, ws)
    assert ctx.sync().status == hx.OK
    mag = oracle.magnitude("*".join(names), dict(zip(names, mats)))
    assert_close(host(out), ref, mag, np.float32, sum(dims[1:-1]) + len(mats))
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    lines = path.read_text().splitlines()
    assert len(lines) == len(mats) - 1 and all(l.startswith("gfx950 ") for l in lines)
    # a later plan of the same shapes takes the tuned configurations
    p2 = ctx.plan(e)
    assert [s["tile"] for s in p2.describe()["steps"]] == [s["tile"] for s in p.describe()["steps"]]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("m", [200, 201])
def test_every_fp32_tile_against_oracle(tmp_path, ta, tb, m):
    """Each FP32 tile (forced through the tuning table), without and with
    split-K, on a ragged product (m = 201: unaligned leading dimension, the
    scalar load path). A context of its own: its table holds one product."""
    ctx = hx.Context(0)
    g = inputs.rng(40 + 4 * ta + 2 * tb + m)
    n, k = 96, 700
    a = inputs.normal(g, k, m, np.float32) if ta else inputs.normal(g, m, k, np.float32)
    b = inputs.normal(g, n, k, np.float32) if tb else inputs.normal(g, k, n, np.float32)
    text = ("trans(A)" if ta else "A") + "*" + ("trans(B)" if tb else "B")
    ref = oracle.evaluate(text, {"A": a, "B": b})
    mag = oracle.magnitude(text, {"A": a, "B": b})
    ea, eb = ctx.leaf(dev(a)), ctx.leaf(dev(b))
    e = (hx.trans(ea) if ta else ea) @ (hx.trans(eb) if tb else eb)
    p = ctx.plan(e)
    out, ws = p.output(), p.workspace()
    p.autotune(out, ws, reps=1)  # learns the product's key for the table
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    target, key = path.read_text().split()[:2]
    for tile in range(8):
        for split in (1, 5, 12):
            path.write_text(f"{target} {key} {tile} {split}\n")
            ctx.tune_load(str(path))
            q = ctx.plan(e)
            assert q.describe()["steps"][0]["tile"] == tile
            out, ws = q.output(), q.workspace()
            q.execute(out, ws)
            assert ctx.sync().status == hx.OK
            assert_close(host(out), ref, mag, np.float32, k + 2, what=f"tile {tile} split {split}")


@pytest.mark.parametrize("sym", [False, True])
def test_every_fp64_tile_against_oracle(tmp_path, sym):
    """Each FP64 tile (forced through the tuning table), without and with
    split-K, on a ragged general product and on a ragged trans(A)*A (the
    symmetric-product mode: lower-triangle tiles, mirrored)."""
    ctx = hx.Context(0)
    g = inputs.rng(90 + sym)
    m, n, k = 201, 130, 700
    if sym:
        a = inputs.normal(g, k, n, np.float64)
        text, leaves = "trans(A)*A", {"A": a}
        ea = ctx.leaf(dev(a))
        e = hx.trans(ea) @ ea
    else:
        a, b = inputs.normal(g, m, k, np.float64), inputs.normal(g, k, n, np.float64)
        text, leaves = "A*B", {"A": a, "B": b}
        e = ctx.leaf(dev(a)) @ ctx.leaf(dev(b))
    ref = oracle.evaluate(text, leaves)
    mag = oracle.magnitude(text, leaves)
    for tile in range(4):
        for split in (1, 5):
            q = _force(ctx, tmp_path, e, tile, split)
            if sym:
                assert q.describe()["steps"][0]["kernel"] == "syrk"
            out, ws = q.output(), q.workspace()
            q.execute(out, ws)
            assert ctx.sync().status == hx.OK
            got = host(out)
            assert_close(got, ref, mag, np.float64, k + 2, norm_tol=1e-13,
                         what=f"tile {tile} split {split}")
            if sym:
                assert np.array_equal(got, got.T), (tile, split)


def _force(ctx, tmp_path, e, tile, split):
    """Plans `e` (one product) with the given tile and split through the tuning table."""
    p = ctx.plan(e)
    out, ws = p.output(), p.workspace()
    p.autotune(out, ws, reps=1)
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    target, key = path.read_text().split()[:2]
    path.write_text(f"{target} {key} {tile} {split}\n")
    ctx.tune_load(str(path))
    q = ctx.plan(e)
    st = q.describe()["steps"][0]
    assert (st["tile"], st["split"]) == (tile, split)
    return q


@pytest.mark.parametrize("dt,tile", [(np.float32, 2), (np.float32, 4), (np.float64, 0)])
def test_split_k_repeats_and_replays(tmp_path, dt, tile):
    """Split-K partials and their fixed-order reduction: repeated executions,
    graph replays and a workspace full of garbage all give the same bits
    (m = 300: a ragged last row of tiles)."""
    ctx = hx.Context(0)
    g = inputs.rng(77)
    m, n, k = 300, 130, 2000
    a, b = inputs.normal(g, m, k, dt), inputs.normal(g, k, n, dt)
    ref = oracle.evaluate("A*B", {"A": a, "B": b})
    mag = oracle.magnitude("A*B", {"A": a, "B": b})
    e = ctx.leaf(dev(a)) @ ctx.leaf(dev(b))
    q = _force(ctx, tmp_path, e, tile, 3)
    out, ws = q.output(), q.workspace()
    ws.fill_(255)  # the partials overwrite whatever the workspace held
    q.execute(out, ws)
    assert ctx.sync().status == hx.OK
    first = out.clone()
    assert_close(host(first), ref, mag, dt, k + 2)
    for _ in range(2):
        out.zero_()
        q.execute(out, ws)
        assert ctx.sync().status == hx.OK
        assert torch.equal(out, first)
    q.capture(out, ws)
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        q.replay()
        assert ctx.sync().status == hx.OK
        assert torch.equal(out, first)


def test_graph_replay_matches_eager(ctx):
    g = inputs.rng(32)
    a, b = inputs.normal(g, 300, 200, np.float32), inputs.normal(g, 200, 100, np.float32)
    c = inputs.normal(g, 300, 100, np.float32)
    ea, eb, ec = ctx.leaf(dev(a)), ctx.leaf(dev(b)), ctx.leaf(dev(c))
    p = ctx.plan(hx.exp(ea @ eb % ec) - 2.0 * ec)
    out, ws = p.output(), p.workspace()
    p.execute(out, ws)
    ctx.sync()
    eager = host(out)
    p.capture(out, ws)
    for _ in range(3):
        out.zero_()                      # eager work between replays
        torch.cuda.synchronize()
        p.replay()
        assert ctx.sync().status == hx.OK
        assert np.array_equal(host(out), eager)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("split", [5, 17, 32])
def test_split_k_reduction_waves(tmp_path, dt, split):
    """The reduction's quad path (m % 4 == 0): wave w of a workgroup sums the
    partials z = w, w + 4, ..., four at a time and then the rest, and the four
    wave sums are added in w order; split counts that leave the waves unequal
    shares (5), a remainder past the groups of four (17) and eight per wave
    (32), with a ragged last quad of workgroups (300 x 130 = 39000 elements,
    9750 quads: 152 full workgroups of 64 quads and a last one of 22)."""
    ctx = hx.Context(0)
    g = inputs.rng(78 + split)
    m, n, k = 300, 130, 2000
    a, b = inputs.normal(g, m, k, dt), inputs.normal(g, k, n, dt)
    ref = oracle.evaluate("A*B", {"A": a, "B": b})
    mag = oracle.magnitude("A*B", {"A": a, "B": b})
    e = ctx.leaf(dev(a)) @ ctx.leaf(dev(b))
    q = _force(ctx, tmp_path, e, 0, split)
    out, ws = q.output(), q.workspace()
    ws.fill_(255)
    q.execute(out, ws)
    assert ctx.sync().status == hx.OK
    assert_close(host(out), ref, mag, dt, k + 2, what=f"split {split}")
