"""Parity of the batched persistent evaluation with the FP64 oracle, per
instance (normwise relative error: 1e-5 for FP32 storage, 1e-12 for FP64).

The workload is the batched form's expression over instances drawn by
``inputs.batched_instances`` (square sizes log-uniform in [8, 512], S
diagonally dominant), plus sizes chosen to hit the kernel's edges: 1, the
panel widths and their neighbours, one 256-row block boundary and the 512
maximum; n = 0 instances write nothing.
"""
import numpy as np
import pytest
import torch

import inputs
import oracle
from paper_2502_03000_amd import hexla as hx

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-12, np.float32: 1e-5}
NAMES = ["A", "B", "v", "S", "b", "p", "q"]
EDGE_SIZES = [1, 2, 7, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 129, 255, 256, 257, 300, 511, 512]


def rel(got, ref):
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(np.asarray(got, np.float64) - ref)
    n = np.linalg.norm(ref)
    return d / n if n > 0 else d


def instance(g, n, dtype, permute=False):
    d = {"A": inputs.normal(g, n, n, dtype), "B": inputs.normal(g, n, n, dtype),
         "v": inputs.normal(g, n, 1, dtype), "S": inputs.diag_dominant(g, n, dtype),
         "b": inputs.normal(g, n, 1, dtype), "p": inputs.normal(g, n, 1, dtype),
         "q": inputs.normal(g, n, 1, dtype)}
    if permute:  # rows of a dominant matrix shuffled: GEPP must undo the shuffle
        d["S"] = np.asfortranarray(d["S"][g.permutation(n)])
    return d


def template(ctx, dt, t=4):
    A, B, S = (ctx.template_leaf(t, "matrix", dt) for _ in range(3))
    v, b, p, q = (ctx.template_leaf(t, "vector", dt) for _ in range(4))
    leaves = {"A": A, "B": B, "v": v, "S": S, "b": b, "p": p, "q": q}
    return leaves


def run_batch(ctx, expr_fn, insts, np_dt, autotune=False, config=None):
    tdt = torch.float64 if np_dt == np.float64 else torch.float32
    dt = hx.F64 if np_dt == np.float64 else hx.F32
    lv = template(ctx, dt)
    root = expr_fn(lv)
    sizes = np.array([d["A"].shape[0] for d in insts], dtype=np.int64)
    arena, ptrs = hx.pack_batch(insts, NAMES, tdt)
    out, optrs, offs = hx.output_arena(sizes, tdt)
    bt = ctx.batch(root, [lv[n] for n in NAMES], sizes, ptrs, optrs)
    ws = bt.workspace()
    if autotune:
        bt.autotune(ws, reps=1)
    if config is not None:
        bt.set_config(*config)
    bt.execute(ws)
    r = ctx.sync()
    host = out.cpu().numpy().astype(np.float64)
    res = [host[o:o + n] for o, n in zip(offs, sizes)]
    return bt, r, res, (arena, out, ws)


BATCHED = lambda L: hx.trans(L["A"]) * L["B"] * L["v"] + hx.solve(L["S"], L["b"]) + 2 * (L["p"] % L["q"])


def check(insts, res, expr, np_dt):
    worst = 0.0
    for i, (d, got) in enumerate(zip(insts, res)):
        ref = oracle.evaluate(expr, d)
        e = rel(got[:, None] if got.ndim == 1 else got, ref)
        worst = max(worst, e)
        assert e <= TOL[np_dt], f"instance {i} (n={d['A'].shape[0]}): {e:.3e}"
    return worst


@pytest.mark.parametrize("np_dt", [np.float32, np.float64])
def test_batched_expression_edges(np_dt):
    g = inputs.rng(4101)
    insts = [instance(g, n, np_dt) for n in EDGE_SIZES]
    ctx = hx.Context(0)
    bt, r, res, _ = run_batch(ctx, BATCHED, insts, np_dt)
    assert r.status == hx.OK
    print(f"worst {check(insts, res, inputs.BATCHED_EXPR, np_dt):.3e}")


# every compiled launch variant (LU panel width, threads), on a small grid
# (instances queue up) and on a full one
VARIANTS = [(np.float32, 32, 256), (np.float32, 64, 256), (np.float32, 16, 256),
            (np.float64, 16, 256), (np.float64, 8, 256)]


@pytest.mark.parametrize("np_dt,panel,threads", VARIANTS)
@pytest.mark.parametrize("grid", [5, 512])
def test_batched_every_variant(np_dt, panel, threads, grid):
    g = inputs.rng(4107)
    insts = [instance(g, n, np_dt, permute=(n % 2 == 1)) for n in EDGE_SIZES]
    ctx = hx.Context(0)
    bt, r, res, _ = run_batch(ctx, BATCHED, insts, np_dt, config=(panel, threads, grid))
    assert r.status == hx.OK
    info = bt.describe()
    assert (info["panel"], info["threads"], info["grid"]) == (panel, threads, grid)
    check(insts, res, inputs.BATCHED_EXPR, np_dt)


def test_batched_set_config_rejects():
    insts = [instance(inputs.rng(4108), 8, np.float32)]
    ctx = hx.Context(0)
    bt, r, _, _ = run_batch(ctx, BATCHED, insts, np.float32)
    for bad in [(12, 256, 512), (32, 100, 512), (32, 256, 0), (32, 256, 10 ** 6)]:
        with pytest.raises(hx.HexlaError):
            bt.set_config(*bad)


@pytest.mark.parametrize("np_dt", [np.float32, np.float64])
def test_batched_expression_generator(np_dt):
    insts = inputs.batched_instances(seed=4102, count=48, lo=8, hi=512, dtype=np_dt)
    ctx = hx.Context(0)
    bt, r, res, _ = run_batch(ctx, BATCHED, insts, np_dt, autotune=True)
    assert r.status == hx.OK
    info = bt.describe()
    assert info["count"] == 48 and info["max_n"] == max(d["A"].shape[0] for d in insts)
    check(insts, res, inputs.BATCHED_EXPR, np_dt)


@pytest.mark.parametrize("np_dt", [np.float32, np.float64])
def test_batched_pivoting(np_dt):
    g = inputs.rng(4103)
    insts = [instance(g, n, np_dt, permute=True) for n in [3, 17, 40, 100, 200, 513 - 1]]
    ctx = hx.Context(0)
    _, r, res, _ = run_batch(ctx, lambda L: hx.solve(L["S"], L["b"]), insts, np_dt)
    assert r.status == hx.OK
    check(insts, res, "solve(S,b)", np_dt)


def test_batched_pivoting_general_fp64():
    # Gaussian S (no dominance): pivots are data-dependent throughout
    g = inputs.rng(4104)
    insts = []
    for n in [5, 33, 64, 150, 320]:
        d = instance(g, n, np.float64)
        d["S"] = inputs.normal(g, n, n, np.float64)
        insts.append(d)
    ctx = hx.Context(0)
    _, r, res, _ = run_batch(ctx, lambda L: hx.inv(L["S"]) * L["b"], insts, np.float64)
    assert r.status == hx.OK
    for d, got in zip(insts, res):
        ref = oracle.evaluate("inv(S)*b", d)
        cond = np.linalg.cond(d["S"])
        assert rel(got[:, None], ref) <= 1e-15 * cond * d["S"].shape[0], cond


FORMS = [
    ("inv(S)*(A*v) - exp(-(p%q))/2",
     lambda L: hx.inv(L["S"]) * (L["A"] * L["v"]) - hx.exp(-(L["p"] % L["q"])) / 2),
    ("-2*A*trans(B)*v", lambda L: -2 * L["A"] * hx.trans(L["B"]) * L["v"]),
    ("A*v", lambda L: L["A"] * L["v"]),
    ("p + q/b", lambda L: L["p"] + L["q"] / L["b"]),
    ("3*(inv(S)*b)", lambda L: 3 * (hx.inv(L["S"]) * L["b"])),
    ("A*(v + 0.5*b)", lambda L: L["A"] * (L["v"] + 0.5 * L["b"])),
    ("trans(A)*solve(S, B*v) - p", lambda L: hx.trans(L["A"]) * hx.solve(L["S"], L["B"] * L["v"]) - L["p"]),
]


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_batched_forms(form):
    text, fn = form
    g = inputs.rng(4105)
    insts = [instance(g, n, np.float32) for n in [1, 9, 64, 130, 257]]
    insts[0]["b"] = np.abs(insts[0]["b"]) + 1.0  # divisor away from zero
    for d in insts:
        d["b"] = np.where(np.abs(d["b"]) < 0.1, 1.0, d["b"]).astype(np.float32)
    ctx = hx.Context(0)
    _, r, res, _ = run_batch(ctx, fn, insts, np.float32)
    assert r.status == hx.OK
    check(insts, res, text, np.float32)


def test_batched_empty_and_zero_sizes():
    g = inputs.rng(4106)
    insts = [instance(g, n, np.float32) for n in [0, 5, 0, 70]]
    ctx = hx.Context(0)
    _, r, res, (_, out, _) = run_batch(ctx, BATCHED, insts, np.float32)
    assert r.status == hx.OK
    check([insts[1], insts[3]], [res[1], res[3]], inputs.BATCHED_EXPR, np.float32)
    # an empty batch launches only the queue reset
    lv = template(ctx, hx.F32)
    bt = ctx.batch(BATCHED(lv), [lv[n] for n in NAMES], np.zeros(0, np.int64),
                   np.zeros((0, 7), np.uint64), np.zeros(0, np.uint64))
    bt.execute(bt.workspace())
    assert ctx.sync().status == hx.OK


def test_batched_singular_instance():
    g = inputs.rng(4107)
    insts = [instance(g, n, np.float64) for n in [6, 40, 9]]
    insts[1]["S"][:, 7] = 0.0
    ctx = hx.Context(0)
    _, r, res, _ = run_batch(ctx, lambda L: hx.solve(L["S"], L["b"]), insts, np.float64)
    assert r.status == hx.E_SINGULAR and r.singular_column == 1
    check([insts[0], insts[2]], [res[0], res[2]], "solve(S,b)", np.float64)
    assert ctx.sync().status == hx.OK  # cleared


def test_batched_graph_replay_matches_eager():
    insts = inputs.batched_instances(seed=4108, count=40, lo=8, hi=300, dtype=np.float32)
    ctx = hx.Context(0)
    bt, r, res, (arena, out, ws) = run_batch(ctx, BATCHED, insts, np.float32)
    eager = out.clone()
    written = torch.zeros_like(out, dtype=torch.bool)
    off = 0
    for d in insts:  # output_arena pads each n_i x 1 result to 64 entries
        n = d["A"].shape[0]
        written[off:off + n] = True
        off += -(-n // 64) * 64
    bt.capture(ws)
    for k in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        bt.replay()
        assert ctx.sync().status == hx.OK
        assert torch.equal(out[written], eager[written]), f"replay {k}"
        assert torch.isnan(out[~written]).all()
        _ = (arena[:1000] * 2).sum().item()  # unrelated eager work between replays


def test_batched_rejects_bad_inputs():
    ctx = hx.Context(0)
    lv = template(ctx, hx.F32)
    g = inputs.rng(4109)
    insts = [instance(g, n, np.float32) for n in [4, 600]]
    sizes = np.array([4, 600], np.int64)
    arena, ptrs = hx.pack_batch(insts, NAMES, torch.float32)
    out, optrs, _ = hx.output_arena(sizes, torch.float32)
    with pytest.raises(hx.HexlaError) as ei:
        ctx.batch(BATCHED(lv), [lv[n] for n in NAMES], sizes, ptrs, optrs)
    assert ei.value.status == hx.E_UNSUPPORTED
    # output aliasing an input
    bad = optrs.copy()
    bad[0] = ptrs[0, 2]
    with pytest.raises(hx.HexlaError) as ei:
        ctx.batch(BATCHED(lv), [lv[n] for n in NAMES], sizes[:1], ptrs[:1], bad[:1])
    assert ei.value.status == hx.E_INVALID_ARG
    # short workspace
    bt = ctx.batch(BATCHED(lv), [lv[n] for n in NAMES], sizes[:1], ptrs[:1], optrs[:1])
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(hx.HexlaError) as ei:
        bt.execute(small)
    assert ei.value.status == hx.E_INVALID_ARG
