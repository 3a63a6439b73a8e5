"""Precision form on the GPU: the bfloat16 split (bit-exact against the
oracle's round-to-nearest-even emulation), split-BF16 products (normwise
error against the FP64 oracle within the FP32-equivalent 1e-5 for x3 and
2e-6 for x6, and componentwise within the split's per-product term plus
k + 2 FP32 roundings of |op(A)| |op(B)|), and the mixed-precision solves
(normwise 1e-12 after refinement; outcome labels as the oracle's refinement
gives them)."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from oracle import bf16
from oracle import refine
from paper_2502_03000_amd import hexla as hx
from parity import SPLIT_TERM, assert_close

pytestmark = pytest.mark.gpu


def dev(a):
    a = np.asarray(a)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(got, ref):
    return np.linalg.norm(np.asarray(got) - ref) / np.linalg.norm(ref)


@pytest.fixture(scope="module")
def ctx():
    return hx.Context(0)


@pytest.mark.parametrize("terms", [2, 3])
def test_split_is_bit_exact(ctx, terms):
    g = inputs.rng(40)
    x = np.concatenate([
        (g.standard_normal(100000) * 10.0 ** g.integers(-30, 30, 100000)).astype(np.float32),
        np.array([0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 3.0e38, -1e-40, 6.1e-5], np.float32),
    ])
    parts = ctx.split_bf16(torch.from_numpy(x).cuda(), terms)
    torch.cuda.synchronize()
    ref = bf16.split(x, terms)
    for got, want in zip(parts, ref):
        got_bits = got.cpu().numpy().view(np.uint16)
        want_bits = (want.view(np.uint32) >> 16).astype(np.uint16)
        assert np.array_equal(got_bits, want_bits)


@pytest.mark.parametrize("prec,bound", [("bf16x3", 1e-5), ("bf16x6", 2e-6)])
@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_split_syrk_error(ctx, prec, bound, cond):
    x, u, s, v = inputs.svd_matrix(50 + int(np.log10(cond)), 4096, 256, cond, dtype=np.float32)
    ref = oracle.evaluate("trans(X)*X", {"X": x})
    ex = ctx.leaf(dev(x))
    p = ctx.plan(hx.trans(ex) @ ex, product_precision=prec)
    assert [st["kernel"] for st in p.describe()["steps"]] == [f"syrk_{prec}"]
    out = ctx.evaluate(hx.trans(ex) @ ex, product_precision=prec)
    got = host(out)
    assert np.array_equal(got, got.T)
    mag = oracle.magnitude("trans(X)*X", {"X": x})
    assert_close(got, ref, mag, np.float32, 4096 + 2, norm_tol=bound, extra=SPLIT_TERM[prec])
    # plain FP32 accumulation meets the FP32-equivalent tolerance too
    plain = host(ctx.evaluate(hx.trans(ex) @ ex))
    assert_close(plain, ref, mag, np.float32, 4096 + 2)


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("mnk", [(300, 200, 1000), (129, 257, 65), (64, 64, 4096)])
def test_split_gemm_against_oracle(ctx, ta, tb, mnk):
    m, n, k = mnk
    g = inputs.rng(m + 3 * n + 7 * k + 2 * ta + tb)
    a = inputs.normal(g, k, m, np.float32) if ta else inputs.normal(g, m, k, np.float32)
    b = inputs.normal(g, n, k, np.float32) if tb else inputs.normal(g, k, n, np.float32)
    expr = ("trans(A)" if ta else "A") + "*" + ("trans(B)" if tb else "B")
    ref = oracle.evaluate(expr, {"A": a, "B": b})
    ea, eb = ctx.leaf(dev(a)), ctx.leaf(dev(b))
    e = (hx.trans(ea) if ta else ea) @ (hx.trans(eb) if tb else eb)
    got3 = host(ctx.evaluate(e, product_precision="bf16x3"))
    got6 = host(ctx.evaluate(e, product_precision="bf16x6"))
    mag = oracle.magnitude(expr, {"A": a, "B": b})
    assert_close(got3, ref, mag, np.float32, k + 2, norm_tol=1e-5, extra=SPLIT_TERM["bf16x3"])
    assert_close(got6, ref, mag, np.float32, k + 2, norm_tol=2e-6, extra=SPLIT_TERM["bf16x6"])


@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-5), ("bf16x6", 2e-6)])
@pytest.mark.parametrize("syrk", [True, False])
@pytest.mark.parametrize("cols", [(150, 90), (152, 88)])
def test_split_family_every_split(tmp_path, prec, tol, syrk, cols):
    """The autotuner's split-K candidates of the split-BF16 family, each
    forced through the tuning table (split 1 writes C directly: mirrored for
    the symmetric product, through the transposed product otherwise; the
    others reduce partials, written as 16-byte stores when the row count is
    a multiple of 4), on ragged shapes. A context of its own: its table
    holds one product."""
    ctx = hx.Context(0)
    g = inputs.rng(62 + syrk)
    x = inputs.normal(g, 700, cols[0], np.float32)
    y = inputs.normal(g, 700, cols[1], np.float32)
    ex, ey = ctx.leaf(dev(x)), ctx.leaf(dev(y))
    if syrk:
        e, text = hx.trans(ex) @ ex, "trans(X)*X"
    else:
        e, text = hx.trans(ex) @ ey, "trans(X)*Y"
    ref = oracle.evaluate(text, {"X": x, "Y": y})
    mag = oracle.magnitude(text, {"X": x, "Y": y})
    p = ctx.plan(e, product_precision=prec)
    out, ws = p.output(), p.workspace()
    p.autotune(out, ws, reps=1)
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    target, key = path.read_text().split()[:2]
    for split in (1, 2, 4, 8, 16, 32):
        path.write_text(f"{target} {key} 0 {split}\n")
        ctx.tune_load(str(path))
        q = ctx.plan(e, product_precision=prec)
        assert q.describe()["steps"][0]["split"] == split
        out, ws = q.output(), q.workspace()
        q.execute(out, ws)
        assert ctx.sync().status == hx.OK
        assert_close(host(out), ref, mag, np.float32, 700 + 2, norm_tol=tol, extra=SPLIT_TERM[prec],
                     what=f"split {split}")


# ------------------------------------------------ mixed-precision solves

@pytest.mark.parametrize("form,cond", [("ir_fp32", 1e3), ("ir_bf16x3", 1e3), ("ir_bf16x6", 1e3),
                                       ("ir_fp16", 1e2)])
@pytest.mark.parametrize("n", [200, 513])
def test_refined_solve_reaches_fp64_accuracy(ctx, form, cond, n):
    s, u, sv, v = inputs.svd_matrix(60 + n, n, n, cond)
    b = inputs.normal(inputs.rng(61 + n), n, 3)
    ref = oracle.evaluate("solve(S,B)", {"S": s, "B": b})
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    p = ctx.plan(hx.solve(es, eb), solve_precision=form)
    assert p.describe()["steps"][-1]["kernel"] == "lu_solve_" + form
    out = p.output()
    p.execute(out, p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.OK
    assert 1 <= rep.ir_iterations <= 30
    assert rep.ir_backward_error <= n * 2.0 ** -53
    assert rel(host(out), ref) <= 1e-12
    if form == "ir_fp32":
        # the oracle's refinement on its own FP32 GEPP factors: same outcome,
        # iteration counts within one (the two FP32 factorisations round
        # differently)
        want = refine.refine(s, b)
        assert want["accepted"]
        assert abs(want["iterations"] - rep.ir_iterations) <= 1, (want["iterations"], rep.ir_iterations)
    # the inverse rewrite takes the same refined path
    got = host(ctx.evaluate(hx.inv(es) @ eb, solve_precision=form))
    assert rel(got, ref) <= 1e-12


def test_refined_solve_many_columns(ctx):
    """1030 right-hand sides: the low-precision triangular solves of every
    refinement step run as two groups of launches (1024 + 6 columns)."""
    n, nrhs = 130, 1030
    s, u, sv, v = inputs.svd_matrix(67, n, n, 1e3)
    b = inputs.normal(inputs.rng(68), n, nrhs)
    ref = oracle.evaluate("solve(S,B)", {"S": s, "B": b})
    p = ctx.plan(hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))), solve_precision="ir_fp32")
    out = p.output()
    p.execute(out, p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.OK
    assert 1 <= rep.ir_iterations <= 30
    assert rel(host(out), ref) <= 1e-12


@pytest.mark.parametrize("form", ["ir_fp32", "ir_bf16x3", "ir_bf16x6", "ir_fp16"])
@pytest.mark.parametrize("n", [200, 513])
def test_refined_solve_reports_divergence(ctx, form, n):
    """cond 1e9 is beyond what FP32 factors can refine (cond * 2^-24 > 1): the
    oracle's refinement does not accept its result, and the library raises
    the deferred E_NO_CONVERGENCE with the backward error it reached."""
    s, _, _, _ = inputs.svd_matrix(80 + n, n, n, 1e9)
    b = inputs.normal(inputs.rng(81 + n), n, 3)
    want = refine.refine(s, b)
    assert not want["accepted"], want["status"]
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    p = ctx.plan(hx.solve(es, eb), solve_precision=form)
    p.execute(p.output(), p.workspace())
    rep = ctx.sync()
    assert rep.status == hx.E_NO_CONVERGENCE
    assert rep.ir_backward_error > n * 2.0 ** -53
    print(f"{form} n={n}: oracle {want['status']} after {want['iterations']}, "
          f"library {rep.ir_iterations} iterations, backward error {rep.ir_backward_error:.2e}")


def test_refined_solve_reports_cap_and_singular(ctx):
    s, _, _, _ = inputs.svd_matrix(70, 100, 100, 1e4)
    b = inputs.normal(inputs.rng(71), 100, 1)
    es, eb = ctx.leaf(dev(s)), ctx.leaf(dev(b))
    with pytest.raises(hx.HexlaError) as ei:
        ctx.evaluate(hx.solve(es, eb), solve_precision="ir_fp32", ir_max_iter=0)
    assert ei.value.status == hx.E_NO_CONVERGENCE
    z = np.eye(8)
    z[:, 5] = 0.0
    with pytest.raises(hx.HexlaError) as ei:
        ctx.evaluate(hx.solve(ctx.leaf(dev(z)), ctx.leaf(dev(np.ones((8, 1))))), solve_precision="ir_fp32")
    assert ei.value.status == hx.E_SINGULAR
    p = ctx.plan(hx.solve(es, eb), solve_precision="ir_fp32")
    with pytest.raises(hx.HexlaError) as ei:
        p.capture(p.output(), p.workspace())
    assert ei.value.status == hx.E_UNSUPPORTED
