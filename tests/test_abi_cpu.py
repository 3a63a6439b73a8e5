"""Host-side tests of the C ABI on a dry-run context (no GPU): exports,
builder size checks, error codes and the planner's choices, with the chain
orders pinned against the oracle's brute force."""
import os
import re

import numpy as np
import pytest

import inputs
from oracle import chain
from paper_2502_03000_amd import hexla as hx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FAKE = 1 << 20  # dry-run leaves never dereference their pointers


def header_functions():
    text = open(os.path.join(ROOT, "include", "hexla.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hexla_status|const char\*)\s+(hexla_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(hx.lib, n), n


@pytest.fixture()
def ctx():
    return hx.Context(device=-1)


def leaf(ctx, rows, cols, dtype=hx.F64, ptr=None, ld=None):
    leaf.counter = getattr(leaf, "counter", 0) + 1
    p = ptr if ptr is not None else FAKE * leaf.counter
    return ctx.leaf_raw(p, rows, cols, ld or max(rows, 1), dtype)


def kernels(plan):
    return [s["kernel"] for s in plan.describe()["steps"]]


def test_small_chain_expression_plan(ctx):
    a, b, c = leaf(ctx, 400, 300), leaf(ctx, 400, 600), leaf(ctx, 600, 200)
    v, d, e = leaf(ctx, 200, 1), leaf(ctx, 300, 1), leaf(ctx, 300, 1)
    y = hx.trans(a) @ b @ c @ v + 0.5 * (d % e)
    p = ctx.plan(y)
    desc = p.describe()
    assert p.shape == (300, 1)
    assert kernels(p) == ["gemv_n", "gemv_n", "gemv_t"]
    assert desc["steps"][-1]["epilogue"] is True
    assert desc["chain_macs"] == 480_000
    assert p.workspace_bytes > 0
    naive = ctx.plan(y, planner="naive")
    assert naive.describe()["chain_macs"] == 300 * 400 * 600 + 300 * 600 * 200 + 300 * 200
    assert "elementwise" in kernels(naive)


def random_chain(ctx, dims, dtype=hx.F32):
    e = leaf(ctx, dims[0], dims[1], dtype)
    for i in range(1, len(dims) - 1):
        e = e @ leaf(ctx, dims[i], dims[i + 1], dtype)
    return e


@pytest.mark.parametrize("seed", range(12))
def test_dp_matches_brute_force_and_greedy_matches_rule(ctx, seed):
    dims = inputs.random_chain_dims(seed=100 + seed, count=1, lmin=3, lmax=8, lo=2, hi=300)[0]
    e = random_chain(ctx, dims)
    best, _ = chain.brute_force_min(list(dims))
    assert ctx.plan(e).describe()["chain_macs"] == best
    _, g = chain.greedy_smallest_result(list(dims))
    assert ctx.plan(e, planner="greedy").describe()["chain_macs"] == g
    l2r = chain.tree_cost(chain.left_to_right(len(dims) - 1), list(dims))
    assert ctx.plan(e, planner="naive").describe()["chain_macs"] == l2r


def test_fp32_chain_golden_costs(ctx):
    e = random_chain(ctx, [8192, 1024, 8192, 512, 4096, 64])
    p = ctx.plan(e)
    assert p.describe()["chain_macs"] == 1_476_395_008
    assert p.info.flops == pytest.approx(2 * 1_476_395_008)
    assert ctx.plan(e, planner="greedy").describe()["chain_macs"] == 4_999_610_368
    assert all(k == "gemm" for k in kernels(p))
    # right to left: every product has 64 columns
    assert all(s["n"] == 64 for s in p.describe()["steps"])


def test_symmetric_product_detected_by_identity(ctx):
    x = leaf(ctx, 1000, 64, hx.F32)
    p = ctx.plan(hx.trans(x) @ x)
    assert kernels(p) == ["syrk"]
    assert p.info.flops == 64 * 65 * 1000
    assert kernels(ctx.plan(x @ hx.trans(x))) == ["syrk"]
    # same values in another buffer are not the same matrix
    y = leaf(ctx, 1000, 64, hx.F32)
    assert kernels(ctx.plan(hx.trans(x) @ y)) == ["gemm"]
    # disabled, and not used by the naive planner
    assert kernels(ctx.plan(hx.trans(x) @ x, syrk=False)) == ["gemm"]
    assert kernels(ctx.plan(hx.trans(x) @ x, planner="naive")) == ["gemm"]
    # a cheaper order wins over the symmetric pair: X^T (X v)
    v = leaf(ctx, 64, 1, hx.F32)
    assert kernels(ctx.plan(hx.trans(x) @ x @ v)) == ["gemv_n", "gemv_t"]


def test_inverse_times_matrix_becomes_solve(ctx):
    s, b = leaf(ctx, 50, 50), leaf(ctx, 50, 3)
    # by default the solver is chosen from the matrix when the plan runs
    assert kernels(ctx.plan(hx.inv(s) @ b)) == ["solve_structured"]
    k = kernels(ctx.plan(hx.inv(s) @ b, solve_structure="general"))
    assert "lu_factor" in k and "lu_solve" in k
    assert k.count("elementwise") == 1  # the working copy of S only
    naive = kernels(ctx.plan(hx.inv(s) @ b, planner="naive"))
    assert naive.count("elementwise") == 2  # copy of S and the identity
    assert naive[-1] == "gemm"
    for opt in ("auto", "general"):
        p1 = ctx.plan(hx.inv(s) @ b, solve_structure=opt)
        p2 = ctx.plan(hx.solve(s, b), solve_structure=opt)
        assert kernels(p1) == kernels(p2)
        assert p1.info.flops == pytest.approx(2 / 3 * 50 ** 3 + 2 * 50 ** 2 * 3)


def test_solve_of_gram_product_plans_cholesky(ctx):
    """solve(A*A.t(), b), the call trace of Sec. IV: the symmetric product
    runs as SYRK and the planner knows the system is positive
    (semi)definite."""
    a, b = leaf(ctx, 300, 40), leaf(ctx, 300, 2)
    k = kernels(ctx.plan(hx.solve(a @ hx.trans(a), b)))
    assert k == ["syrk", "solve_spd"]
    c = leaf(ctx, 40, 300)
    assert kernels(ctx.plan(hx.solve(a @ c, b))) == ["gemm", "solve_structured"]
    assert kernels(ctx.plan(hx.inv(hx.trans(c) @ c) @ b)) == ["syrk", "solve_spd"]


def test_elementwise_fusion(ctx):
    a, b, c = leaf(ctx, 64, 64, hx.F32), leaf(ctx, 64, 64, hx.F32), leaf(ctx, 64, 64, hx.F32)
    y = 0.5 * hx.exp(-(a % a)) + b / c
    p = ctx.plan(y)
    assert kernels(p) == ["elementwise"]
    st = p.describe()["steps"][0]
    assert st["leaves"] == 3 and p.workspace_bytes == 0
    unfused = ctx.plan(y, fuse=False)
    assert len(kernels(unfused)) == 6  # %, neg, exp, scale, /, +
    assert unfused.workspace_bytes > 0


def test_long_elementwise_chain_is_one_pass(ctx):
    ls = [leaf(ctx, 10, 10) for _ in range(8)]
    e = ls[0]
    for i, x in enumerate(ls[1:]):
        e = e + x if i % 2 else e - x
    e = (e % ls[0]) / 3.0 + 2.0
    assert kernels(ctx.plan(e)) == ["elementwise"]


def test_builder_errors(ctx):
    a, b = leaf(ctx, 3, 4), leaf(ctx, 5, 6)
    with pytest.raises(hx.HexlaError) as ei:
        a @ b
    assert ei.value.status == hx.E_DIM
    with pytest.raises(hx.HexlaError) as ei:
        a + b
    assert ei.value.status == hx.E_DIM
    with pytest.raises(hx.HexlaError) as ei:
        hx.inv(a)
    assert ei.value.status == hx.E_NOT_SQUARE
    with pytest.raises(hx.HexlaError) as ei:
        hx.solve(a, leaf(ctx, 3, 1))
    assert ei.value.status == hx.E_NOT_SQUARE
    with pytest.raises(hx.HexlaError) as ei:
        leaf(ctx, 3, 3) + leaf(ctx, 3, 3, hx.F32)
    assert ei.value.status == hx.E_DTYPE
    with pytest.raises(hx.HexlaError) as ei:
        ctx.leaf_raw(FAKE, 10, 2, 5, hx.F64)
    assert ei.value.status == hx.E_INVALID_ARG
    with pytest.raises(hx.HexlaError) as ei:
        ctx.leaf_raw(0, 10, 2, 10, hx.F64)
    assert ei.value.status == hx.E_INVALID_ARG
    with pytest.raises(hx.HexlaError) as ei:
        ctx.plan(ctx.scalar(2.0) * 3.0)
    assert ei.value.status == hx.E_UNSUPPORTED
    p = ctx.plan(leaf(ctx, 3, 3) + 1.0)
    with pytest.raises(hx.HexlaError) as ei:
        p.execute(FAKE, None, ld_out=3)
    assert ei.value.status == hx.E_UNSUPPORTED


def test_plan_describes_transposed_views(ctx):
    a = leaf(ctx, 30, 20)
    p = ctx.plan(hx.trans(a) @ leaf(ctx, 30, 40))
    st = p.describe()["steps"][0]
    assert st["A"]["trans"] is True and st["m"] == 20 and st["k"] == 30 and st["n"] == 40


def test_row_vector_result_uses_gemv(ctx):
    a, x = leaf(ctx, 1, 50), leaf(ctx, 50, 70)
    p = ctx.plan(a @ x)
    assert kernels(p) == ["gemv_t"]
    assert p.shape == (1, 70)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with a message before it
    touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_plan_keeps_borrowed_tensors_alive_after_clear(ctx):
    """A plan holds the tensors its leaves borrow: clearing the context's
    nodes and dropping every other reference leaves them allocated."""
    import gc
    import weakref

    import torch
    a = torch.ones(64, 32, dtype=torch.float64)
    b = torch.ones(32, 16, dtype=torch.float64)
    refs = [weakref.ref(a), weakref.ref(b)]
    p = ctx.plan(ctx.leaf(a) @ ctx.leaf(b))
    ctx.clear()
    del a, b
    gc.collect()
    assert all(r() is not None for r in refs)
    del p
    gc.collect()
    assert all(r() is None for r in refs)


# ------------------------------- diagonals, traces and views (dry-run plans)

def test_diagonal_rewrites_plan_no_full_product(ctx):
    a, b = leaf(ctx, 300, 500), leaf(ctx, 500, 300)
    s, v, w = leaf(ctx, 300, 300), leaf(ctx, 300, 1), leaf(ctx, 300, 1)
    assert kernels(ctx.plan(hx.diag(a @ b))) == ["diag_product"]
    assert ctx.plan(hx.diag(a @ b)).shape == (300, 1)
    assert kernels(ctx.plan(hx.trace(a @ b))) == ["trace_product"]
    assert ctx.plan(hx.trace(a @ b)).shape == (1, 1)
    # expression (4): zeros, then the product's diagonal written onto them
    assert kernels(ctx.plan(hx.diagmat(a @ b))) == ["elementwise", "diag_product"]
    # expression (3): one element-wise pass scaling rows (matrix or vector diagonal)
    assert kernels(ctx.plan(hx.diagmat(s) @ a)) == ["elementwise"]
    assert kernels(ctx.plan(hx.diagmat(v) @ a)) == ["elementwise"]
    assert kernels(ctx.plan(b @ hx.diagmat(s))) == ["elementwise"]
    # expression (7): one multiply-and-sum pass
    p = ctx.plan(hx.trans(v) @ hx.diagmat(s) @ w)
    assert kernels(p) == ["sum"] and p.shape == (1, 1)
    # the naive planner forms the full product or the dense diagonal matrix
    assert "gemm" in kernels(ctx.plan(hx.diag(a @ b), planner="naive"))
    assert "gemm" in kernels(ctx.plan(hx.diagmat(s) @ a, planner="naive"))
    # traces and diagonals of element-wise values read only the diagonals
    p = ctx.plan(hx.trace(s + 2.0 * s))
    assert kernels(p) == ["sum"]
    assert kernels(ctx.plan(hx.diag(s % s) + v)) == ["elementwise"]
    # four factors: the split with the fewest multiply-adds, each side by the
    # DP: (A (B C)) and D, 3e6 + 3e6 + 300 * 20 (the diagonal of a 300 x 20
    # by 20 x 300 product) against 6.15e6 for A and (B C) D
    c = leaf(ctx, 300, 20)
    d = leaf(ctx, 20, 300)
    p = ctx.plan(hx.diag(a @ b @ c @ d))
    assert kernels(p) == ["gemm", "gemm", "diag_product"]
    assert p.describe()["chain_macs"] == 500 * 300 * 20 + 300 * 500 * 20 + 300 * 20


def test_strided_broadcast_copied_before_large_passes(ctx):
    """diagmat(S) * B reads S's diagonal (stride ld + 1) once per column of
    B: past 2^20 elements the plan first copies it into a contiguous column
    (one more element-wise step); small passes, and contiguous vectors, read
    it in place."""
    big_s, big_b = leaf(ctx, 2048, 2048), leaf(ctx, 2048, 1024)
    assert kernels(ctx.plan(hx.diagmat(big_s) @ big_b)) == ["elementwise", "elementwise"]
    p = ctx.plan(hx.diagmat(big_s) @ big_b)
    first = p.describe()["steps"][0]  # the copied diagonal, a 2048 x 1 temporary
    assert (first["out"]["rows"], first["out"]["cols"], first["out"]["buf"]) == (2048, 1, "work")
    assert kernels(ctx.plan(hx.diagmat(leaf(ctx, 2048, 1)) @ big_b)) == ["elementwise"]
    small_s, small_b = leaf(ctx, 300, 300), leaf(ctx, 300, 200)
    assert kernels(ctx.plan(hx.diagmat(small_s) @ small_b)) == ["elementwise"]
    # a multiply-and-sum over a strided diagonal read once is left alone
    v = leaf(ctx, 2048, 1)
    assert kernels(ctx.plan(hx.trans(v) @ hx.diagmat(big_s) @ v)) == ["sum"]


def test_submatrix_views(ctx):
    a, b = leaf(ctx, 40, 30), leaf(ctx, 20, 40)
    e = a.col(0) + hx.trans(b.row(1))
    assert e.shape == (40, 1)
    assert kernels(ctx.plan(e)) == ["elementwise"]
    # a view of a leaf feeds a product without a copy
    x = leaf(ctx, 30, 1)
    assert kernels(ctx.plan(a.submat(5, 0, 20, 30) @ x)) == ["gemv_n"]
    with pytest.raises(hx.HexlaError) as ei:
        a.submat(30, 0, 20, 1)
    assert ei.value.status == hx.E_DIM
    with pytest.raises(hx.HexlaError):
        a.col(30)


def _plan_roofline_time(plan, esz, peak):
    t = 0.0
    for s in plan.describe()["steps"]:
        m, n, k = s["m"], s["n"], s["k"]
        t += max(2.0 * m * n * k / peak, (m * k + k * n + m * n) * esz / 8e12)
    return t


@pytest.mark.parametrize("dtype,esz,peak", [(hx.F32, 4, 157.3e12), (hx.F64, 8, 78.6e12)])
def test_roofline_planner_matches_brute_force(ctx, dtype, esz, peak):
    """The roofline planner's bracketing has the oracle's brute-force
    minimum of summed roofline times (chains of 3-6 factors, dims
    log-uniform in [1, 8192])."""
    for dims in inputs.random_chain_dims(seed=77, count=40, lmin=3, lmax=6, lo=1, hi=8192):
        e = None
        for a, b in zip(dims[:-1], dims[1:]):
            x = leaf(ctx, a, b, dtype)
            e = x if e is None else e @ x
        p = ctx.plan(e, planner="roofline")
        want, _ = chain.brute_force_min_time(list(dims), esz, peak, 8e12)
        assert _plan_roofline_time(p, esz, peak) == pytest.approx(want, rel=1e-9), dims
        # never fewer multiply-adds than the DP's minimum
        assert p.describe()["chain_macs"] >= chain.brute_force_min(list(dims))[0]


def test_roofline_planner_golden_order(ctx):
    dims = [1, 4, 8192, 4]
    e = None
    for a, b in zip(dims[:-1], dims[1:]):
        x = leaf(ctx, a, b, hx.F32)
        e = x if e is None else e @ x
    first = ctx.plan(e, planner="roofline").describe()["steps"][0]
    assert (first["m"], first["k"], first["n"]) == (4, 8192, 4)
    assert ctx.plan(e).describe()["chain_macs"] == 65536
    assert ctx.plan(e, planner="roofline").describe()["chain_macs"] == 131088
