"""Batch plans on a dry-run context (no GPU): the per-instance program the
template compiles to, the algorithmic counts, and the creation-time checks."""
import numpy as np
import pytest

from paper_2502_03000_amd import hexla as hx

NAMES = ["A", "B", "v", "S", "b", "p", "q"]


def setup(t=4, dt=hx.F32):
    ctx = hx.Context(-1)
    L = {n: ctx.template_leaf(t, "matrix" if n in "ABS" else "vector", dt) for n in NAMES}
    return ctx, L


def fake(sizes):
    sizes = np.asarray(sizes, np.int64)
    ptrs = (np.arange(len(sizes) * 7, dtype=np.uint64).reshape(len(sizes), 7) + 1) << np.uint64(24)
    outs = (np.arange(len(sizes), dtype=np.uint64) + 1) << np.uint64(24)
    outs = outs + (np.uint64(1) << np.uint64(44))
    return sizes, ptrs, outs


def ops(desc):
    return [(o["op"], o["dst"], o.get("src"), o.get("leaf"), o.get("trans")) for o in desc["ops"]]


def batched(L):
    return hx.trans(L["A"]) * L["B"] * L["v"] + hx.solve(L["S"], L["b"]) + 2 * (L["p"] % L["q"])


def test_batched_expression_program():
    ctx, L = setup()
    sizes, ptrs, outs = fake([8, 512, 0, 100])
    d = ctx.batch(batched(L), [L[n] for n in NAMES], sizes, ptrs, outs).describe()
    # right-to-left matrix-vector products, then the solve, then one fused pass
    assert ops(d) == [("load", 0, None, 2, None), ("gemv", 1, 0, 1, 0), ("gemv", 0, 1, 0, 1),
                      ("load", 1, None, 4, None), ("solve", 1, 1, 3, None),
                      ("ew", -1, None, None, None)]
    assert d["out_slot"] == -1 and d["max_n"] == 512 and d["count"] == 4
    # flops: 2 GEMVs (2n^2 each), LU solve (2n^3/3 + 2n^2), 4 element-wise ops
    n = sizes.astype(np.float64)
    want = (2 * n**3 / 3 + 6 * n**2 + 4 * n).sum()
    assert d["flops"] == pytest.approx(want, rel=1e-12)
    # bytes: A, B, S once (n^2), v, b, p, q and the output (n), FP32
    assert d["bytes"] == pytest.approx(((3 * n**2 + 5 * n) * 4).sum(), rel=1e-12)


def test_forms_and_slot_reuse():
    ctx, L = setup()
    sizes, ptrs, outs = fake([10, 20])
    lv = [L[n] for n in NAMES]
    d = ctx.batch(-2 * L["A"] * hx.trans(L["B"]) * L["v"], lv, sizes, ptrs, outs).describe()
    assert ops(d) == [("load", 0, None, 2, None), ("gemv", 1, 0, 1, 1), ("gemv", 0, 1, 0, 0)]
    assert d["ops"][1]["alpha"] == -2 and d["out_slot"] == 0
    d = ctx.batch(L["p"] + L["q"], lv, sizes, ptrs, outs).describe()
    assert ops(d) == [("ew", -1, None, None, None)]
    d = ctx.batch(3 * (hx.inv(L["S"]) * L["b"]), lv, sizes, ptrs, outs).describe()
    assert [o[0] for o in ops(d)] == ["load", "solve", "ew"]
    d = ctx.batch(L["A"] * (L["v"] + 0.5 * L["b"]), lv, sizes, ptrs, outs).describe()
    assert [o[0] for o in ops(d)] == ["ew", "gemv"]


@pytest.mark.parametrize("bad", ["matrix_sum_factor", "matrix_result", "inv_of_trans"])
def test_unsupported_forms(bad):
    ctx, L = setup()
    sizes, ptrs, outs = fake([10])
    lv = [L[n] for n in NAMES]
    expr = {"matrix_sum_factor": (L["A"] + L["B"]) * L["v"],
            "matrix_result": L["A"] * L["B"],
            "inv_of_trans": hx.inv(hx.trans(L["S"])) * L["v"]}[bad]
    with pytest.raises(hx.HexlaError) as ei:
        ctx.batch(expr, lv, sizes, ptrs, outs)
    assert ei.value.status in (hx.E_UNSUPPORTED, hx.E_DIM)


def test_creation_checks():
    ctx, L = setup()
    lv = [L[n] for n in NAMES]
    sizes, ptrs, outs = fake([10, 513])
    with pytest.raises(hx.HexlaError) as ei:
        ctx.batch(batched(L), lv, sizes, ptrs, outs)
    assert ei.value.status == hx.E_UNSUPPORTED
    sizes, ptrs, outs = fake([10, 20, 30])
    o = outs.copy()
    o[2] = ptrs[1, 5] + np.uint64(4)  # inside instance 1's p
    with pytest.raises(hx.HexlaError) as ei:
        ctx.batch(batched(L), lv, sizes, ptrs, o)
    assert ei.value.status == hx.E_INVALID_ARG
    o = outs.copy()
    o[1] = o[0] + np.uint64(8)  # two outputs overlap
    with pytest.raises(hx.HexlaError):
        ctx.batch(batched(L), lv, sizes, ptrs, o)
    p = ptrs.copy()
    p[1, 3] = 0  # null S of a non-empty instance
    with pytest.raises(hx.HexlaError):
        ctx.batch(batched(L), lv, sizes, p, outs)
    with pytest.raises(hx.HexlaError):  # ld < n
        ctx.batch(batched(L), lv, sizes, ptrs, outs, lds=np.full((3, 7), 15))
    # shared inputs across instances are fine; n = 0 instances need no pointers
    p = ptrs.copy()
    p[:, 0] = p[0, 0]
    ctx.batch(batched(L), lv, sizes, p, outs)
    z = np.zeros_like(ptrs)
    ctx.batch(batched(L), lv, np.zeros(3, np.int64), z, np.zeros(3, np.uint64))
    # a template leaf missing from the list
    with pytest.raises(hx.HexlaError) as ei:
        ctx.batch(batched(L), lv[:-1], sizes, ptrs[:, :-1], outs)
    assert ei.value.status == hx.E_INVALID_ARG


def test_execute_on_dry_run_context_is_unsupported():
    ctx, L = setup()
    sizes, ptrs, outs = fake([10])
    bt = ctx.batch(batched(L), [L[n] for n in NAMES], sizes, ptrs, outs)
    with pytest.raises(hx.HexlaError) as ei:
        bt.execute(1 << 20)
    assert ei.value.status == hx.E_UNSUPPORTED


def test_product_features():
    f = hx.product_features(hx.F32, 0, 0, 0, 1, 1024, 64, 8192, 3, 4)
    assert f.shape == (32,) and f.dtype == np.float32
    assert f[7] == 1 and f[6] == 0 and f[10] == 1 and f[9] == 0  # FP32, tb
    assert f[12 + 3] == 1 and f[12:20].sum() == 1               # tile one-hot
    assert f[29] == 1                                            # split-K
    assert abs(f[0] - 10 / 13) < 1e-6 and abs(f[2] - 1.0) < 1e-6  # log2 m, log2 k scaled
    g = hx.product_features(hx.F64, 0, 1, 1, 0, 512, 512, 100, 0, 1)
    assert g[6] == 1 and g[8] == 1 and g[29] == 0 and 0 < g[25] <= 1
    with pytest.raises(hx.HexlaError):
        hx.product_features(hx.F64, 0, 0, 0, 0, 16, 16, 16, 4, 1)  # FP64 has 4 tiles


def test_learned_planner_without_model_is_dp():
    ctx = hx.Context(-1)
    import torch
    dims = [300, 20, 500, 10, 400]
    bufs = [torch.zeros(a * b, dtype=torch.float32) for a, b in zip(dims[:-1], dims[1:])]
    def chain(planner):
        ls = [ctx.leaf_raw(t.data_ptr(), a, b, a, hx.F32)
              for t, a, b in zip(bufs, dims[:-1], dims[1:])]
        e = ls[0]
        for x in ls[1:]:
            e = e @ x
        return ctx.plan(e, planner=planner).describe()
    d, l = chain("dp"), chain("learned")
    assert l["chain_macs"] == d["chain_macs"] and "learned" not in l
    assert [s["m"] for s in l["steps"]] == [s["m"] for s in d["steps"]]


def test_objects_outliving_their_context():
    """Destroying a context first detaches its plans and batch plans: they
    reject every call but destruction, in either order of release."""
    import ctypes as C
    ctx, L = setup()
    sizes, ptrs, outs = fake([8, 16])
    bt = ctx.batch(batched(L), [L[n] for n in NAMES], sizes, ptrs, outs)
    plan = ctx.plan(L["p"] % L["q"])
    info, binfo = hx.PlanInfo(), hx.BatchInfo()
    assert hx.lib.hexla_plan_get_info(plan.handle, C.byref(info)) == hx.OK
    assert hx.lib.hexla_ctx_destroy(ctx.handle) == hx.OK
    ctx.handle = None
    assert hx.lib.hexla_plan_get_info(plan.handle, C.byref(info)) == hx.E_INVALID_ARG
    assert hx.lib.hexla_batch_get_info(bt.handle, C.byref(binfo)) == hx.E_INVALID_ARG
    assert hx.lib.hexla_batch_set_config(bt.handle, 32, 256, 512) == hx.E_INVALID_ARG
    assert hx.lib.hexla_plan_destroy(plan.handle) == hx.OK
    assert hx.lib.hexla_batch_destroy(bt.handle) == hx.OK
    plan.handle = bt.handle = None
