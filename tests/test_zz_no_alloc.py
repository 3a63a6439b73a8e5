"""The allocation-free entry point (hexla_execute_static) against
hexla_execute on the same plans: the same kernels on the same inputs, so the
results are bitwise equal, and both meet the oracle's tolerance. Two calls in
a row, the second on a smaller input; then the first again, over whatever the
second left in the shared scratch."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from paper_2502_03000_amd import hexla as hx
from parity import assert_close

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda").t()


def chain_plan(ctx, scale):
    dims = inputs.fp32_chain_dims(scale=scale)
    mats = inputs.fp32_chain(seed=1001, dims=dims)
    e = None
    for m in mats:
        x = ctx.leaf(dev(m))
        e = x if e is None else e @ x
    names = [f"M{i}" for i in range(len(mats))]
    env = dict(zip(names, mats))
    text = "*".join(names)
    return ctx.plan(e), oracle.evaluate(text, env), oracle.magnitude(text, env), sum(dims[1:-1]) + 5


def test_static_entry_point_matches_execute():
    ctx = hx.Context(0)
    assert hx.static_scratch_bytes() == 64 << 20
    runs = []
    for scale in (8, 16):  # the second call has the smaller input
        p, ref, mag, k = chain_plan(ctx, scale)
        assert 0 < p.workspace_bytes <= hx.static_scratch_bytes()
        want = p.output()
        p.execute(want, p.workspace())
        got = p.output()
        got.fill_(float("nan"))
        p.execute_static(got)
        assert ctx.sync().status == hx.OK
        assert torch.equal(got, want), f"scale {scale}"
        assert_close(got.cpu().numpy(), ref, mag, np.float32, k, what=f"scale {scale}")
        runs.append((p, want))
    # the first plan again, over the second call's leftovers in the scratch
    p, want = runs[0]
    again = p.output()
    p.execute_static(again)
    assert ctx.sync().status == hx.OK
    assert torch.equal(again, want)


def test_static_entry_point_small_expression_and_refined_solve():
    ctx = hx.Context(0)
    env = inputs.small_chain_expr(1000)
    L = {k: ctx.leaf(dev(v)) for k, v in env.items()}
    p = ctx.plan(hx.trans(L["A"]) @ L["B"] @ L["C"] @ L["v"] + 0.5 * (L["d"] % L["e"]))
    want, got = p.output(), p.output()
    p.execute(want, p.workspace())
    p.execute_static(got)
    assert ctx.sync().status == hx.OK
    assert torch.equal(got, want)
    # a refined solve (LU, norms and the correction loop in the scratch)
    s, _, _, _ = inputs.svd_matrix(91, 300, 300, 1e3)
    b = inputs.normal(inputs.rng(92), 300, 2)
    q = ctx.plan(hx.solve(ctx.leaf(dev(s)), ctx.leaf(dev(b))), solve_precision="ir_fp32")
    want, got = q.output(), q.output()
    q.execute(want, q.workspace())
    assert ctx.sync().status == hx.OK
    q.execute_static(got)
    assert ctx.sync().status == hx.OK
    assert torch.equal(got, want)
    ref = oracle.evaluate("solve(S,B)", {"S": s, "B": b})
    assert np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-12


def test_static_entry_point_rejects_large_workspace():
    ctx = hx.Context(0)
    n = 3000  # the LU working copy alone is 72 MB
    s = torch.eye(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, 1, dtype=torch.float64, device="cuda")
    p = ctx.plan(hx.solve(ctx.leaf(s), ctx.leaf(b)))
    assert p.workspace_bytes > hx.static_scratch_bytes()
    with pytest.raises(hx.HexlaError) as ei:
        p.execute_static(p.output())
    assert ei.value.status == hx.E_INVALID_ARG
    assert "static scratch" in ctx.last_error()
