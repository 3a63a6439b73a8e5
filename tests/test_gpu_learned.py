"""The learned cost model's kernels against the FP64 oracle network
(oracle.mlp), and the learned planner end to end.

Tolerances: FP32 kernels against FP64 definitions -- gradients 1e-4
(normwise relative, per layer), predictions 1e-5, one Adam step 1e-6
(relative to the parameter norm; the step is driven by the kernel's own
gradient, so this pins the update arithmetic alone).
"""
import time

import numpy as np
import pytest
import torch

import inputs
import oracle
from oracle import mlp
from paper_2502_03000_amd import hexla as hx
from paper_2502_03000_amd import learn
from parity import assert_close

pytestmark = pytest.mark.gpu

WIDTHS = [32, 64, 64, 64, 1]


def flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def unflat(v):
    out, off = [], 0
    for fi, fo in zip(WIDTHS[:-1], WIDTHS[1:]):
        w = v[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = v[off:off + fo]
        off += fo
        out.append((w.astype(np.float64), b.astype(np.float64)))
    return out


def rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (n if n > 0 else 1.0)


def setup(seed, n):
    g = inputs.rng(seed)
    params = [(w.astype(np.float32).astype(np.float64), b) for w, b in mlp.init(WIDTHS, g)]
    params = [(w, g.standard_normal(b.shape).astype(np.float32).astype(np.float64) * 0.1)
              for w, b in params]
    x = g.uniform(0.0, 1.0, (n, 32)).astype(np.float32)
    t = g.standard_normal(n).astype(np.float32)
    ctx = hx.Context(0)
    m = hx.Model.create(ctx, 0)
    m.set_params(flat(params))
    return ctx, m, params, x, t


@pytest.mark.parametrize("n", [1, 64, 200, 1000])
def test_gradient_matches_oracle(n):
    ctx, m, params, x, t = setup(5001 + n, n)
    g, loss = m.grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    y, cache = mlp.forward(params, x.astype(np.float64))
    ref = mlp.backward(params, cache, y, t.astype(np.float64))
    assert abs(loss - mlp.mse(y, t)) <= 1e-5 * mlp.mse(y, t)
    got = unflat(g)
    for l, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        assert rel(gw, rw) <= 1e-4, f"dW{l + 1}: {rel(gw, rw):.2e}"
        assert rel(gb, rb) <= 1e-4, f"db{l + 1}: {rel(gb, rb):.2e}"


def test_predict_matches_oracle_forward():
    ctx, m, params, x, t = setup(5002, 333)
    m.set_params(flat(params), y_mean=1.5, y_std=2.0)
    got = m.predict(torch.from_numpy(x).cuda()).cpu().numpy()
    y, _ = mlp.forward(params, x.astype(np.float64))
    assert rel(got, 1.5 + 2.0 * y) <= 1e-5


def test_adam_step_matches_oracle():
    ctx, m, params, x, t = setup(5003, 300)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    g, _ = m.grad(xt, tt)
    state = {}
    want = mlp.adam_step(params, unflat(g), state, lr=1e-2)
    for step in range(2):
        m.step(xt, tt, lr=1e-2)
        got, _, _ = m.params()
        if step == 0:
            assert rel(got, flat(want)) <= 1e-6
            g2, _ = m.grad(xt, tt)
            want = mlp.adam_step(want, unflat(g2), state, lr=1e-2)
    assert rel(got, flat(want)) <= 1e-6


def test_training_fits_a_smooth_function():
    g = inputs.rng(5004)
    x = g.uniform(0.0, 1.0, (4096, 32)).astype(np.float32)
    y = (2 * x[:, 0] + 3 * x[:, 1] * x[:, 2] - x[:, 3] + np.sin(3 * x[:, 4]) + 0.5 * x[:, 5] ** 2)
    ctx = hx.Context(0)
    m, loss = learn.train(ctx, x, y.astype(np.float32), epochs=150, batch=256, lr=2e-3)
    assert loss < 0.02, loss  # standardised MSE: R^2 > 0.98
    pred = m.predict(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.sqrt(np.mean((pred - y) ** 2)) < 0.15 * y.std()


def test_save_load_roundtrip(tmp_path):
    ctx, m, params, x, t = setup(5005, 100)
    m.set_params(flat(params), 0.25, 3.0)
    p = tmp_path / "model.txt"
    m.save(str(p))
    m2 = hx.Model.load(ctx, str(p))
    a, am, asd = m.params()
    b, bm, bsd = m2.params()
    assert np.array_equal(a, b) and am == bm and asd == bsd
    txt = p.read_text().replace("gfx950", "gfx942", 1)
    p.write_text(txt)
    with pytest.raises(hx.HexlaError):
        hx.Model.load(ctx, str(p))


def test_timing_log_records_every_candidate(tmp_path):
    ctx = hx.Context(0)
    log = tmp_path / "t.jsonl"
    learn.timing_sweep(ctx, [(256, 128, 512, 0, 1), (96, 200, 64, 1, 0)], str(log), reps=1)
    recs = learn.read_log(str(log))
    assert {(r["m"], r["n"], r["k"], r["ta"], r["tb"]) for r in recs} == {(256, 128, 512, 0, 1),
                                                                          (96, 200, 64, 1, 0)}
    assert all(r["us"] > 0 for r in recs) and len(recs) >= 8
    x, y = learn.dataset(recs)
    assert x.shape == (len(recs), 32) and np.isfinite(y).all()


def chain_leaves(ctx, dims, pool, off=0):
    leaves, mats = [], []
    for a, b in zip(dims[:-1], dims[1:]):
        t = pool[off:off + a * b].view(b, a).t()  # a x b, column-major
        leaves.append(ctx.leaf(t))
        mats.append(t)
        off += a * b
    e = leaves[0]
    for x in leaves[1:]:
        e = e @ x
    return e, mats


def plan_timed(ctx, e, planner):
    """The plan and its host planning time in ms (the learned planner's
    inference launch and its wait included)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = ctx.plan(e, planner=planner)
    return p, (time.perf_counter() - t0) * 1e3


def time_plan(p, reps=5):
    """Median over reps of one graph replay of the plan, in ms."""
    out, ws = p.output(), p.workspace()
    p.capture(out, ws)
    p.replay()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        p.replay()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), out


def test_learned_planner_end_to_end(tmp_path):
    """Trains on a shape sweep disjoint from the evaluation chains (seed
    2005), then plans held-out random chains (seed 1005) with and without the
    model. Every learned result matches the FP64 oracle; the DP check holds;
    planning and execution times are reported for both planners (total,
    per-chain geomean of the DP/learned ratio, win rate) and the learned
    plans execute no slower than the DP's in total."""
    ctx = hx.Context(0)
    log = tmp_path / "sweep.jsonl"
    learn.timing_sweep(ctx, learn.log_uniform_shapes(2005, 48, 16, 2048), str(log), reps=1)
    x, y = learn.dataset(learn.read_log(str(log)))
    model, loss = learn.train(ctx, x, y, epochs=150)
    assert loss < 0.2, loss
    ctx.set_model(model)
    chains = inputs.random_chain_dims(seed=1005, count=24, lmin=3, lmax=6, lo=16, hi=2048)
    pool = torch.randn(32 * 1024 * 1024, device="cuda")
    rows = []
    for dims in chains:
        e, mats = chain_leaves(ctx, dims, pool)
        env = {f"M{i}": m.cpu().numpy() for i, m in enumerate(mats)}
        text = "*".join(env)
        ref, mag = oracle.evaluate(text, env), oracle.magnitude(text, env)
        pd, plan_dp = plan_timed(ctx, e, "dp")
        pl, plan_ln = plan_timed(ctx, e, "learned")
        notes = pl.describe().get("learned")
        assert notes
        assert notes[0]["chosen"] == "dp" or notes[0]["macs_learned"] <= 2 * notes[0]["macs_dp"]
        ex_dp, _ = time_plan(pd)
        ex_ln, out = time_plan(pl)
        assert_close(out.cpu().numpy(), ref, mag, np.float32, sum(dims[1:-1]) + len(dims),
                     what=f"chain {dims}")
        rows.append((plan_dp, ex_dp, plan_ln, ex_ln))
        del pd, pl, out
        ctx.clear()
    r = np.array(rows)
    e2e_dp, e2e_ln = r[:, 0] + r[:, 1], r[:, 2] + r[:, 3]
    print(f"planning ms: dp {r[:, 0].sum():.3f}, learned {r[:, 2].sum():.3f}; "
          f"execution ms: dp {r[:, 1].sum():.3f}, learned {r[:, 3].sum():.3f}; "
          f"end to end ms: dp {e2e_dp.sum():.3f}, learned {e2e_ln.sum():.3f}")
    print(f"execution: geomean dp/learned {np.exp(np.mean(np.log(r[:, 1] / r[:, 3]))):.3f}, "
          f"learned faster on {np.mean(r[:, 3] < r[:, 1]):.0%} of chains; end to end: geomean "
          f"{np.exp(np.mean(np.log(e2e_dp / e2e_ln))):.3f}, learned faster on "
          f"{np.mean(e2e_ln < e2e_dp):.0%}")
    assert r[:, 3].sum() <= r[:, 1].sum()
