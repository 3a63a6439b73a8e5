"""Benchmark of the expression evaluator on one MI355X.

Workload (one step): the FP32-at-scale pair of expressions
  job 1  M1*M2*M3*M4*M5 with dims 8192x1024, 1024x8192, 8192x512, 512x4096,
         4096x64, entries N(0, 1/k)   (reordered by the DP planner: four GEMMs)
  job 2  0.5*exp(-(A%A)) + B/C over 16384 x 16384, A,B ~ N(0,1), C ~ U[1,2]
         (one fused element-wise pass)
Inputs are generated once, resident in HBM before timing. The value is the
whole step's algorithmic GFLOP/s; the same step in plain FP64 gives the
speedup of the chosen form, and every other configuration (the small FP64
expression, the symmetric product and solve forms, the batched form, the
learned planner) is summarized under "jobs". Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "expression GFLOP/s & % roofline, chosen form vs plain FP64 at stated error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, datasheet
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix, datasheet


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=16384, help="element-wise matrix size")
    ap.add_argument("--count", type=int, default=10000, help="instances (batched workload)")
    ap.add_argument("--chains", type=int, default=2000, help="random chains (learned workload)")
    ap.add_argument("--sweep", type=int, default=600, help="training shapes (learned workload)")
    ap.add_argument("--workload", default="expr",
                    choices=["expr", "small", "syrk", "solve", "batched", "learned", "diag",
                             "struct"],
                    help="expr: the FP32 chain + fused element-wise step, its plain-FP64 "
                         "leg and a summary of every other configuration (default); the "
                         "others print that configuration's own line")
    ap.add_argument("--quick", action="store_true",
                    help="expr workload: the FP32 step alone (no FP64 leg, no other jobs)")
    ap.add_argument("--reps", type=int, default=100, help="runs per median")
    ap.add_argument("--overlap", action="store_true",
                    help="expr workload: the chain's launches on a second stream beside the "
                         "element-wise pass")
    ap.add_argument("--forms", default="",
                    help="comma-separated subset of forms (syrk, solve; batched: batched_fp64, "
                         "plain_fp64_per_instance beside the FP32 launch, which always runs)")
    ap.add_argument("--no-tune", action="store_true", help="skip product autotuning")
    ap.add_argument("--tune-save", default="",
                    help="write the context's tuning table here after the run")
    ap.add_argument("--tune-load", default="",
                    help="read a tuning table before planning and skip autotuning (profiling "
                         "runs: the same configurations as the run that saved it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def cpu_baseline(chain_np, ew_host, ew_flops_per_elem, min_seconds=10.0):
    """The FP64 oracle, as it stands, on the host cores: the full chain job
    plus a column sample of the element-wise job, repeated until at least
    min_seconds of CPU work."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        threads = os.cpu_count() or 1
    names = [f"M{i}" for i in range(len(chain_np))]
    env = dict(zip(names, chain_np))
    t_chain = t_ew = 0.0
    reps = 0
    while t_chain + t_ew < min_seconds:
        t0 = time.perf_counter()
        oracle.evaluate("*".join(names), env)
        t_chain += time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.evaluate("0.5*exp(-(A%A)) + B/C", ew_host)
        t_ew += time.perf_counter() - t0
        reps += 1
    dims = [m.shape[0] for m in chain_np] + [chain_np[-1].shape[1]]
    from oracle import chain as ch
    chain_flops = 2.0 * ch.brute_force_min(dims)[0]
    ew_elems = ew_host["A"].size
    flops = reps * (chain_flops + ew_flops_per_elem * ew_elems)
    return {
        "value": flops / (t_chain + t_ew) / 1e9, "unit": "GFLOP/s", "cores": int(threads),
        "kind": "oracle",
        "sample": f"{reps} x (full 5-factor chain + element-wise job on a "
                  f"{ew_host['A'].shape[0]}x{ew_host['A'].shape[1]} column sample); "
                  f"chain {t_chain:.2f} s, element-wise {t_ew:.2f} s, float64 numpy",
    }


def profiled_traffic(source_hash):
    """HBM bytes per launch of the element-wise kernel from the committed
    rocprofv3 counter summary, if that summary was taken on this very kernel
    (same generated source); otherwise None."""
    import re
    path = os.path.join(ROOT, "profiles", "fused_elementwise_fp32_16384.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    h = re.search(r"source hash `([0-9a-f]+)`", text)
    t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if h and t and h.group(1) == source_hash:
        return int(t.group(1))
    return None


BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix, datasheet
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 matrix, datasheet


def time_plan(torch, p, out, ws, reps):
    p.capture(out, ws)
    p.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        p.replay()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_syrk(args, ctx, hx, torch, inputs):
    """trans(X)*X, X 65536 x 2048 FP32 built from an SVD with cond 1e4: each
    form timed (graph replay, HIP events) and its error stated against FP64."""
    rows, cols, cond = 65536, 2048, 1e4
    x, s, v = inputs.svd_matrix_device(1003, rows, cols, cond)
    x64 = x.double()
    xh = x.cpu().numpy().astype(np.float64)
    closed = (v * s ** 2) @ v.T                       # V S^2 V^T (unrounded X)
    g = inputs.rng(7)
    pairs = [(int(i), int(j)) for i, j in zip(g.integers(0, cols, 256), g.integers(0, cols, 256))]
    import oracle  # sampled entries of X^T X, one FP64 dot product each
    exact = np.array([oracle.evaluate("trans(a)*b", {"a": xh[:, i:i + 1], "b": xh[:, j:j + 1]})[0, 0]
                      for i, j in pairs])
    flops = float(cols) * (cols + 1) * rows
    forms = []
    for name, leaf, prec in [("fp64", x64, "plain"), ("fp32", x, "plain"),
                             ("bf16x3", x, "bf16x3"), ("bf16x6", x, "bf16x6")]:
        ex = ctx.leaf(leaf)
        p = ctx.plan(hx.trans(ex) @ ex, product_precision=prec)
        out, ws = p.output(), p.workspace()
        if not args.no_tune:
            p.autotune(out, ws, reps=2)
        ms = time_plan(torch, p, out, ws, max(args.steps, 3))
        got = out.double().cpu().numpy()
        samp = np.array([got[i, j] for i, j in pairs])
        forms.append({
            "form": name, "ms": ms, "tflops_algorithmic": flops / (ms * 1e-3) / 1e12,
            "max_rel_err_sampled": float(np.max(np.abs(samp - exact) / np.abs(exact).max())),
            "rel_err_vs_closed_form": float(np.linalg.norm(got - closed) / np.linalg.norm(closed)),
            "kernels": [f"{st['kernel']} tile{st.get('tile', 0)} split{st.get('split', 1)}"
                        for st in p.describe()["steps"]],
        })
        del p, out, ws
        torch.cuda.empty_cache()
    by = {f["form"]: f for f in forms}
    chosen = by["bf16x3"]
    mfma_tflops = 3 * flops / (chosen["ms"] * 1e-3) / 1e12
    res = {
        "metric": METRIC, "value": flops / (chosen["ms"] * 1e-3) / 1e9, "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": chosen["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
        "data": "synthetic (seeded)",
        "config": {"workload": f"trans(X)*X, X {rows}x{cols} FP32 from an SVD, cond {cond:g}",
                   "form": "split-BF16 x3 SYRK (FP32 accumulation)"},
        "roofline": {"bound": "mfma", "achieved": mfma_tflops, "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": mfma_tflops / BF16_PEAK_TFLOPS, "traffic": None,
                     "note": "achieved counts the 3 BF16 products executed per FP32 product"},
        "speedup_vs_plain_fp64": by["fp64"]["ms"] / chosen["ms"],
        "fp64_frac_of_peak": by["fp64"]["tflops_algorithmic"] / FP64_PEAK_TFLOPS,
        "forms": forms,
    }
    return res


def bench_solve(args, ctx, hx, torch, inputs):
    """solve(S, B), S 8192^2 FP64 = U diag(s) V^T with cond 1e3, B 8192x64:
    plain FP64 LU vs the mixed-precision forms, error against the closed form
    X = V diag(1/s) U^T B."""
    n, nrhs, cond = 8192, 64, 1e3
    s_dev, sv, v, u = inputs.svd_matrix_device(1004, n, n, cond, dtype=torch.float64, return_u=True)
    bh = inputs.normal(inputs.rng(1005), n, nrhs)
    b_dev = torch.from_numpy(np.ascontiguousarray(bh.T)).cuda().t()
    closed = (v / sv[None, :]) @ (u.T @ bh)
    flops = 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nrhs
    es, eb = ctx.leaf(s_dev), ctx.leaf(b_dev)
    forms = []
    wanted = [f for f in args.forms.split(",") if f] or ["plain", "ir_fp32", "ir_bf16x3", "ir_bf16x6", "ir_fp16"]
    for form in wanted:
        p = ctx.plan(hx.solve(es, eb), solve_precision=form)
        out, ws = p.output(), p.workspace()
        p.execute(out, ws)           # warm-up (also compiles nothing: no element-wise pass)
        ctx.sync()
        reps = max(1, min(args.steps, 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            p.execute(out, ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        rep = ctx.sync()
        got = out.cpu().numpy()
        forms.append({"form": form, "ms": ms, "gflops_algorithmic": flops / (ms * 1e-3) / 1e9,
                      "status": int(rep.status), "ir_iterations": int(rep.ir_iterations),
                      "rel_err_vs_closed_form": float(np.linalg.norm(got - closed) / np.linalg.norm(closed)),
                      "backward_err": float(np.linalg.norm(bh - s_dev.cpu().numpy() @ got) /
                                            (np.linalg.norm(s_dev.cpu().numpy()) * np.linalg.norm(got)))})
        del p, out, ws
    by = {f["form"]: f for f in forms}
    if "plain" not in by:
        return {"forms": forms}
    best = min((f for f in forms if f["form"] != "plain" and f["rel_err_vs_closed_form"] <= 1e-12),
               key=lambda f: f["ms"], default=by["plain"])
    res = {
        "metric": METRIC, "value": flops / (best["ms"] * 1e-3) / 1e9, "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": best["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": f"solve(S,B), S {n}x{n} FP64 from an SVD (cond {cond:g}), B {n}x{nrhs}",
                   "form": best["form"]},
        "roofline": {"bound": "mfma", "achieved": flops / (by["plain"]["ms"] * 1e-3) / 1e12,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / (by["plain"]["ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "traffic": None, "note": "plain FP64 LU + solve, whole-solve rate"},
        "speedup_vs_plain_fp64": by["plain"]["ms"] / best["ms"],
        "forms": forms,
    }
    return res


def bench_learned(args, ctx, hx, torch, inputs):
    """The learned planner: timings from the evaluator's own autotuner (the
    products of the FP32 chain, trans(X)*X at 65536 x 2048 in FP32 and FP64,
    and a log-uniform shape sweep whose seed is disjoint from the evaluation
    chains), a model trained on the GPU, then `chains` random FP32 chains
    (length 3-8, dims log-uniform in [16, 8192], N(0,1)) planned by the DP
    (default tiles) and by the learned planner, each timed by graph replay."""
    import tempfile
    import oracle
    from paper_2502_03000_amd import learn
    log = os.path.join(tempfile.mkdtemp(), "timings.jsonl")
    t0 = time.perf_counter()
    # autotune records of the FP32 chain and the symmetric products
    ctx.timing_log(log)
    chain_np = inputs.fp32_chain(seed=1001)
    chain_t = [torch.from_numpy(np.ascontiguousarray(m.T)).cuda().t() for m in chain_np]
    e = None
    for t in chain_t:
        e = ctx.leaf(t) if e is None else e @ ctx.leaf(t)
    p = ctx.plan(e)
    p.autotune(p.output(), p.workspace(), reps=2)
    x = torch.randn(2048, 65536, device="cuda").t()  # 65536 x 2048, column-major
    for dt in (torch.float32, torch.float64):
        xe = ctx.leaf(x.to(dt))
        p = ctx.plan(hx.trans(xe) @ xe)
        p.autotune(p.output(), p.workspace(), reps=1)
    ctx.timing_log(None)
    ctx.clear()
    del p, x, chain_t
    torch.cuda.empty_cache()
    learn.timing_sweep(ctx, learn.log_uniform_shapes(2005, args.sweep, 16, 8192), log, reps=2)
    sweep_s = time.perf_counter() - t0
    recs = learn.read_log(log)
    xs, ys = learn.dataset(recs)
    t1 = time.perf_counter()
    model, loss = learn.train(ctx, xs, ys, epochs=200)
    train_s = time.perf_counter() - t1
    ctx.set_model(model)

    chains = inputs.random_chain_dims(seed=1005, count=args.chains)
    need = max(sum(a * b for a, b in zip(d[:-1], d[1:])) for d in chains)
    g = torch.Generator(device="cuda")
    g.manual_seed(1005)
    pool = torch.randn(need, generator=g, device="cuda")

    def build(dims, planner):
        off, ls = 0, []
        for a, b in zip(dims[:-1], dims[1:]):
            ls.append(ctx.leaf(pool[off:off + a * b].view(b, a).t()))
            off += a * b
        ex = ls[0]
        for q in ls[1:]:
            ex = ex @ q
        return ctx.plan(ex, planner=planner)

    def timed(pl, reps=3):
        out, ws = pl.output(), pl.workspace()
        pl.capture(out, ws)
        pl.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pl.replay()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps, out

    rows = []
    fl = {"dp": 0.0, "learned": 0.0, "roofline": 0.0}
    n_learned = 0
    sample = set(inputs.rng(12).choice(len(chains), 8, replace=False).tolist())
    err = 0.0
    t1 = time.perf_counter()
    for i, dims in enumerate(chains):
        row = {}
        for planner in ("dp", "learned", "roofline"):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            pl = build(dims, planner)
            plan_ms = (time.perf_counter() - tp) * 1e3
            ex_ms, out = timed(pl)
            row[planner] = (plan_ms, ex_ms)
            fl[planner] += pl.info.flops
            if planner == "learned":
                n_learned += pl.describe()["learned"][0]["chosen"] == "learned"
                if i in sample:  # rows of the product against FP64 row-vector products
                    got = out.cpu().numpy().astype(np.float64)
                    mats, off = [], 0
                    for r, c in zip(dims[:-1], dims[1:]):
                        mats.append(pool[off:off + r * c].view(c, r).t().cpu().numpy().astype(np.float64))
                        off += r * c
                    for rr in inputs.rng(i).integers(0, dims[0], 2):
                        v = mats[0][rr:rr + 1]
                        for m in mats[1:]:
                            v = v @ m
                        err = max(err, float(np.linalg.norm(got[rr] - v[0]) / np.linalg.norm(v[0])))
            del pl, out
        rows.append(row)
        ctx.clear()
    eval_s = time.perf_counter() - t1

    def stats(name):
        plan = np.array([r[name][0] for r in rows])
        ex = np.array([r[name][1] for r in rows])
        return plan, ex

    pd_, ed = stats("dp")
    summary = {}
    for name in ("dp", "learned", "roofline"):
        pp, ee = stats(name)
        summary[name] = {"plan_ms_total": float(pp.sum()), "exec_ms_total": float(ee.sum()),
                         "end_to_end_ms_total": float((pp + ee).sum()), "gflop": fl[name] / 1e9}
        if name != "dp":
            summary[name].update({
                "exec_geomean_speedup_vs_dp": float(np.exp(np.mean(np.log(ed / ee)))),
                "exec_win_rate_vs_dp": float(np.mean(ee < ed)),
                "exec_speedup_total_vs_dp": float(ed.sum() / ee.sum()),
                "end_to_end_geomean_speedup_vs_dp": float(np.exp(np.mean(np.log((pd_ + ed) / (pp + ee))))),
                "end_to_end_win_rate_vs_dp": float(np.mean(pp + ee < pd_ + ed)),
                "end_to_end_speedup_total_vs_dp": float((pd_ + ed).sum() / (pp + ee).sum())})
            # executions of each plan after which the extra planning time is
            # repaid by the faster executions (None: never, or no extra cost)
            extra, gain = float((pp - pd_).sum()), float((ed - ee).sum())
            summary[name]["break_even_executions_per_plan"] = (
                extra / gain if gain > 0 and extra > 0 else None)
    summary["learned"]["chains_learned_order"] = n_learned
    t_ln = summary["learned"]["exec_ms_total"]
    t_dp = summary["dp"]["exec_ms_total"]
    fl_ln = fl["learned"]
    tflops = fl_ln / (t_ln * 1e-3) / 1e12
    res = {
        "metric": METRIC, "value": fl_ln / (t_ln * 1e-3) / 1e9, "unit": "GFLOP/s",
        "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": t_ln,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": f"{len(chains)} random FP32 chains, length 3-8, dims log-uniform "
                               "in [16, 8192], N(0,1); learned planner vs FLOP DP vs roofline DP",
                   "training_records": len(recs), "training_loss_std_mse": loss,
                   "sweep_s": sweep_s, "train_s": train_s, "eval_s": eval_s,
                   "timing": "execution: graph replay, mean of 3; planning: host wall time of "
                             "hexla_plan_create (the learned planner's inference launch and its "
                             "wait included); end to end: planning + one execution"},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP32_MFMA_PEAK_TFLOPS, "traffic": None,
                     "note": "all products of all chains, learned plans"},
        "speedup_vs_dp": t_dp / t_ln,
        "dp": summary["dp"], "learned": summary["learned"], "roofline_planner": summary["roofline"],
        "max_rel_err_sampled_rows": err,
    }
    if not args.no_cpu_baseline:  # the oracle on whole chains, in order, for about 10 s
        t1 = time.perf_counter()
        done, fl = 0, 0.0
        from oracle import chain as ch
        for dims in chains:
            env, off = {}, 0
            for j, (r, c) in enumerate(zip(dims[:-1], dims[1:])):
                env[f"M{j}"] = pool[off:off + r * c].view(c, r).t().cpu().numpy()
                off += r * c
            oracle.evaluate("*".join(env), env)
            fl += 2.0 * ch.brute_force_min(list(dims))[0]
            done += 1
            if time.perf_counter() - t1 >= 10.0:
                break
        el = time.perf_counter() - t1
        res["cpu_baseline"] = {"value": fl / el / 1e9, "unit": "GFLOP/s", "cores": _threads(),
                               "kind": "oracle",
                               "sample": f"the first {done} of the {len(chains)} chains, in the "
                                         f"oracle's cheapest order ({el:.1f} s, float64 numpy)"}
    return res


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([x.get("num_threads", 1) for x in threadpool_info()] or [1]))
    except Exception:  # noqa: BLE001
        return os.cpu_count() or 1


BATCH_NAMES = ["A", "B", "v", "S", "b", "p", "q"]


def bench_batched(args, ctx, hx, torch, inputs):
    """count instances of trans(A)*B*v + solve(S,b) + 2*(p%q), n log-uniform
    in [8, 512], S diagonally dominant: one persistent launch (autotuned,
    graph-replayed) in FP32 and FP64, against the plain FP64 path (one plan per
    instance, launched eagerly one after another). Errors against the FP64
    oracle on a sample of instances."""
    import oracle
    t0 = time.perf_counter()
    insts = inputs.batched_instances(seed=1003, count=args.count, dtype=np.float32)
    sizes = np.array([d["A"].shape[0] for d in insts], dtype=np.int64)
    arena32, ptrs32 = hx.pack_batch(insts, BATCH_NAMES, torch.float32)
    arena64 = arena32.double()
    ptrs64 = arena64.data_ptr() + (ptrs32 - arena32.data_ptr()) // 4 * 8
    gen_s = time.perf_counter() - t0
    g = inputs.rng(11)
    order = np.argsort(sizes)
    sample = sorted(set(order[:4].tolist() + order[-4:].tolist() +
                        g.choice(len(insts), 16, replace=False).tolist()))
    refs = {i: oracle.evaluate(inputs.BATCHED_EXPR, insts[i])[:, 0] for i in sample}

    def err_of(host_out, offs):
        e = 0.0
        for i in sample:
            got = host_out[offs[i]:offs[i] + sizes[i]].astype(np.float64)
            e = max(e, float(np.linalg.norm(got - refs[i]) / np.linalg.norm(refs[i])))
        return e

    def template(dt):
        L = {n: ctx.template_leaf(4, "matrix" if n in "ABS" else "vector", dt) for n in BATCH_NAMES}
        root = hx.trans(L["A"]) * L["B"] * L["v"] + hx.solve(L["S"], L["b"]) + 2 * (L["p"] % L["q"])
        return root, [L[n] for n in BATCH_NAMES]

    def time_replay(bt, reps):
        st = torch.cuda.current_stream()
        for _ in range(max(args.warmup, 1)):
            bt.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            bt.replay()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    forms = []
    batches = {}
    wanted = [f for f in args.forms.split(",") if f] or ["batched_fp64", "plain_fp64_per_instance"]
    for name, tdt, hdt, ptrs in [("batched_fp32", torch.float32, hx.F32, ptrs32),
                                 ("batched_fp64", torch.float64, hx.F64, ptrs64)]:
        if name != "batched_fp32" and name not in wanted:
            continue
        root, leaves = template(hdt)
        out, optrs, offs = hx.output_arena(sizes, tdt)
        bt = ctx.batch(root, leaves, sizes, ptrs, optrs)
        ws = bt.workspace()
        t1 = time.perf_counter()
        if not args.no_tune:
            bt.autotune(ws, reps=2)
        tune_s = time.perf_counter() - t1
        bt.capture(ws)
        ms = time_replay(bt, max(args.steps, 3))
        rep = ctx.sync()
        info = bt.describe()
        forms.append({"form": name, "ms": ms, "status": int(rep.status),
                      "gflops": info["flops"] / (ms * 1e-3) / 1e9,
                      "gbs": info["bytes"] / (ms * 1e-3) / 1e9,
                      "max_rel_err_sampled": err_of(out.cpu().numpy(), offs),
                      "config": {"panel": info["panel"], "threads": info["threads"],
                                 "grid": info["grid"]}, "autotune_s": tune_s})
        batches[name] = (bt, ws, out, info)

    # plain FP64 path: one ordinary plan per instance over views of the FP64 arena
    if "plain_fp64_per_instance" in wanted:
        base = arena64.data_ptr()
        out64, optrs64, offs64 = hx.output_arena(sizes, torch.float64)
        plans, max_ws = [], 1
        t1 = time.perf_counter()
        for i, n in enumerate(sizes):
            n = int(n)
            off = [(int(ptrs64[i, j]) - base) // 8 for j in range(7)]
            mat = lambda j: arena64[off[j]:off[j] + n * n].view(n, n).t()
            vec = lambda j: arena64[off[j]:off[j] + n]
            A, B, v, S, b, p, q = (ctx.leaf(mat(j) if j in (0, 1, 3) else vec(j)) for j in range(7))
            pl = ctx.plan(hx.trans(A) * B * v + hx.solve(S, b) + 2 * (p % q))
            plans.append((pl, out64[offs64[i]:offs64[i] + n]))
            max_ws = max(max_ws, pl.workspace_bytes)
            ctx.clear()
        plan_s = time.perf_counter() - t1
        ws64 = torch.empty(max_ws, dtype=torch.uint8, device="cuda")

        def plain_all():
            for pl, o in plans:
                pl.execute(o, ws64)

        plain_all()  # warm-up
        ctx.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain_all()
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t1) * 1e3
        rep = ctx.sync()
        flops = batches["batched_fp32"][3]["flops"]
        forms.append({"form": "plain_fp64_per_instance", "ms": ms_plain, "status": int(rep.status),
                      "gflops": flops / (ms_plain * 1e-3) / 1e9,
                      "max_rel_err_sampled": err_of(out64.cpu().numpy(), offs64),
                      "plan_s": plan_s, "launch": "eager, one plan per instance"})
    by = {f["form"]: f for f in forms}
    chosen = by["batched_fp32"]
    info = batches["batched_fp32"][3]
    t_hbm = info["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_alu = info["flops"] / (FP32_MFMA_PEAK_TFLOPS * 1e12)
    ms = chosen["ms"]
    if t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": info["bytes"] / (ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": info["flops"] / (ms * 1e-3) / 1e12,
                "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["ideal_ms"] = {"hbm": t_hbm * 1e3, "fp32_alu": t_alu * 1e3}
    res = {
        "metric": METRIC, "value": info["flops"] / (ms * 1e-3) / 1e9, "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": f"batched: {args.count} x (trans(A)*B*v + solve(S,b) + 2*(p%q)), "
                               "FP32, n log-uniform in [8,512], S diagonally dominant",
                   "form": "one persistent launch, autotuned, hip graph replay",
                   "total_gflop": info["flops"] / 1e9, "total_gbytes": info["bytes"] / 1e9},
        "roofline": roof,
        "speedup_vs_plain_fp64": (by["plain_fp64_per_instance"]["ms"] / ms
                                  if "plain_fp64_per_instance" in by else None),
        "forms": forms, "generate_s": gen_s,
    }
    if not args.no_cpu_baseline:
        t1 = time.perf_counter()
        done, fl = 0, 0.0
        for i in g.permutation(len(insts)):
            oracle.evaluate(inputs.BATCHED_EXPR, insts[i])
            n = float(sizes[i])
            fl += 2 * n ** 3 / 3 + 6 * n * n + 4 * n
            done += 1
            if time.perf_counter() - t1 >= 10.0:
                break
        el = time.perf_counter() - t1
        try:
            from threadpoolctl import threadpool_info
            threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
        except Exception:  # noqa: BLE001
            threads = os.cpu_count() or 1
        res["cpu_baseline"] = {"value": fl / el / 1e9, "unit": "GFLOP/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"{done} random instances of the {args.count} "
                                         f"({el:.1f} s, float64 numpy)"}
    return res


def bench_diag(args, ctx, hx, torch, inputs):
    """The diagonal rewrites of expressions (3)-(5), (7) and the view of
    expression (2) at sizes where HBM decides, each against the naive
    evaluation (full product / dense diagonal matrix / temporaries): FP64,
    n = 8192 (A, B 8192^2 N(0,1); vectors of 2^25 for expression (7))."""
    import oracle
    n = 8192
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1006)
    a = torch.randn((n, n), generator=gen, device="cuda", dtype=torch.float64).t()
    b = torch.randn((n, n), generator=gen, device="cuda", dtype=torch.float64).t()
    nv = 1 << 25
    x, w, y = (torch.randn(nv, generator=gen, device="cuda", dtype=torch.float64) for _ in range(3))
    ea, eb = ctx.leaf(a), ctx.leaf(b)
    ex, ew_, ey = ctx.leaf(x), ctx.leaf(w), ctx.leaf(y)
    cases = [
        ("diag(A*B)", hx.diag(ea @ eb), 2.0 * n * n * 8),
        ("trace(A*B)", hx.trace(ea @ eb), 2.0 * n * n * 8),
        ("diagmat(A*B)", hx.diagmat(ea @ eb), (2.0 * n * n + n * n) * 8),
        ("diagmat(A)*B", hx.diagmat(ea) @ eb, (n + 2.0 * n * n) * 8),
        ("trans(x)*diagmat(w)*y", hx.trans(ex) @ hx.diagmat(ew_) @ ey, 3.0 * nv * 8),
        ("A(:,1) + B(2,:)^T", ea.col(0) + hx.trans(eb.row(1)), 3.0 * n * 8),
    ]
    ah = b_h = None
    forms = []
    reps = max(args.reps // 4, 10)
    for text, e, nbytes in cases:
        row = {"expression": text, "algorithmic_bytes": nbytes}
        for planner in ("dp", "naive"):
            if planner == "naive" and text.startswith("trans(x)"):
                continue  # the naive form builds a 2^25 x 2^25 diagonal matrix
            p = ctx.plan(e, planner=planner)
            o, ws = p.output(), p.workspace()
            run = lambda: p.execute(o, ws)  # noqa: E731
            run()
            ctx.sync()
            ms = median_ms(torch, run, reps)
            row[planner] = {"ms": ms, "kernels": [st["kernel"] for st in p.describe()["steps"]]}
            if planner == "dp":
                row["gbs"] = nbytes / (ms * 1e-3) / 1e9
                row["frac_hbm"] = row["gbs"] / HBM_PEAK_GBS
                out_dp = o
            del p, ws
        if "naive" in row:
            row["speedup_vs_naive"] = row["naive"]["ms"] / row["dp"]["ms"]
        # error against the FP64 oracle on a slice the oracle computes exactly
        g = inputs.rng(7)
        if text in ("diag(A*B)", "trace(A*B)", "diagmat(A*B)"):
            if ah is None:
                ah, b_h = a.cpu().numpy(), b.cpu().numpy()
            idx = np.sort(g.choice(n, 16, replace=False))
            ref = np.array([ah[i, :] @ b_h[:, i] for i in idx])
            if text == "trace(A*B)":
                ref_t = oracle.evaluate("trace(A*B)", {"A": ah, "B": b_h})[0, 0]
                got = out_dp.cpu().numpy()[0, 0]
                row["rel_err_vs_fp64"] = abs(got - ref_t) / abs(ref_t)
            else:
                d = out_dp.cpu().numpy()
                got = d[idx, 0] if text == "diag(A*B)" else d[idx, idx]
                row["rel_err_vs_fp64"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        forms.append(row)
        del out_dp
    best = forms[0]
    return {"metric": METRIC, "value": best["gbs"], "unit": "GB/s", "ms_per_step": best["dp"]["ms"],
            "dtype": "f64",
            "config": {"workload": f"diagonal rewrites and views, FP64, n = {n}"},
            "roofline": {"bound": "hbm", "achieved": best["gbs"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": best["gbs"] / HBM_PEAK_GBS,
                         "kernel": "diag_product of diag(A*B)"},
            "forms": forms}


def bench_struct(args, ctx, hx, torch, inputs):
    """Structure-aware solves at n = 8192, B 8192 x 64, FP64: each matrix
    solved with the structure analysis (auto) and with the general LU
    (general); backward error ||B - S X|| / (||S|| ||X||) of each."""
    n, r = 8192, 64
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1007)
    g = torch.randn((n, n), generator=gen, device="cuda", dtype=torch.float64)
    mats = {
        "spd": (g @ g.t() / n + torch.eye(n, device="cuda", dtype=torch.float64)),
        "lower": torch.tril(g / n ** 0.5) + 2.0 * torch.eye(n, device="cuda", dtype=torch.float64),
        "tridiagonal": (torch.diag(torch.rand(n, generator=gen, device="cuda", dtype=torch.float64) * 0.6 - 0.3)
                        + torch.diag(1.0 + 0.2 * torch.randn(n - 1, generator=gen, device="cuda",
                                                              dtype=torch.float64), -1)
                        + torch.diag(-1.0 + 0.2 * torch.randn(n - 1, generator=gen, device="cuda",
                                                               dtype=torch.float64), 1)),
    }
    del g
    bmat = torch.randn((r, n), generator=gen, device="cuda", dtype=torch.float64).t()
    forms = []
    for kind, m in mats.items():
        s_dev = m.t().contiguous().t()  # column-major
        es, eb = ctx.leaf(s_dev), ctx.leaf(bmat)
        row = {"matrix": kind}
        for opt in ("auto", "general"):
            p = ctx.plan(hx.solve(es, eb), solve_structure=opt)
            o, ws = p.output(), p.workspace()
            p.execute(o, ws)
            rep = ctx.sync()
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                p.execute(o, ws)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            rep = ctx.sync()
            res_ = bmat - s_dev @ o
            berr = float(torch.linalg.norm(res_) / (torch.linalg.norm(s_dev) * torch.linalg.norm(o)))
            row[opt] = {"ms": float(np.median(ts)), "status": int(rep.status),
                        "solver": hx.SOLVERS.get(int(rep.solver), "lu"), "backward_error": berr}
            del p, o, ws
        row["speedup_vs_lu"] = row["general"]["ms"] / row["auto"]["ms"]
        forms.append(row)
        ctx.clear()
    spd = forms[0]
    flops = n ** 3 / 3.0 + 2.0 * n * n * r
    return {"metric": METRIC, "value": flops / (spd["auto"]["ms"] * 1e-3) / 1e9, "unit": "GFLOP/s",
            "ms_per_step": spd["auto"]["ms"], "dtype": "f64",
            "config": {"workload": f"structure-aware solve(S,B), S {n}x{n} (spd, lower, "
                                   f"tridiagonal), B {n}x{r}, FP64"},
            "roofline": {"bound": "mfma", "achieved": flops / (spd["auto"]["ms"] * 1e-3) / 1e12,
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / (spd["auto"]["ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                         "kernel": "whole Cholesky solve, n^3/3 + 2 n^2 nrhs flops"},
            "forms": forms}


def median_ms(torch, fn, reps, stream=None):
    """Median over reps of one call of fn, each bracketed by HIP events on
    the launch stream (a GPU-side spin first, so that the events see kernel
    time, not the host's launch rate)."""
    st = stream or torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(200_000)
        ev0.record(st)
        fn()
        ev1.record(st)
        ev1.synchronize()
        ts.append(ev0.elapsed_time(ev1))
    return float(np.median(ts))


def cold_ms(torch, fn, flush):
    """One call of fn right after 512 MB of unrelated writes (the caches hold
    none of its operands)."""
    flush.add_(1.0)
    return median_ms(torch, fn, 1)


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def expr_jobs(args, ctx, hx, torch, inputs, dt, tune=True):
    """The two jobs of the FP32-at-scale workload in storage type dt (FP32,
    or FP64 for the plain-FP64 leg): plans, per-job median and cold times,
    sampled errors against the FP64 oracle."""
    import oracle
    dev = "cuda:0"
    chain_np = inputs.fp32_chain(seed=1001)
    chain_t = [torch.from_numpy(np.ascontiguousarray(m.T)).to(dev).to(dt).t() for m in chain_np]
    ew = inputs.fp32_elementwise_device(seed=1001, n=args.n, device=dev)
    if dt != torch.float32:
        ew = {k: v.t().contiguous().to(dt).t() for k, v in ew.items()}
    torch.cuda.synchronize()
    e1 = None
    for t in chain_t:
        x = ctx.leaf(t)
        e1 = x if e1 is None else e1 @ x
    t0 = time.perf_counter()
    p1 = ctx.plan(e1)
    A, B, Cm = (ctx.leaf(ew[k]) for k in ("A", "B", "C"))
    p2 = ctx.plan(0.5 * hx.exp(-(A % A)) + B / Cm)
    plan_ms = (time.perf_counter() - t0) * 1e3
    out1, out2 = p1.output(dev), p2.output(dev)
    ws1, ws2 = p1.workspace(dev), p2.workspace(dev)
    if tune and not args.no_tune:
        p1.autotune(out1, ws1)
    run1 = lambda: p1.execute(out1, ws1)  # noqa: E731
    run2 = lambda: p2.execute(out2, ws2)  # noqa: E731
    for _ in range(3):
        run1()
        run2()
    if ctx.sync().status != hx.OK:
        raise SystemExit("deferred error in the expression jobs")
    reps = max(args.reps, 1)
    flush = torch.empty(1 << 27, dtype=torch.float32, device=dev)
    ms_chain, ms_ew = median_ms(torch, run1, reps), median_ms(torch, run2, reps)
    cold_chain, cold_ew = cold_ms(torch, run1, flush), cold_ms(torch, run2, flush)
    del flush
    # sampled parity against the FP64 oracle: rows of the chain, columns of job 2
    g = inputs.rng(99)
    rows = sorted(set([0, chain_np[0].shape[0] - 1] + g.integers(0, chain_np[0].shape[0], 6).tolist()))
    names = [f"M{i}" for i in range(len(chain_np))]
    env = dict(zip(names, chain_np), M0=np.asfortranarray(chain_np[0][rows, :]))
    ref = oracle.evaluate("*".join(names), env)
    got = out1.cpu().numpy().astype(np.float64)[rows]
    err_chain = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    cols = sorted(set([0, args.n - 1] + g.integers(0, args.n, 6).tolist()))
    idx = torch.tensor(cols, device=dev)
    sub = {k: v.index_select(1, idx).cpu().numpy().astype(np.float64) for k, v in ew.items()}
    ref = oracle.evaluate("0.5*exp(-(A%A)) + B/C", sub)
    got = out2.index_select(1, idx).cpu().numpy().astype(np.float64)
    err_ew = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    d1, d2 = p1.describe(), p2.describe()
    res = {"p1": p1, "p2": p2, "run1": run1, "run2": run2, "d1": d1, "d2": d2,
           "chain_np": chain_np, "ew": ew, "plan_ms": plan_ms,
           "chain": {"ms_median": ms_chain, "ms_cold": cold_chain, "gflop": p1.info.flops / 1e9,
                     "tflops": p1.info.flops / (ms_chain * 1e-3) / 1e12,
                     "kernels": [f"{s['kernel']} {s['m']}x{s['n']}x{s['k']} tile{s.get('tile')} "
                                 f"split{s.get('split', 1)}" for s in d1["steps"]],
                     "rel_err_vs_fp64_sampled_rows": err_chain},
           "elementwise": {"ms_median": ms_ew, "ms_cold": cold_ew, "gbytes": d2["bytes"] / 1e9,
                           "gbs": d2["bytes"] / (ms_ew * 1e-3) / 1e9,
                           "rel_err_vs_fp64_sampled_cols": err_ew}}
    # the same three reads and one write with no arithmetic to speak of: the
    # HBM rate a generated element-wise kernel of this shape reaches
    p3 = ctx.plan(A + B + Cm)
    out3 = p3.output(dev)
    ws3 = p3.workspace(dev)
    run3 = lambda: p3.execute(out3, ws3)  # noqa: E731
    run3()
    ms_stream = median_ms(torch, run3, reps)
    d3 = p3.describe()
    res["stream_probe"] = {"expression": "A + B + C", "ms_median": ms_stream,
                           "gbs": d3["bytes"] / (ms_stream * 1e-3) / 1e9,
                           "elementwise_rate_over_probe": (d2["bytes"] / ms_ew) / (d3["bytes"] / ms_stream)}
    del p3, out3, ws3
    return res


def summarize(job, key_ms="ms_per_step"):
    """The few figures of a workload's own line that its job entry keeps."""
    out = {k: job[k] for k in ("value", "unit", key_ms) if k in job}
    for k in ("speedup_vs_plain_fp64", "speedup_vs_dp", "dtype"):
        if k in job:
            out[k] = job[k]
    if "roofline" in job:
        out["roofline"] = {k: job["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    out["workload"] = job.get("config", {}).get("workload")
    for k in ("forms", "dp", "learned", "roofline_planner", "end_to_end"):
        if k in job:
            out[k] = job[k]
    return out


def bench_small(args, ctx, hx, torch, inputs):
    """The plain FP64 expression trans(A)*B*C*v + 0.5*(d % e) at its own size:
    planned into three matrix-vector products with the element-wise part as
    the last one's epilogue. Its work is 3.85 MB and 0.96 MFLOP, so launch
    latency decides its time: the median of eager executions (three queued
    launches), of graph replays, and of the left-to-right (naive) plan."""
    import oracle
    env = inputs.small_chain_expr(1000)
    t = {k: torch.from_numpy(np.ascontiguousarray(v.T)).cuda().t() for k, v in env.items()}
    L = {k: ctx.leaf(v) for k, v in t.items()}
    y = hx.trans(L["A"]) @ L["B"] @ L["C"] @ L["v"] + 0.5 * (L["d"] % L["e"])
    ref = oracle.evaluate(inputs.SMALL_CHAIN_EXPR, env)
    out = {}
    for planner in ("dp", "naive"):
        p = ctx.plan(y, planner=planner)
        o, ws = p.output(), p.workspace()
        run = lambda: p.execute(o, ws)  # noqa: E731
        run()
        ctx.sync()
        ms = median_ms(torch, run, max(args.reps, 100))
        p.capture(o, ws)
        ms_graph = median_ms(torch, p.replay, max(args.reps, 100))
        err = float(np.linalg.norm(o.cpu().numpy() - ref) / np.linalg.norm(ref))
        d = p.describe()
        out[planner] = {"ms_eager": ms, "ms_graph": ms_graph, "launches": len(d["steps"]),
                        "gflop": d["flops"] / 1e9, "mbytes": d["bytes"] / 1e6,
                        "gbs_eager": d["bytes"] / (ms * 1e-3) / 1e9,
                        "rel_err_vs_fp64": err, "kernels": [s["kernel"] for s in d["steps"]]}
        del p, o, ws
    dp = out["dp"]
    ideal_us = out["dp"]["mbytes"] * 1e6 / (HBM_PEAK_GBS * 1e9) * 1e6
    return {"metric": METRIC, "value": out["dp"]["gflop"] / (dp["ms_eager"] * 1e-3),
            "unit": "GFLOP/s", "ms_per_step": dp["ms_eager"], "dtype": "f64",
            "config": {"workload": "trans(A)*B*C*v + 0.5*(d%e), FP64, A 400x300, B 400x600, "
                                   "C 600x200, v 200x1, d,e 300x1"},
            "roofline": {"bound": "hbm", "achieved": dp["gbs_eager"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": dp["gbs_eager"] / HBM_PEAK_GBS},
            "ideal_us_at_hbm_peak": ideal_us,
            "launch_overhead_us": dp["ms_eager"] * 1e3 - ideal_us,
            "speedup_vs_naive_order": out["naive"]["ms_eager"] / dp["ms_eager"],
            "forms": [dict(planner=k, **v) for k, v in out.items()]}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import inputs
    from paper_2502_03000_amd import hexla as hx

    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = hx.Context(0)
    if args.tune_load:
        ctx.tune_load(args.tune_load)
        args.no_tune = True
    single = {"small": bench_small, "syrk": bench_syrk, "solve": bench_solve,
              "batched": bench_batched, "learned": bench_learned, "diag": bench_diag,
              "struct": bench_struct}
    if args.workload in single:
        line = single[args.workload](args, ctx, hx, torch, inputs)
        if args.tune_save:
            ctx.tune_save(args.tune_save)
        print(json.dumps(line), flush=True)
        return

    # ---- the headline step: the FP32 chain job, then the element-wise job
    j32 = expr_jobs(args, ctx, hx, torch, inputs, torch.float32)
    run1, run2 = j32["run1"], j32["run2"]
    main_stream = torch.cuda.current_stream()
    if args.overlap:
        # the two jobs are independent plans: the chain's launches on a second
        # stream (default priority) beside the element-wise pass
        side = torch.cuda.Stream()

        def step():
            ctx.set_stream(side.cuda_stream)
            run1()
            ctx.set_stream(main_stream.cuda_stream)
            run2()
    else:
        def step():
            run1()
            run2()

    if args.copy_probe:  # a plain copy of 1 GiB: reference for HBM byte counters
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    r = ctx.sync()
    if r.status != hx.OK:
        raise SystemExit(f"deferred error {r.status}")

    # ---- timed region: K whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    p1, p2, d2 = j32["p1"], j32["p2"], j32["d2"]
    flops_step = p1.info.flops + p2.info.flops
    chain_np, ew = j32["chain_np"], j32["ew"]

    ew_ms = j32["elementwise"]["ms_median"]
    ew_kernel = {"bound": "hbm", "achieved": d2["bytes"] / (ew_ms * 1e-3) / 1e9,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    ew_kernel["frac"] = ew_kernel["achieved"] / HBM_PEAK_GBS
    ew_kernel["traffic"] = profiled_traffic(d2["steps"][0].get("source_hash", "")) \
        if args.n == 16384 else None
    ew_kernel["kernel"] = "generated element-wise pass, median of per-launch HIP event times"
    chain32 = {k: v for k, v in j32["chain"].items()}
    chain32["frac_fp32_mfma_peak"] = chain32["tflops"] / FP32_MFMA_PEAK_TFLOPS
    jobs = {"chain_fp32": chain32, "elementwise_fp32": j32["elementwise"],
            "stream_probe_fp32": j32["stream_probe"]}
    cpu_inputs = None
    if not args.no_cpu_baseline:
        ncol = max(1, args.n // 2)
        cpu_inputs = (chain_np, {k: ew[k][:, :ncol].cpu().numpy() for k in ("A", "B", "C")},
                      d2["flops"] / float(args.n) ** 2)
    del j32, run1, run2, step
    p1 = p2 = None
    ctx.clear()
    torch.cuda.empty_cache()

    # ---- the same workload in plain FP64 (the metric's comparison)
    speedup = None
    if not args.quick:
        j64 = expr_jobs(args, ctx, hx, torch, inputs, torch.float64, tune=True)
        ms64 = j64["chain"]["ms_median"] + j64["elementwise"]["ms_median"]
        ms32 = jobs["chain_fp32"]["ms_median"] + jobs["elementwise_fp32"]["ms_median"]
        speedup = ms64 / ms32
        c64 = dict(j64["chain"])
        c64["frac_fp64_mfma_peak"] = c64["tflops"] / FP64_PEAK_TFLOPS
        jobs["chain_fp64"] = c64
        jobs["elementwise_fp64"] = j64["elementwise"]
        jobs["step_fp64_vs_fp32"] = {"ms_fp64": ms64, "ms_fp32": ms32, "speedup": speedup}
        del j64
        ctx.clear()
        torch.cuda.empty_cache()

    res = {
        "metric": METRIC,
        "value": flops_step / (ms_per_step * 1e-3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded)",
        "config": {"workload": "fp32 chain 8192x1024x8192x512x4096x64 (DP order) then fused "
                               f"0.5*exp(-(A%A))+B/C over {args.n}x{args.n}",
                   "chain_dims": list(inputs.FP32_CHAIN_DIMS), "elementwise_n": args.n,
                   "planner": "dp", "form": "plain fp32",
                   "launch": ("eager, the chain and the element-wise pass on two streams"
                              if args.overlap else "eager, one stream, one job after the other"),
                   "autotuned": not args.no_tune,
                   "timing": f"value: {args.steps} whole steps between two synchronisations; "
                             f"jobs: median of {args.reps} event-timed runs and one run after "
                             "a 512 MB flush (cold)"},
        "speedup_vs_plain_fp64": speedup,
        "roofline": ew_kernel,
        "jobs": jobs,
        "host": host_info(),
    }
    # ---- the other configurations, each in its own form, summarized
    if not args.quick:
        for name, fn in [("small_fp64_expression", bench_small), ("syrk_65536x2048", bench_syrk),
                         ("solve_8192", bench_solve), ("batched_10000", bench_batched),
                         ("learned_2000_chains", bench_learned), ("diagonal_rewrites", bench_diag),
                         ("structured_solves", bench_struct)]:
            t1 = time.perf_counter()
            jr = fn(args, ctx, hx, torch, inputs)
            jr_s = summarize(jr)
            jr_s["wall_s"] = time.perf_counter() - t1
            res["jobs"][name] = jr_s
            ctx.clear()
            torch.cuda.empty_cache()
    if cpu_inputs is not None:
        res["cpu_baseline"] = cpu_baseline(*cpu_inputs)
        res["cpu_baseline"].update(host_info())
    if args.tune_save:
        ctx.tune_save(args.tune_save)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
