"""Pins for the oracle's bfloat16 split, iterative refinement and MLP."""
import numpy as np
import pytest
import torch

import inputs
from oracle import bf16, mlp, refine


def test_rne_matches_torch_bfloat16_conversion():
    # torch's float32 -> bfloat16 cast rounds to nearest, ties to even
    g = inputs.rng(20)
    x = np.concatenate([
        g.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** g.integers(-20, 20, 20000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 3.4e38, -3.4e38, 1e-40, np.inf, -np.inf], np.float32),
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = bf16.rne(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_rne_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: the even neighbour is 1
    assert bf16.rne(np.float32(1 + 2 ** -8)) == np.float32(1.0)
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert bf16.rne(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)
    assert np.isnan(bf16.rne(np.float32(np.nan)))


def test_split_reconstruction_bounds():
    g = inputs.rng(21)
    x = (g.standard_normal(50000) * 3).astype(np.float32)
    hi, lo = bf16.split(x, 2)
    assert np.array_equal(hi, bf16.rne(x))
    assert np.all(np.abs(x.astype(np.float64) - hi - lo) <= 2.0 ** -16 * np.abs(x))
    assert np.all(np.abs(x.astype(np.float64) - hi) <= 2.0 ** -8 * np.abs(x))
    h3, m3, l3 = bf16.split(x, 3)
    assert np.all(np.abs(x.astype(np.float64) - h3 - m3 - l3) <= 2.0 ** -24 * np.abs(x))


def test_split_gram_error_bound():
    x, _, _, _ = inputs.svd_matrix(22, 512, 16, 1e2, dtype=np.float32)
    x = x.astype(np.float32)
    exact = x.astype(np.float64).T @ x.astype(np.float64)
    scale = np.abs(x.astype(np.float64)).T @ np.abs(x.astype(np.float64))
    g3 = bf16.split_gram(x, 2, 3)
    g6 = bf16.split_gram(x, 3, 6)
    # dropped products: lo*lo (2 terms) is below 2^-16 relative per product
    assert np.all(np.abs(g3 - exact) <= 2.0 ** -15 * scale)
    assert np.all(np.abs(g6 - exact) <= 2.0 ** -22 * scale)
    # and the split products are not trivially exact (the bound is not vacuous)
    assert np.max(np.abs(g3 - exact)) > 0


def test_refinement_converges_to_fp64_solution():
    x0, _, _, _ = inputs.svd_matrix(23, 96, 96, 1e3)
    g = inputs.rng(24)
    b = inputs.normal(g, 96, 3)
    out = refine.refine(x0, b)
    ref = np.linalg.solve(x0, b)
    assert out["status"] in ("converged", "stagnated") and out["accepted"]
    assert out["backward_errors"][-1] <= 96 * 2.0 ** -53
    assert np.linalg.norm(out["x"] - ref) / np.linalg.norm(ref) < 1e-12
    r = out["residuals"]
    assert all(r[i + 1] < r[i] for i in range(len(r) - 1))
    # the float32 starting point alone is far from float64 accuracy
    x_first = refine.low_precision_solver(x0)(b)
    assert np.linalg.norm(x_first - ref) / np.linalg.norm(ref) > 1e-10


def test_mlp_one_unit_by_hand():
    # y = w2 * relu(w1 x + b1) + b2 with w1 = 2, b1 = -1, w2 = 3, b2 = 0.5
    p = [(np.array([[2.0]]), np.array([-1.0])), (np.array([[3.0]]), np.array([0.5]))]
    y, cache = mlp.forward(p, np.array([[1.0], [0.25]]))
    assert np.array_equal(y, [3.5, 0.5])  # relu(1)=1 -> 3.5 ; relu(-0.5)=0 -> 0.5
    grads = mlp.backward(p, cache, y, np.array([3.0, 0.0]))
    # dL/dy = 2(y-t)/N = [0.5, 0.5]; only the first sample is active
    assert grads[1][0][0, 0] == 0.5 * 1.0 and grads[1][1][0] == 1.0
    assert grads[0][0][0, 0] == 0.5 * 3.0 * 1.0 and grads[0][1][0] == 0.5 * 3.0


def test_mlp_gradients_against_finite_differences():
    g = inputs.rng(25)
    p = mlp.init([5, 8, 8, 8, 1], g)
    p = [(w, b + 0.1 * g.standard_normal(b.shape)) for w, b in p]
    x = g.standard_normal((17, 5))
    t = g.standard_normal(17)
    y, cache = mlp.forward(p, x)
    grads = mlp.backward(p, cache, y, t)
    h = 1e-6
    for l in range(len(p)):
        for which in (0, 1):
            arr = p[l][which]
            for idx in list(np.ndindex(arr.shape))[:6]:
                plus = [(w.copy(), b.copy()) for w, b in p]
                minus = [(w.copy(), b.copy()) for w, b in p]
                plus[l][which][idx] += h
                minus[l][which][idx] -= h
                fd = (mlp.mse(mlp.forward(plus, x)[0], t) - mlp.mse(mlp.forward(minus, x)[0], t)) / (2 * h)
                assert grads[l][which][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_adam_first_step_moves_by_lr_times_sign():
    p = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[3.0, -0.25]]), np.array([1e-3]))]
    state = {}
    new = mlp.adam_step(p, grads, state, lr=1e-2)
    # bias-corrected m/sqrt(v) = g/|g| on the first step
    assert np.allclose(new[0][0], [[1.0 - 1e-2, -2.0 + 1e-2]], atol=1e-9)
    assert np.allclose(new[0][1], [0.5 - 1e-2], atol=1e-7)
    assert state["t"] == 1


def test_adam_second_step_by_hand():
    # one scalar parameter p0 = 1, gradients 3 then 1, lr 0.01, betas 0.9 / 0.999:
    #   step 1: m = 0.3, v = 0.009; bias-corrected 3 / sqrt(9) = 1 -> p1 = 0.99
    #   step 2: m = 0.9*0.3 + 0.1*1 = 0.37, v = 0.999*0.009 + 0.001*1 = 0.009991
    #           mhat = 0.37 / 0.19, vhat = 0.009991 / 0.001999
    #           p2 = 0.99 - 0.01 * 1.9473684210 / 2.2356652 = 0.9812893605
    p = [(np.array([[1.0]]), np.array([0.0]))]
    state = {}
    p = mlp.adam_step(p, [(np.array([[3.0]]), np.array([0.0]))], state, lr=1e-2)
    assert p[0][0][0, 0] == pytest.approx(0.99, abs=1e-9)
    p = mlp.adam_step(p, [(np.array([[1.0]]), np.array([0.0]))], state, lr=1e-2)
    assert p[0][0][0, 0] == pytest.approx(0.9812893605, abs=1e-9)
    assert state["t"] == 2
    # a zero gradient leaves the bias at zero through both steps
    assert p[0][1][0] == 0.0


def _scaled_exact_solver(s, factor):
    # a "low-precision" solve that returns factor times the exact correction:
    # the error of X is multiplied by (1 - factor) at every step
    return lambda r: factor * np.linalg.solve(s, r)


@pytest.mark.parametrize("factor,status,accepted", [
    (0.75, "converged", True),    # error x (-0.25) per step: corrections shrink 4x
    (1.6, "stagnated", False),    # error x (-0.6): the second correction is 0.6x the first
    (2.5, "diverging", False),    # error x (-1.5): the second correction grows
])
def test_refinement_outcomes_in_closed_form(factor, status, accepted):
    g = inputs.rng(26)
    s = inputs.diag_dominant(g, 40)
    b = inputs.normal(g, 40, 2)
    out = refine.refine(s, b, solve_low=_scaled_exact_solver(s, factor))
    assert out["status"] == status
    assert out["accepted"] is accepted
    assert len(out["backward_errors"]) == len(out["residuals"])
    if status == "diverging":
        # the growing correction was dropped: X is the first corrected iterate
        x = np.linalg.solve(s, b)
        x1 = factor * x + factor * (x - factor * x)
        assert np.allclose(out["x"], x1, rtol=1e-12, atol=1e-12)
        assert out["iterations"] == 1


def test_refinement_cap_is_not_accepted():
    g = inputs.rng(27)
    s = inputs.diag_dominant(g, 30)
    b = inputs.normal(g, 30, 1)
    out = refine.refine(s, b, solve_low=_scaled_exact_solver(s, 0.75), cap=1)
    assert out["status"] == "cap" and out["accepted"] is False and out["iterations"] == 1
