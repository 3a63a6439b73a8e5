"""Mixed-precision iterative refinement, step by step (test infrastructure).

Solves S X = B with a factorisation computed in a lower precision and a
residual computed in float64 (the classic refinement of Wilkinson/Moler; the
paper names reduced-precision types only as future work, Sec. IV, so every
choice here is a reading):

  X_0 = solve_low(B)
  repeat:
      R = B - S X                     (float64)
      stop if ||R||_inf <= 2^-53 * ||S||_inf * ||X||_inf
      D = solve_low(R)
      stop (diverging) if ||D||_inf > ||D_prev||_inf, keeping X
      X = X + D                       (float64)
      stop (stagnated) if ||D||_inf > 0.5 * ||D_prev||_inf
  until the iteration cap.

Each residual's backward error ||R||_inf / (||S||_inf ||X||_inf) is kept. The
result is accepted when the loop converged, or when it stagnated and the
backward error of the last residual formed is at most n * 2^-53 (the level of
a backward-stable FP64 solve); a diverging or capped loop is not accepted.

``solve_low`` solves with the low-precision factors; the oracle's default
factorises in float32 with partial pivoting (``gepp.lu_partial_pivot`` with
dtype float32) and substitutes in float64 on the float32 factors.
"""
from __future__ import annotations

import numpy as np

from . import gepp as _gepp


def norm_inf(a) -> float:
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.sum(np.abs(a), axis=1))) if a.size else 0.0


def low_precision_solver(s, dtype=np.float32):
    perm, lu = _gepp.lu_partial_pivot(s, dtype=dtype)

    def solve_low(r):
        return _gepp.lu_solve(perm, lu, r)

    return solve_low


def refine(s, b, solve_low=None, cap: int = 30) -> dict:
    s = np.asarray(s, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if solve_low is None:
        solve_low = low_precision_solver(s)
    n = s.shape[0]
    u = 2.0 ** -53
    s_norm = norm_inf(s)
    x = solve_low(b)
    history, berr = [], []
    d_prev = None
    status = "cap"
    for it in range(cap + 1):
        r = b - s @ x
        rn = norm_inf(r)
        history.append(rn)
        scale = s_norm * norm_inf(x)
        berr.append(rn / scale if scale > 0 else (np.inf if rn > 0 else 0.0))
        if rn <= u * scale:
            status = "converged"
            break
        if it == cap:
            break
        d = solve_low(r)
        dn = norm_inf(d)
        if d_prev is not None and dn > d_prev:
            status = "diverging"
            break
        x = x + d
        if d_prev is not None and dn > 0.5 * d_prev:
            status = "stagnated"
            break
        d_prev = dn
    accepted = status == "converged" or (status == "stagnated" and berr[-1] <= n * u)
    return {"x": x, "iterations": len(history) - 1, "residuals": history,
            "backward_errors": berr, "status": status, "accepted": accepted}
