"""Gaussian elimination with partial pivoting and the solves built on it
(test infrastructure).

The paper rewrites inv(A)*b into a call that solves the linear system without
forming the inverse (xGESV: LU with partial pivoting, then two triangular
solves; Sec. I and Sec. II, expression (9) of Sec. III). The naive mapping it
avoids forms the inverse explicitly (xGETRF + xGETRI, then a product; Sec. I).
Both are written out here in their textbook form, in float64.

Readings where the paper is silent:
* the pivot of column k is the first row (lowest index) holding the largest
  |a_ik|, i >= k, as IxAMAX returns it;
* an exactly zero pivot raises ``SingularMatrix``.
"""
from __future__ import annotations

import numpy as np


class SingularMatrix(ArithmeticError):
    def __init__(self, column):
        super().__init__(f"exact zero pivot in column {column}")
        self.column = column


def lu_partial_pivot(s, dtype=np.float64):
    """Row-by-row elimination on a copy of ``s``.

    Returns (perm, lu): rows of the permuted input are s[perm]; lu holds the
    unit lower factor L strictly below the diagonal and U on and above it, so
    that s[perm] == L @ U. ``dtype`` selects the storage (and arithmetic)
    precision of the elimination.
    """
    a = np.array(s, dtype=dtype, copy=True)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix required")
    perm = np.arange(n)
    for k in range(n):
        col = np.abs(a[k:, k])
        p = k + int(np.argmax(col))  # argmax returns the first maximum
        if a[p, k] == 0:
            raise SingularMatrix(k)
        if p != k:
            a[[k, p], :] = a[[p, k], :]
            perm[[k, p]] = perm[[p, k]]
        a[k + 1:, k] = a[k + 1:, k] / a[k, k]
        a[k + 1:, k + 1:] -= np.outer(a[k + 1:, k], a[k, k + 1:])
    return perm, a


def unpack_lu(lu):
    n = lu.shape[0]
    lower = np.tril(lu, -1) + np.eye(n, dtype=lu.dtype)
    upper = np.triu(lu)
    return lower, upper


def forward_unit(lu, b):
    """Solve L y = b with L unit lower triangular (strict lower part of lu)."""
    y = np.array(b, dtype=np.float64, copy=True)
    n = lu.shape[0]
    for i in range(n):
        if i:
            y[i] -= lu[i, :i].astype(np.float64) @ y[:i]
    return y


def backward(lu, y):
    """Solve U x = y with U upper triangular (upper part of lu)."""
    x = np.array(y, dtype=np.float64, copy=True)
    n = lu.shape[0]
    for i in range(n - 1, -1, -1):
        if i < n - 1:
            x[i] -= lu[i, i + 1:].astype(np.float64) @ x[i + 1:]
        x[i] /= np.float64(lu[i, i])
    return x


def lu_solve(perm, lu, b):
    b = np.asarray(b, dtype=np.float64)
    squeeze = b.ndim == 1
    if squeeze:
        b = b[:, None]
    x = backward(lu, forward_unit(lu, b[perm]))
    return x[:, 0] if squeeze else x


def solve(s, b):
    """x with s x = b, by partial-pivoting elimination and substitution."""
    perm, lu = lu_partial_pivot(s)
    return lu_solve(perm, lu, b)


def gauss_jordan_inverse(s):
    """Explicit inverse by Gauss-Jordan elimination on [s | I] with partial
    pivoting (the naive inverse that the solve rewrite avoids)."""
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[0]
    aug = np.hstack([s, np.eye(n)])
    for k in range(n):
        p = k + int(np.argmax(np.abs(aug[k:, k])))
        if aug[p, k] == 0:
            raise SingularMatrix(k)
        if p != k:
            aug[[k, p], :] = aug[[p, k], :]
        aug[k, :] = aug[k, :] / aug[k, k]
        for i in range(n):
            if i != k and aug[i, k] != 0:
                aug[i, :] -= aug[i, k] * aug[k, :]
    return aug[:, n:]
