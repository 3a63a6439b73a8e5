"""Plain FP64 evaluation of a parsed expression (test infrastructure).

Every operator is evaluated by its definition, with no rewrites and no fusion:
  * ``+ - % /`` and unary minus are element-wise; a scalar operand broadcasts
    (the element-wise loop of Sec. II, Z[i] = 0.4*X[i] + 0.6*Y[i]);
  * ``exp`` is element-wise;
  * ``*`` between a scalar and a matrix scales it; between two matrices it is
    the matrix product (AB)_ij = sum_k A_ik B_kj, sizes checked first (the
    conformance checks of Sec. II);
  * ``trans`` is the plain transpose (real data);
  * ``diag(X)``: d_i = X_ii, i < min(m, n), a column vector;
    ``diagmat(v)`` of a vector: the n x n matrix with D_ii = v_i, zeros
    elsewhere; ``diagmat(X)`` of a matrix: X_ij where i == j, else 0;
    ``trace(X)``: sum_i X_ii as a 1 x 1 matrix (expressions (3)-(5), (7) of
    Sec. III); on a number each is the number itself;
  * ``col(X, j)``, ``row(X, i)``, ``submat(X, r0, c0, rows, cols)``: the
    submatrix (0-based), expression (2);
  * ``inv(S) * Y`` is S^{-1} Y, computed by elimination (``gepp.solve``),
    ``solve(S, Y)`` likewise; a bare ``inv(S)`` (or ``X * inv(S)``) forms the
    inverse by Gauss-Jordan elimination, or every ``inv`` does when
    ``explicit_inverse=True`` (the naive mapping of Sec. I).

A chain of matrix products is multiplied in the bracketing with the fewest
multiply-adds, found by brute force over all bracketings (``chain``): in exact
arithmetic every bracketing gives the same matrix, and the cheap one keeps the
oracle fast. Inputs are widened to float64 first, so the result is the
float64 evaluation of the stored values.
"""
from __future__ import annotations

import numpy as np

from . import chain as _chain
from . import gepp as _gepp
from .parse import parse


class OracleDimError(ValueError):
    pass


def _is_scalar(v):
    return isinstance(v, float)


def _elementwise(op, a, b):
    if not _is_scalar(a) and not _is_scalar(b) and a.shape != b.shape:
        raise OracleDimError(f"element-wise {op}: {a.shape} vs {b.shape}")
    if op == "add":
        r = a + b
    elif op == "sub":
        r = a - b
    elif op == "schur":
        r = a * b
    elif op == "div":
        r = a / b
    else:
        raise ValueError(op)
    return float(r) if _is_scalar(a) and _is_scalar(b) else r


def _product(mats):
    """Product of a list of float64 matrices in the cheapest bracketing."""
    for x, y in zip(mats, mats[1:]):
        if x.shape[1] != y.shape[0]:
            raise OracleDimError(f"product: {x.shape} * {y.shape}")
    if len(mats) == 1:
        return mats[0]
    dims = [mats[0].shape[0]] + [m.shape[1] for m in mats]
    _, best = _chain.brute_force_min(dims) if len(mats) <= 9 else (None, [_chain.left_to_right(len(mats))])

    def run(t):
        if isinstance(t, int):
            return mats[t]
        return run(t[0]) @ run(t[1])

    return run(best[0])


def _diagonal_function(name, x):
    if _is_scalar(x):
        return x
    m, n = x.shape
    if name == "diag":
        return np.array([[x[i, i]] for i in range(min(m, n))], dtype=np.float64).reshape(-1, 1)
    if name == "trace":
        return np.array([[sum(x[i, i] for i in range(min(m, n)))]], dtype=np.float64)
    if m == 1 or n == 1:  # diagmat of a vector
        v = x.reshape(-1)
        d = np.zeros((v.size, v.size))
        for i in range(v.size):
            d[i, i] = v[i]
        return d
    d = np.zeros((m, n))
    for i in range(min(m, n)):
        d[i, i] = x[i, i]
    return d


def _submatrix(name, x, idx):
    if _is_scalar(x) or not all(_is_scalar(i) and float(i).is_integer() for i in idx):
        raise OracleDimError(f"{name}: a matrix and integer indices are required")
    idx = [int(i) for i in idx]
    m, n = x.shape
    if name == "col":
        r0, c0, rows, cols = 0, idx[0], m, 1
    elif name == "row":
        r0, c0, rows, cols = idx[0], 0, 1, n
    else:
        r0, c0, rows, cols = idx
    if min(r0, c0, rows, cols) < 0 or r0 + rows > m or c0 + cols > n:
        raise OracleDimError(f"{name}: indices out of range for {x.shape}")
    return np.ascontiguousarray(x[r0:r0 + rows, c0:c0 + cols])


class _Evaluator:
    def __init__(self, env, explicit_inverse):
        self.env = env
        self.explicit_inverse = explicit_inverse

    def factors(self, node):
        if node[0] == "mul":
            return self.factors(node[1]) + self.factors(node[2])
        if node[0] == "call" and node[1] == "inv":
            s = self.value(node[2][0])
            if _is_scalar(s):
                return [("val", 1.0 / s)]
            if s.shape[0] != s.shape[1]:
                raise OracleDimError(f"inv of non-square {s.shape}")
            return [("inv", s)]
        return [("val", self.value(node))]

    def chain(self, node):
        scale = 1.0
        items = []
        for kind, v in self.factors(node):
            if kind == "val" and _is_scalar(v):
                scale *= v
            else:
                items.append((kind, v))
        if not items:
            return scale
        result = self.reduce(items)
        return result * scale if scale != 1.0 else result

    def reduce(self, items):
        # an inverse applies to the product of everything on its right
        for idx, (kind, v) in enumerate(items):
            if kind == "inv":
                left = [m for _, m in items[:idx]]
                rest = items[idx + 1:]
                if rest and not self.explicit_inverse:
                    rhs = self.reduce(rest)
                    if rhs.shape[0] != v.shape[0]:
                        raise OracleDimError(f"inv(S)*Y: {v.shape} vs {rhs.shape}")
                    mid = _gepp.solve(v, rhs)
                    if mid.ndim == 1:
                        mid = mid[:, None]
                else:
                    mid = _gepp.gauss_jordan_inverse(v)
                    if rest:
                        mid = _product([mid, self.reduce(rest)])
                return _product(left + [mid]) if left else mid
        return _product([v for _, v in items])

    def value(self, node):
        kind = node[0]
        if kind == "num":
            return float(node[1])
        if kind == "var":
            v = self.env[node[1]]
            if np.isscalar(v):
                return float(v)
            a = np.asarray(v, dtype=np.float64)
            if a.ndim == 1:
                a = a[:, None]
            return a
        if kind == "neg":
            v = self.value(node[1])
            return -v
        if kind in ("add", "sub", "schur", "div"):
            return _elementwise(kind, self.value(node[1]), self.value(node[2]))
        if kind == "mul":
            return self.chain(node)
        if kind == "call":
            name, args = node[1], node[2]
            if name == "trans":
                v = self.value(args[0])
                return v if _is_scalar(v) else np.ascontiguousarray(v.T)
            if name == "exp":
                v = self.value(args[0])
                return float(np.exp(v)) if _is_scalar(v) else np.exp(v)
            if name == "inv":
                return self.chain(node)
            if name in ("diag", "diagmat", "trace"):
                return _diagonal_function(name, self.value(args[0]))
            if name in ("col", "row", "submat"):
                return _submatrix(name, self.value(args[0]), [self.value(a) for a in args[1:]])
            if name == "solve":
                s, b = self.value(args[0]), self.value(args[1])
                if s.shape[0] != s.shape[1]:
                    raise OracleDimError(f"solve with non-square {s.shape}")
                if s.shape[0] != b.shape[0]:
                    raise OracleDimError(f"solve: {s.shape} vs {b.shape}")
                if self.explicit_inverse:
                    return _product([_gepp.gauss_jordan_inverse(s), b])
                return _gepp.solve(s, b)
        raise ValueError(f"unknown node {node!r}")


def evaluate(expr, env: dict, explicit_inverse: bool = False):
    """Evaluate ``expr`` (text or AST) over ``env`` (name -> array or number).

    Returns a float64 2-D array (or a float for a scalar-valued expression).
    """
    node = parse(expr) if isinstance(expr, str) else expr
    return _Evaluator(env, explicit_inverse).value(node)


class _MagnitudeEvaluator(_Evaluator):
    """Pairs (value, magnitude) for the componentwise error scale.

    The magnitude M of a result bounds, to first order, how far a computation
    that rounds every operation can land from the exact value: an evaluation
    whose operations each carry a relative error of at most u (sums of length
    k count k times) stays within about K u M componentwise, K being the
    number of such roundings on the longest path. Rules:
      leaf or number x          |x|
      -a, trans(a)              M(a), transposed for trans
      a + b, a - b              M(a) + M(b)
      s * a (s a number)        |s| M(a)
      a % b                     M(a) M(b) (element-wise)
      a / b                     (M(a) + |a / b| M(b)) / |b|
      exp(a)                    exp(a) (1 + M(a))
      a * b (matrix product)    M(a) M(b) (matrix product of the magnitudes)
      diag, diagmat, trace,     the same function of M(a)
      submatrices
    so a product's magnitude is |op(A)| |op(B)|, the scale of the classical
    componentwise bound |fl(AB) - AB| <= k u |A| |B|. Solves and inverses have
    no such scale here (their error is measured normwise and by the backward
    error).
    """

    def vm(self, node):
        kind = node[0]
        if kind in ("num", "var"):
            v = self.value(node)
            return v, (abs(v) if _is_scalar(v) else np.abs(v))
        if kind == "neg":
            v, m = self.vm(node[1])
            return -v, m
        if kind in ("add", "sub"):
            (a, ma), (b, mb) = self.vm(node[1]), self.vm(node[2])
            return _elementwise(kind, a, b), ma + mb
        if kind == "schur":
            (a, ma), (b, mb) = self.vm(node[1]), self.vm(node[2])
            return _elementwise(kind, a, b), ma * mb
        if kind == "div":
            (a, ma), (b, mb) = self.vm(node[1]), self.vm(node[2])
            q = _elementwise(kind, a, b)
            return q, (ma + np.abs(q) * mb) / np.abs(b)
        if kind == "mul":
            # a chain: values and magnitudes each multiplied in the cheapest
            # bracketing (every bracketing is the same matrix)
            factors = []

            def flatten(n):
                if n[0] == "mul":
                    flatten(n[1])
                    flatten(n[2])
                else:
                    factors.append(self.vm(n))

            flatten(node)
            sv, sm = 1.0, 1.0
            vals, mags = [], []
            for v, m in factors:
                if _is_scalar(v):
                    sv, sm = sv * v, sm * m
                else:
                    vals.append(v)
                    mags.append(m)
            if not vals:
                return sv, sm
            return _product(vals) * sv, _product(mags) * sm
        if kind == "call":
            name, args = node[1], node[2]
            if name == "trans":
                v, m = self.vm(args[0])
                if _is_scalar(v):
                    return v, m
                return np.ascontiguousarray(v.T), np.ascontiguousarray(m.T)
            if name == "exp":
                v, m = self.vm(args[0])
                e = np.exp(v)
                return e, e * (1.0 + m)
            if name in ("diag", "diagmat", "trace"):
                # the same function of the magnitude: a diagonal entry keeps
                # its scale, a trace's error is bounded by the sum of them
                v, m = self.vm(args[0])
                return _diagonal_function(name, v), _diagonal_function(name, m)
            if name in ("col", "row", "submat"):
                v, m = self.vm(args[0])
                idx = [self.value(a) for a in args[1:]]
                return _submatrix(name, v, idx), _submatrix(name, m, idx)
            raise ValueError(f"magnitude: {name} has no componentwise scale")
        raise ValueError(f"unknown node {node!r}")


def magnitude(expr, env: dict):
    """The componentwise error scale M of ``expr`` over ``env`` (see
    ``_MagnitudeEvaluator``): a float64 array of the result's shape."""
    node = parse(expr) if isinstance(expr, str) else expr
    return _MagnitudeEvaluator(env, False).vm(node)[1]
