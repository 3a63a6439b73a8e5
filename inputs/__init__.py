"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only draws random numbers and shapes them into matrices; it holds
none of the arithmetic of the expression evaluator. Every generator takes an
explicit seed and uses numpy's PCG64, so the same seed gives the same inputs on
any host. Matrices are returned column-major (Fortran order), the storage
convention of the BLAS/LAPACK routines the paper maps expressions onto
(Sec. I, Sec. II).

Workload recipes (the sizes and distributions of the evaluation workloads):

* ``small_chain_expr``   trans(A)*B*C*v + 0.5*(d % e), FP64, A 400x300,
                         B 400x600, C 600x200, v 200x1, d,e 300x1, N(0,1).
* ``fp32_chain``         5-matrix FP32 chain 8192x1024, 1024x8192, 8192x512,
                         512x4096, 4096x64, entries N(0, 1/k) with k the
                         contraction length of that factor.
* ``fp32_elementwise``   0.5*exp(-(A%A)) + B/C over n x n FP32, A,B ~ N(0,1),
                         C ~ U[1,2].
* ``svd_matrix``         U diag(s) V^T with Haar-distributed orthonormal
                         factors and geometric singular values (condition
                         number fixed by the caller).
* ``batched_instances``  n = round(exp(U[ln 8, ln 512])) per instance,
                         diagonally dominant S.
* ``random_chains``      chains of length U{3..8}, dims log-uniform [16, 8192].
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng", "normal", "uniform", "small_ints", "small_chain_expr", "fp32_chain",
    "fp32_chain_dims", "fp32_elementwise", "haar_orthonormal", "svd_matrix",
    "batched_sizes", "diag_dominant", "batched_instances", "random_chain_dims",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def normal(g: np.random.Generator, rows: int, cols: int, dtype=np.float64,
           std: float = 1.0) -> np.ndarray:
    x = g.standard_normal((rows, cols))
    if std != 1.0:
        x *= std
    return np.asfortranarray(x.astype(dtype))


def uniform(g: np.random.Generator, rows: int, cols: int, lo: float, hi: float,
            dtype=np.float64) -> np.ndarray:
    return np.asfortranarray(g.uniform(lo, hi, (rows, cols)).astype(dtype))


def small_ints(g: np.random.Generator, rows: int, cols: int, lo: int = -8,
               hi: int = 8, dtype=np.float64) -> np.ndarray:
    """Integers in [lo, hi]: sums of products stay exactly representable."""
    return np.asfortranarray(g.integers(lo, hi + 1, (rows, cols)).astype(dtype))


# ---------------------------------------------------------------- workloads

SMALL_CHAIN_EXPR = "trans(A)*B*C*v + 0.5*(d % e)"


def small_chain_expr(seed: int = 1000, dtype=np.float64) -> dict:
    g = rng(seed)
    return {
        "A": normal(g, 400, 300, dtype), "B": normal(g, 400, 600, dtype),
        "C": normal(g, 600, 200, dtype), "v": normal(g, 200, 1, dtype),
        "d": normal(g, 300, 1, dtype), "e": normal(g, 300, 1, dtype),
    }


FP32_CHAIN_DIMS = (8192, 1024, 8192, 512, 4096, 64)


def fp32_chain_dims(scale: int = 1) -> tuple:
    """Dims of the 5-factor chain, optionally divided by ``scale`` (>=1)."""
    return tuple(max(1, d // scale) for d in FP32_CHAIN_DIMS)


def fp32_chain(seed: int = 1001, dims=FP32_CHAIN_DIMS, dtype=np.float32) -> list:
    """Factors M_i (dims[i] x dims[i+1]) with entries N(0, 1/k_i).

    k_i is the contraction length the factor takes part in: the column count
    of the first factor, the row count of the others, so products stay O(1).
    """
    g = rng(seed)
    out = []
    for i in range(len(dims) - 1):
        r, c = dims[i], dims[i + 1]
        k = c if i == 0 else r
        out.append(normal(g, r, c, dtype, std=1.0 / math.sqrt(k)))
    return out


ELEMENTWISE_EXPR = "0.5*exp(-(A%A)) + B/C"


def fp32_elementwise(seed: int = 1001, n: int = 16384, cols: int | None = None,
                     dtype=np.float32) -> dict:
    g = rng(seed + 7)
    c = n if cols is None else cols
    return {"A": normal(g, n, c, dtype), "B": normal(g, n, c, dtype),
            "C": uniform(g, n, c, 1.0, 2.0, dtype)}


def haar_orthonormal(g: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Columns of a Haar-distributed orthonormal matrix (QR of a Gaussian with
    the signs of R's diagonal moved into Q)."""
    z = g.standard_normal((rows, cols))
    q, r = np.linalg.qr(z)
    q *= np.sign(np.diag(r))[None, :]
    return q


def svd_matrix(seed: int, rows: int, cols: int, cond: float,
               dtype=np.float64) -> tuple:
    """X = U diag(s) V^T, s_i = cond^(-(i-1)/(n-1)); returns (X, U, s, V)."""
    g = rng(seed)
    n = min(rows, cols)
    u = haar_orthonormal(g, rows, n)
    v = haar_orthonormal(g, cols, n)
    s = cond ** (-np.arange(n) / max(n - 1, 1))
    x = (u * s[None, :]) @ v.T
    return np.asfortranarray(x.astype(dtype)), u, s, v


def batched_sizes(g: np.random.Generator, count: int, lo: int = 8,
                  hi: int = 512) -> np.ndarray:
    return np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def diag_dominant(g: np.random.Generator, n: int, dtype=np.float64) -> np.ndarray:
    """Off-diagonal N(0,1); s_jj = 1 + max(row, column) off-diagonal abs sum,
    so S is strictly dominant by rows and by columns."""
    s = g.standard_normal((n, n))
    np.fill_diagonal(s, 0.0)
    d = 1.0 + np.maximum(np.abs(s).sum(axis=0), np.abs(s).sum(axis=1))
    s[np.arange(n), np.arange(n)] = d
    return np.asfortranarray(s.astype(dtype))


BATCHED_EXPR = "trans(A)*B*v + solve(S,b) + 2*(p % q)"


def batched_instances(seed: int = 1003, count: int = 10000, lo: int = 8,
                      hi: int = 512, dtype=np.float32) -> list:
    g = rng(seed)
    sizes = batched_sizes(g, count, lo, hi)
    out = []
    for n in sizes:
        n = int(n)
        out.append({
            "A": normal(g, n, n, dtype), "B": normal(g, n, n, dtype),
            "v": normal(g, n, 1, dtype), "S": diag_dominant(g, n, dtype),
            "b": normal(g, n, 1, dtype), "p": normal(g, n, 1, dtype),
            "q": normal(g, n, 1, dtype),
        })
    return out


def random_chain_dims(seed: int = 1005, count: int = 2000, lmin: int = 3,
                      lmax: int = 8, lo: int = 16, hi: int = 8192) -> list:
    """Chains of length L ~ U{lmin..lmax}; L+1 dims log-uniform in [lo, hi]."""
    g = rng(seed)
    out = []
    for _ in range(count):
        length = int(g.integers(lmin, lmax + 1))
        d = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), length + 1)))
        out.append(tuple(int(x) for x in d))
    return out


# ------------------------------------------------- device-side generation
# Large inputs are drawn directly on the GPU with torch's seeded Philox
# generator (same seed -> same values on any MI355X); a caller that needs them
# on the host copies them back.

def fp32_elementwise_device(seed: int = 1001, n: int = 16384, cols: int | None = None,
                            device: str = "cuda") -> dict:
    import torch
    c = n if cols is None else cols
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def colmajor_normal():
        return torch.randn((c, n), generator=g, device=device, dtype=torch.float32).t()

    a = colmajor_normal()
    b = colmajor_normal()
    cc = torch.rand((c, n), generator=g, device=device, dtype=torch.float32).t() + 1.0
    return {"A": a, "B": b, "C": cc}


def svd_matrix_device(seed: int, rows: int, cols: int, cond: float, device: str = "cuda",
                      dtype=None, return_u: bool = False):
    """Device version of ``svd_matrix`` for large shapes: X = U diag(s) V^T in
    float64 (torch's seeded generator and QR), returned as (X column-major in
    ``dtype`` (default float32), s, V[, U]) with s, V, U as float64 host arrays."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n = min(rows, cols)

    def haar(r, c):
        z = torch.randn((r, c), generator=g, device=device, dtype=torch.float64)
        q, rr = torch.linalg.qr(z)
        return q * torch.sign(torch.diagonal(rr))[None, :]

    u = haar(rows, n)
    v = haar(cols, n)
    s = cond ** (-torch.arange(n, device=device, dtype=torch.float64) / max(n - 1, 1))
    x = (u * s[None, :]) @ v.T
    xc = torch.empty((cols, rows), device=device, dtype=dtype or torch.float32).t()
    xc.copy_(x)
    del x
    out = (xc, s.cpu().numpy(), v.cpu().numpy())
    if return_u:
        out = out + (u.cpu().numpy(),)
    del u
    return out
