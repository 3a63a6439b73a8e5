"""Error measures shared by the parity tests.

Two measures against the FP64 oracle, both from the tolerance reading of the
build (normwise relative Frobenius error, plus the componentwise error scaled
by the magnitude of the computation):

* ``rel(got, ref)`` -- ||got - ref||_F / ||ref||_F (absolute when ref is 0);
* ``comp(got, ref, mag)`` -- max_ij |got - ref|_ij / mag_ij, where ``mag`` is
  the oracle's componentwise scale (``oracle.magnitude``: |op(A)| |op(B)| for
  a product). Entries with mag == 0 must match exactly.

``bound(dtype, K)`` is K unit roundoffs of the storage type: a computation
whose longest path has K roundings (a length-k sum counts k) stays within
K u of the magnitude componentwise, to first order.
"""
import numpy as np

U = {np.float32: 2.0 ** -24, np.float64: 2.0 ** -53}
NORM_TOL = {np.float32: 1e-5, np.float64: 1e-12}
# split-BF16 products: per product, the dropped and rounded terms stay below
# 3 * 2^-16 (two terms, three products) or 6 * 2^-24 (three terms, six
# products) of |a| |b|
SPLIT_TERM = {"bf16x3": 3 * 2.0 ** -16, "bf16x6": 6 * 2.0 ** -24}


def rel(got, ref):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64).reshape(ref.shape)
    d = np.linalg.norm(got - ref)
    n = np.linalg.norm(ref)
    return d / n if n > 0 else d


def comp(got, ref, mag):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64).reshape(ref.shape)
    mag = np.asarray(mag, np.float64).reshape(ref.shape)
    if ref.size == 0:
        return 0.0
    d = np.abs(got - ref)
    zero = mag == 0
    if np.any(d[zero] != 0):
        return np.inf
    return float(np.max(np.where(zero, 0.0, d / np.where(zero, 1.0, mag))))


def bound(dtype, k):
    return float(k) * U[dtype]


def assert_close(got, ref, mag, dtype, k, norm_tol=None, extra=0.0, what=""):
    """Normwise within ``norm_tol`` (the storage type's tolerance by default)
    and componentwise within k unit roundoffs plus ``extra`` (per-product
    error of a split form) of the magnitude."""
    tol = NORM_TOL[dtype] if norm_tol is None else norm_tol
    e = rel(got, ref)
    c = comp(got, ref, mag)
    lim = bound(dtype, k) + extra
    assert e <= tol, f"{what} normwise {e:.3e} > {tol:.1e}"
    assert c <= lim, f"{what} componentwise {c:.3e} > {lim:.3e}"
    return e, c
