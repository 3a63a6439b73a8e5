"""bfloat16 rounding and the hi/lo splitting of FP32 values (test infrastructure).

The paper names BF16 as a future element type and cites its use for
higher-precision results (Sec. IV, the Henry et al. reference). The split
represents an FP32 value x as a sum of bfloat16 terms:
  hi  = rne(x)
  mid = rne(x - hi)             (x - hi is exact in FP32)
  lo  = rne(x - hi - mid)
and a product x*y is approximated by the term products whose combined
weight is at least 2^-16 relative: hi*hi + hi*mid + mid*hi (three products,
"BF16x3") or additionally mid*mid + hi*lo + lo*hi (six products, "BF16x6").

``rne`` is round-to-nearest, ties to even, on the FP32 bit pattern: keep the
top 16 bits, adding 0x7FFF plus the lowest kept bit before truncation. NaN
inputs stay NaN.
"""
from __future__ import annotations

import numpy as np


def rne(x) -> np.ndarray:
    """Nearest bfloat16 value of each float32 entry, returned as float32."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    keep = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + keep) >> np.uint64(16)) << np.uint64(16)
    out = rounded.astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = np.where(nan, np.float32(np.nan), out)
    return out


def split(x, terms: int = 2) -> list:
    """[hi, mid(, lo)] bfloat16 terms (as float32) of float32 ``x``."""
    x = np.asarray(x, dtype=np.float32)
    parts = []
    rest = x
    for _ in range(terms):
        t = rne(rest)
        parts.append(t)
        rest = (rest - t).astype(np.float32)
    return parts


def product_terms(terms: int, products: int) -> list:
    """Index pairs (i, j) of term products kept in the split product."""
    if terms == 2 and products == 3:
        return [(0, 0), (0, 1), (1, 0)]
    if terms == 3 and products == 6:
        return [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0)]
    raise ValueError("supported: 2 terms / 3 products, 3 terms / 6 products")


def split_gram(x, terms: int = 2, products: int = 3) -> np.ndarray:
    """Sum over kept (i, j) of t_i^T t_j, each term product formed in float64
    (bf16 x bf16 products are exact there): the value a split-BF16 X^T X
    approximates before FP32 accumulation."""
    parts = [p.astype(np.float64) for p in split(x, terms)]
    g = np.zeros((x.shape[1], x.shape[1]))
    for i, j in product_terms(terms, products):
        g += parts[i].T @ parts[j]
    return g
