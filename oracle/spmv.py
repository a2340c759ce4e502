"""Plain CSR SpMV and its correctly rounded reference (test infrastructure).

Algorithm 1 of the paper (CSR SpMV, Section 2) as printed drops the
accumulation and writes the inner range as ``rowptr[i], rowptr[i+1]``.  The
reading used here: ``y[i]`` starts at +0.0 and every nonzero of the
half-open range ``[rowptr[i], rowptr[i+1])`` adds ``val[j] * x[colind[j]]``
(a separate multiply and add, in increasing ``j``).  Indices are 0-based.
"""
from __future__ import annotations

import math

import numpy as np


def spmv_seq(rowptr, colind, val, x) -> np.ndarray:
    """Algorithm 1: y_i = sum_j val[j] * x[colind[j]], sequentially in j.

    The loop over j is vectorised across rows (position p of every row that
    has more than p entries is added at step p), which keeps each row's own
    order of additions exactly sequential.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(rowptr) - 1
    y = np.zeros(n, dtype=np.float64)
    if n == 0:
        return y
    L = np.diff(rowptr)
    order = np.argsort(-L, kind="stable")       # longest rows first
    Ls = L[order]
    maxlen = int(Ls[0]) if n else 0
    # count[p] = number of rows with more than p entries
    for p in range(maxlen):
        cnt = int(np.searchsorted(-Ls, -p, side="left"))  # rows with L > p
        rows = order[:cnt]
        k = rowptr[rows] + p
        prod = val[k] * x[colind[k]]
        y[rows] = y[rows] + prod
    return y


def spmv_seq_rows(rowptr, colind, val, x, rows) -> np.ndarray:
    """Algorithm 1 restricted to the listed rows (pure Python per row)."""
    out = np.zeros(len(rows), dtype=np.float64)
    for t, i in enumerate(rows):
        s = 0.0
        for j in range(int(rowptr[i]), int(rowptr[i + 1])):
            s = s + float(val[j]) * float(x[colind[j]])
        out[t] = s
    return out


def _two_product(a: np.ndarray, b: np.ndarray):
    """Error-free product a*b = p + e (Dekker 1971, Veltkamp splitting).

    Exact when no overflow or underflow occurs; uses no fused multiply-add.
    """
    c = 134217729.0  # 2**27 + 1
    ta = c * a
    ah = ta - (ta - a)
    al = a - ah
    tb = c * b
    bh = tb - (tb - b)
    bl = b - bh
    p = a * b
    e = al * bl - (((p - ah * bh) - al * bh) - ah * bl)
    return p, e


def _two_sum(a: np.ndarray, b: np.ndarray):
    """Error-free sum a + b = s + e (Knuth's TwoSum, no branch)."""
    s = a + b
    z = s - a
    e = (a - (s - z)) + (b - z)
    return s, e


def spmv_dot2(rowptr, colind, val, x):
    """(y_ref, scale): every row's dot product by Dot2 of Ogita, Rump and
    Oishi (SIAM J. Sci. Comput. 26(6), 2005), and scale_i = sum |a_ij| |x_j|.

    Dot2 keeps the running sum p and accumulates the rounding errors of each
    product and each addition (both exact by the error-free transformations)
    in a second sum s; the row's result is p + s.  It is as accurate as the
    plain sum in twice the working precision followed by one rounding:
    |y_ref,i - exact_i| <= u |exact_i| + gamma_L^2 scale_i (u = 2^-53, L the
    row length).  Vectorised across rows as ``spmv_seq`` is: position p of
    every row longer than p is processed at step p, so each row sees its own
    products in column order.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(rowptr) - 1
    p = np.zeros(n)
    s = np.zeros(n)
    sc = np.zeros(n)
    if n == 0:
        return p, sc
    L = np.diff(rowptr)
    order = np.argsort(-L, kind="stable")
    Ls = L[order]
    for q in range(int(Ls[0])):
        cnt = int(np.searchsorted(-Ls, -q, side="left"))
        rows = order[:cnt]
        k = rowptr[rows] + q
        a, b = val[k], x[colind[k]]
        h, r = _two_product(a, b)
        sc[rows] = sc[rows] + np.abs(a) * np.abs(b)
        if q == 0:
            p[rows], s[rows] = h, r
        else:
            pn, e = _two_sum(p[rows], h)
            p[rows] = pn
            s[rows] = s[rows] + (e + r)
    return p + s, sc


def spmv_exact(rowptr, colind, val, x, rows=None):
    """Correctly rounded y_i and the scale s_i = sum |a_ij| |x_j|.

    Each product is split exactly into p + e, and ``math.fsum`` (Shewchuk's
    exact summation) rounds the exact row sum once.  ``rows`` restricts the
    computation to a subset (returned in that order).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(rowptr) - 1
    if rows is None:
        rows = np.arange(n)
    rows = np.asarray(rows, dtype=np.int64)
    y = np.zeros(len(rows))
    s = np.zeros(len(rows))
    for t, i in enumerate(rows):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        if a == b:
            continue
        av = val[a:b]
        xv = x[colind[a:b]]
        p, e = _two_product(av, xv)
        y[t] = math.fsum(np.concatenate([p, e]).tolist())
        s[t] = float(np.sum(np.abs(av) * np.abs(xv)))
    return y, s


def within_tolerance(y, y_ref, scale, tol):
    """|y - y_ref| <= tol * scale for every row; rows with scale 0 need y == 0."""
    y = np.asarray(y, dtype=np.float64)
    err = np.abs(y - y_ref)
    ok = err <= tol * scale
    zero = scale == 0
    ok[zero] = y[zero] == 0
    return bool(np.all(ok)), float(np.max(np.where(scale > 0, err / np.where(scale > 0, scale, 1), 0.0))) if len(y) else 0.0
