"""Conjugate gradients on a CSR matrix (test infrastructure).

The paper's selection is paid once per matrix and repaid over the SpMVs of
an iterative solver (Introduction; Section 5 on overhead).  This is the
textbook method of Hestenes and Stiefel (1952) for a symmetric positive
definite A, written plainly in FP64 with the oracle's SpMV:

    r = b - A x;  p = r;  rr = r.r
    repeat: q = A p;  alpha = rr / (p.q);  x = x + alpha p;  r = r - alpha q;
            rr' = r.r;  stop when sqrt(rr') <= rtol * ||b|| or after max_iters;
            beta = rr' / rr;  p = r + beta p;  rr = rr'
"""
from __future__ import annotations

import math

import numpy as np

from .spmv import spmv_seq


def cg_ref(rowptr, colind, val, b, x0=None, max_iters: int = 1000, rtol: float = 1e-8):
    """(x, iterations, ||r|| / ||b||, residual history) with r the updated residual."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - spmv_seq(rowptr, colind, val, x)
    p = r.copy()
    rr = float(r @ r)
    nb = math.sqrt(float(b @ b))
    hist = [math.sqrt(rr) / nb if nb > 0 else 0.0]
    it = 0
    if nb == 0.0 or math.sqrt(rr) <= rtol * nb:
        return x, 0, hist[-1], hist
    while it < max_iters:
        q = spmv_seq(rowptr, colind, val, p)
        alpha = rr / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        it += 1
        hist.append(math.sqrt(rr_new) / nb)
        if math.sqrt(rr_new) <= rtol * nb:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it, hist[-1], hist
