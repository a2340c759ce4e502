"""Structural matrix features of Table 1 (test infrastructure).

Per row i with L_i nonzeros and sorted columns c_0 < ... < c_{L-1}:

* ``bw_i``     column distance between the first and last nonzero (Table 1
               caption): c_{L-1} - c_0, and 0 for rows with at most one entry.
* ``disp_i``   L_i / distance_i (Table 1 caption).  The distance is read as
               the inclusive span bw_i + 1, so single-entry rows have
               dispersion 1; it is held in Q31 fixed point as
               q_i = floor(2**31 * L_i / (bw_i + 1)) (0 for an empty row).
* ``misses_i`` entries of the row, after its first, whose distance from the
               previous entry of the same row exceeds the cache line
               (Table 1 caption): (c_k - c_{k-1}) * xb > 128 with xb the size
               of an x element and a 128-byte line.

Readings where the paper is silent: empty rows count in N and add 0 to
every sum (nnz_min may be 0); the standard deviations are the population
ones (1/N) printed in Table 1; ``miss_ratio`` is stored per nonzero (the
paper's per-row value is miss_per_nnz * NNZ / N); ``size`` tests the CSR
working set 4(N+1) + (4+vb) NNZ + xb M + yb N against a 256 MiB last-level
cache.

Twelve features are returned, in this order:
N, NNZ, nnz_avg, nnz_sd, nnz_max, nnz_min, bw_avg, bw_sd,
dispersion_avg, dispersion_sd, miss_per_nnz, size.

All sums are exact integers; the finalisation is a fixed sequence of
single IEEE double operations (``float(int)`` rounds to nearest even).
"""
from __future__ import annotations

import math

import numpy as np

LINE_BYTES = 128
LLC_BYTES = 256 * 2 ** 20
Q31 = 2 ** 31

FEATURE_NAMES = ["N", "NNZ", "nnz_avg", "nnz_sd", "nnz_max", "nnz_min",
                 "bw_avg", "bw_sd", "dispersion_avg", "dispersion_sd",
                 "miss_per_nnz", "size"]


def row_quantities(rowptr, colind, x_bytes: int = 8):
    """(L, bw, q, misses) per row as int64 arrays."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    n = len(rowptr) - 1
    L = np.diff(rowptr)
    nonempty = L > 0
    first = np.zeros(n, dtype=np.int64)
    last = np.zeros(n, dtype=np.int64)
    first[nonempty] = colind[rowptr[:-1][nonempty]]
    last[nonempty] = colind[rowptr[1:][nonempty] - 1]
    bw = np.where(L > 1, last - first, 0)
    q = np.where(nonempty, (L << 31) // (bw + 1), 0)
    # misses: consecutive pairs (k-1, k) inside one row whose gap is too long
    misses = np.zeros(n, dtype=np.int64)
    nnz = len(colind)
    if nnz > 1:
        gap_miss = (np.diff(colind) * x_bytes) > LINE_BYTES   # pair (k-1, k)
        row_of = np.repeat(np.arange(n, dtype=np.int64), L)
        same_row = row_of[1:] == row_of[:-1]
        hit = gap_miss & same_row
        np.add.at(misses, row_of[1:][hit], 1)
    return L, bw, q, misses


def accumulators(rowptr, colind, x_bytes: int = 8) -> dict:
    """Exact integer sums over rows (Python ints)."""
    return row_sums(*row_quantities(rowptr, colind, x_bytes))


def row_sums(L, bw, q, misses) -> dict:
    """The exact sums over rows of the per-row quantities (int64 arrays, as
    row_quantities gives them)."""
    n = len(L)
    Lo = L.astype(object)
    bwo = bw.astype(object)
    qo = q.astype(object)
    return {
        "N": n,
        "NNZ": int(np.sum(L)),
        "nnz_min": int(L.min()) if n else 0,
        "nnz_max": int(L.max()) if n else 0,
        "S_L2": int(np.dot(Lo, Lo)) if n else 0,
        "S_bw": int(np.sum(bwo)) if n else 0,
        "S_bw2": int(np.dot(bwo, bwo)) if n else 0,
        "S_q": int(np.sum(qo)) if n else 0,
        "S_q2": int(np.dot(qo, qo)) if n else 0,
        "S_miss": int(np.sum(misses)),
    }


def row_sums_of_kinds(L, bw, q, misses, counts) -> dict:
    """row_sums of a matrix whose rows come in a few kinds: entry j of the
    per-row arrays stands for counts[j] identical rows (exact Python ints)."""
    kinds = [(int(c), int(a), int(b), int(d), int(e))
             for c, a, b, d, e in zip(counts, L, bw, q, misses) if c > 0]
    n = sum(c for c, *_ in kinds)
    return {
        "N": n,
        "NNZ": sum(c * a for c, a, _, _, _ in kinds),
        "nnz_min": min(a for _, a, _, _, _ in kinds) if n else 0,
        "nnz_max": max(a for _, a, _, _, _ in kinds) if n else 0,
        "S_L2": sum(c * a * a for c, a, _, _, _ in kinds),
        "S_bw": sum(c * b for c, _, b, _, _ in kinds),
        "S_bw2": sum(c * b * b for c, _, b, _, _ in kinds),
        "S_q": sum(c * d for c, _, _, d, _ in kinds),
        "S_q2": sum(c * d * d for c, _, _, d, _ in kinds),
        "S_miss": sum(c * e for c, _, _, _, e in kinds),
    }


def finalize(acc: dict, n_cols: int, val_bytes: int = 8, x_bytes: int = 8,
             y_bytes: int = 8) -> list[float]:
    """The twelve FP64 features from the exact accumulators."""
    n, nnz = acc["N"], acc["NNZ"]
    if n == 0:
        return [0.0] * 12
    f0 = float(n)
    f1 = float(nnz)
    nn = f0 * f0
    nnz_avg = f1 / f0
    nnz_sd = math.sqrt(float(n * acc["S_L2"] - nnz * nnz) / nn)
    nnz_max = float(acc["nnz_max"])
    nnz_min = float(acc["nnz_min"])
    bw_avg = float(acc["S_bw"]) / f0
    bw_sd = math.sqrt(float(n * acc["S_bw2"] - acc["S_bw"] ** 2) / nn)
    disp_avg = (float(acc["S_q"]) / 2.0 ** 31) / f0
    disp_sd = math.sqrt(float(n * acc["S_q2"] - acc["S_q"] ** 2) / 2.0 ** 62 / nn)
    miss = float(acc["S_miss"]) / f1 if nnz > 0 else 0.0
    ws = 4 * (n + 1) + (4 + val_bytes) * nnz + x_bytes * n_cols + y_bytes * n
    size = 1.0 if ws <= LLC_BYTES else 0.0
    return [f0, f1, nnz_avg, nnz_sd, nnz_max, nnz_min, bw_avg, bw_sd,
            disp_avg, disp_sd, miss, size]


def features_ref(rowptr, colind, n_cols: int, val_bytes: int = 8,
                 x_bytes: int = 8, y_bytes: int = 8):
    """(features[12], accumulators) for a CSR pattern."""
    acc = accumulators(rowptr, colind, x_bytes)
    return finalize(acc, n_cols, val_bytes, x_bytes, y_bytes), acc
