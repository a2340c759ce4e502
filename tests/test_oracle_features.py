"""Pins of the oracle features (Table 1) against closed forms and brute force."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle.features import accumulators, features_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute(rowptr, colind, n_cols, xb=8):
    """Table 1 definitions per row, with exact rationals."""
    n = len(rowptr) - 1
    Ls, bws, disps, qs, miss = [], [], [], [], 0
    for i in range(n):
        c = [int(t) for t in colind[rowptr[i]:rowptr[i + 1]]]
        L = len(c)
        bw = c[-1] - c[0] if L > 1 else 0
        Ls.append(L)
        bws.append(bw)
        disps.append(Fraction(L, bw + 1) if L else Fraction(0))
        qs.append((L * 2 ** 31) // (bw + 1) if L else 0)
        miss += sum(1 for k in range(1, L) if (c[k] - c[k - 1]) * xb > 128)
    return Ls, bws, disps, qs, miss


def laplace_geometry(n):
    """nnz_i, bw_i and misses_i of the 5-point Laplacian from grid geometry."""
    L, bw, miss = [], [], 0
    for i in range(n):
        for j in range(n):
            r = i * n + j
            cols = sorted(c for c, ok in [(r - n, i > 0), (r - 1, j > 0), (r, True),
                                          (r + 1, j < n - 1), (r + n, i < n - 1)] if ok)
            L.append(len(cols))
            bw.append(cols[-1] - cols[0])
            miss += sum(1 for a, b in zip(cols, cols[1:]) if (b - a) * 8 > 128)
    return L, bw, miss


def test_laplace64_closed_form():
    with open(os.path.join(GOLDEN, "laplace64_features.json")) as f:
        gold = json.load(f)
    rp, ci, _ = synth.laplace2d(64)
    feats, acc = features_ref(rp, ci, 4096)
    L, bw, miss = laplace_geometry(64)
    assert acc["N"] == gold["N"] == 4096
    assert acc["NNZ"] == gold["NNZ"] == sum(L) == 20224
    assert acc["nnz_min"] == gold["nnz_min"] == 3
    assert acc["nnz_max"] == gold["nnz_max"] == 5
    assert acc["S_bw"] == gold["S_bw"] == sum(bw) == 516222
    hist = {int(k): v for k, v in gold["bw_histogram"].items()}
    assert {b: bw.count(b) for b in set(bw)} == hist
    assert acc["S_miss"] == gold["S_miss"] == miss == 8064
    assert acc["S_L2"] == sum(t * t for t in L)
    assert acc["S_bw2"] == sum(t * t for t in bw)
    assert feats[2] == 79 / 16
    var = Fraction(gold["nnz_var"][0], gold["nnz_var"][1])
    assert var == Fraction(sum(t * t for t in L), 4096) - Fraction(sum(L), 4096) ** 2
    assert abs(feats[3] - math.sqrt(var)) <= 2e-16 * math.sqrt(var)
    assert feats[6] == gold["bw_avg"] == 258111 / 2048
    bw_var = Fraction(gold["bw_var"][0], gold["bw_var"][1])
    assert abs(feats[7] - math.sqrt(bw_var)) <= 4e-16 * math.sqrt(bw_var)
    disp = Fraction(gold["dispersion_avg"][0], gold["dispersion_avg"][1])
    assert abs(feats[8] - float(disp)) < 2.0 ** -31
    assert feats[10] == 8064 / 20224
    assert feats[11] == 1.0


def test_bruteforce_random_tiny():
    rng = np.random.default_rng(2024)
    for t in range(200):
        n = int(rng.integers(0, 30))
        m = int(rng.integers(1, 300))
        dens = float(rng.choice([0.0, 0.01, 0.05, 0.2, 0.6, 1.0]))
        rp, ci, _ = synth.tiny_random_csr(rng, n, m, dens)
        xb = int(rng.choice([4, 8]))
        feats, acc = features_ref(rp, ci, m, x_bytes=xb)
        if n == 0:
            assert feats == [0.0] * 12
            continue
        Ls, bws, disps, qs, miss = brute(rp, ci, m, xb)
        assert acc["nnz_min"] == min(Ls) and acc["nnz_max"] == max(Ls)
        assert acc["S_L2"] == sum(v * v for v in Ls)
        assert acc["S_bw"] == sum(bws) and acc["S_bw2"] == sum(v * v for v in bws)
        assert acc["S_q"] == sum(qs) and acc["S_q2"] == sum(v * v for v in qs)
        assert acc["S_miss"] == miss
        N = Fraction(n)
        avg = Fraction(sum(Ls)) / N
        sd = math.sqrt(sum((Fraction(v) - avg) ** 2 for v in Ls) / N)
        assert feats[0] == n and feats[1] == sum(Ls)
        assert abs(feats[2] - float(avg)) <= 1e-15 * max(1, float(avg))
        assert abs(feats[3] - sd) <= 1e-12 * max(1.0, sd)
        bavg = Fraction(sum(bws)) / N
        bsd = math.sqrt(sum((Fraction(v) - bavg) ** 2 for v in bws) / N)
        assert abs(feats[6] - float(bavg)) <= 1e-15 * max(1, float(bavg))
        assert abs(feats[7] - bsd) <= 1e-12 * max(1.0, bsd)
        davg = sum(disps) / N
        dsd = math.sqrt(sum((d - davg) ** 2 for d in disps) / N)
        assert abs(feats[8] - float(davg)) <= 2.0 ** -30
        assert abs(feats[9] - dsd) <= 1e-4 * max(dsd, 1e-3) + 2.0 ** -29
        nnz = sum(Ls)
        assert feats[10] == (miss / nnz if nnz else 0.0)


def test_row_permutation_invariant():
    rp, ci, _ = synth.banded(3000, 200, 300, seed=3)
    f0, _ = features_ref(rp, ci, 3000)
    perm = np.random.default_rng(5).permutation(3000)
    L = np.diff(rp)[perm]
    nrp = np.zeros(3001, dtype=np.int32)
    nrp[1:] = np.cumsum(L)
    nci = np.concatenate([ci[rp[p]:rp[p + 1]] for p in perm])
    f1, _ = features_ref(nrp, nci, 3000)
    assert f0 == f1


def test_identity_features():
    n = 1000
    f, _ = features_ref(np.arange(n + 1), np.arange(n), n)
    assert f[2:6] == [1.0, 0.0, 1.0, 1.0]
    assert f[6:11] == [0.0, 0.0, 1.0, 0.0, 0.0]


def test_column_shift_invariant():
    rp, ci, _ = synth.banded(2000, 100, 50, seed=8)
    f0, _ = features_ref(rp, ci, 5000)
    f1, _ = features_ref(rp, ci + 1234, 5000)
    assert f0 == f1


def test_sums_over_row_kinds_equal_sums_over_rows():
    """row_sums_of_kinds (rows given as kinds with multiplicities) equals
    row_sums over the rows written out, on random matrices grouped by their
    per-row quantities, with a kind of count 0 added (it must not count),
    and on an empty matrix."""
    from oracle.features import row_quantities, row_sums, row_sums_of_kinds
    rng = np.random.default_rng(11)
    for trial in range(20):
        n = int(rng.integers(1, 60))
        lens = rng.integers(0, 6, n)
        rp = np.concatenate([[0], np.cumsum(lens)])
        ci = np.concatenate([np.sort(rng.choice(500, int(L), replace=False)) for L in lens]
                            + [np.zeros(0, np.int64)]).astype(np.int64)
        per = row_quantities(rp, ci, 8)
        want = row_sums(*per)
        assert want == accumulators(rp, ci, 8)
        keys, counts = np.unique(np.stack(per, axis=1), axis=0, return_counts=True)
        cols = [np.append(keys[:, j], 7 + j) for j in range(4)]  # plus a kind of count 0
        assert row_sums_of_kinds(*cols, np.append(counts, 0)) == want, trial
    empty = [np.zeros(0, np.int64)] * 4
    assert row_sums_of_kinds(*empty, np.zeros(0, np.int64)) == row_sums(*empty)
