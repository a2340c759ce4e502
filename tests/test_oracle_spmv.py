"""Pins of the oracle SpMV (Algorithm 1) against mathematics, not itself."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import cref
from oracle.spmv import spmv_exact, spmv_seq, spmv_seq_rows, within_tolerance


def dense(rowptr, colind, val, n_cols):
    n = len(rowptr) - 1
    A = np.zeros((n, n_cols))
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            A[i, colind[k]] = val[k]
    return A


def random_cases(count=60, seed=7):
    rng = np.random.default_rng(seed)
    for t in range(count):
        n = int(rng.integers(0, 40))
        m = int(rng.integers(1, 50))
        dens = float(rng.choice([0.0, 0.05, 0.3, 0.9, 1.0]))
        yield synth.tiny_random_csr(rng, n, m, dens, int_valued=bool(t % 2 == 0)), m, rng


def test_dense_bruteforce_integer_exact():
    """Integer-valued A and x: every summation order is exact -> bit-equal."""
    for (rp, ci, v), m, rng in random_cases():
        if not np.all(v == np.round(v)):
            continue
        x = rng.integers(-1024, 1025, size=m).astype(np.float64)
        y = spmv_seq(rp, ci, v, x)
        ref = dense(rp, ci, v, m) @ x
        assert np.array_equal(y, ref)


def test_dense_bruteforce_real_values():
    for (rp, ci, v), m, rng in random_cases():
        x = rng.uniform(-1, 1, size=m)
        y = spmv_seq(rp, ci, v, x)
        ye, s = spmv_exact(rp, ci, v, x)
        ok, _ = within_tolerance(y, ye, s, 1e-14)
        assert ok
        np.testing.assert_allclose(y, dense(rp, ci, v, m) @ x, rtol=0, atol=1e-12)


def test_exact_reference_matches_fractions():
    """spmv_exact rounds the exact rational row sum once."""
    for (rp, ci, v), m, rng in random_cases(30, seed=11):
        x = rng.uniform(-1, 1, size=m) * 10.0 ** rng.integers(-8, 8, size=m)
        ye, _ = spmv_exact(rp, ci, v, x)
        for i in range(len(rp) - 1):
            tot = sum((Fraction(float(v[k])) * Fraction(float(x[ci[k]]))
                       for k in range(rp[i], rp[i + 1])), Fraction(0))
            assert ye[i] == float(tot)


def test_sequential_order_matches_python_loop_and_c():
    rp, ci, v = synth.powerlaw(3000, 109, 1500, seed=5)
    x = synth.vector(3000, 5)
    y = spmv_seq(rp, ci, v, x)
    rows = np.arange(0, 3000, 7)
    assert np.array_equal(y[rows], spmv_seq_rows(rp, ci, v, x, rows))
    yc, _ = cref.spmv(rp, ci, v, x)
    assert np.array_equal(y, yc)
    yo, _ = cref.spmv(rp, ci, v, x, threads=True)
    assert np.array_equal(y, yo)


def test_identity():
    n = 257
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    v = np.ones(n)
    x = synth.vector(n, 3)
    assert np.array_equal(spmv_seq(rp, ci, v, x), x)


def permute_rows(rp, ci, v, perm):
    """Row i of the result is row perm[i] of A (row order kept)."""
    L = np.diff(rp)[perm]
    nrp = np.zeros(len(rp), dtype=np.int32)
    nrp[1:] = np.cumsum(L)
    idx = np.concatenate([np.arange(rp[p], rp[p + 1]) for p in perm]) if len(perm) else np.zeros(0, int)
    return nrp, ci[idx], v[idx]


def test_row_permutation_bit_exact():
    rp, ci, v = synth.banded(500, 128, 40, seed=9)
    x = synth.vector(500, 9)
    perm = np.random.default_rng(0).permutation(500)
    y = spmv_seq(rp, ci, v, x)
    prp, pci, pv = permute_rows(rp, ci, v, perm)
    assert np.array_equal(spmv_seq(prp, pci, pv, x), y[perm])


def symmetric_permutation(rp, ci, v, perm):
    """P A P^T with columns re-sorted inside each row."""
    n = len(rp) - 1
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    prp, pci, pv = permute_rows(rp, ci, v, perm)
    newc = inv[pci]
    for i in range(n):
        a, b = prp[i], prp[i + 1]
        o = np.argsort(newc[a:b], kind="stable")
        newc[a:b] = newc[a:b][o]
        pv[a:b] = pv[a:b][o]
    return prp, newc.astype(np.int32), pv


@pytest.mark.parametrize("values", ["random", "int"])
def test_symmetric_permutation(values):
    rp, ci, v = synth.banded(400, 160, 30, seed=4, values=values)
    x = synth.vector(400, 4) if values == "random" else synth.int_vector(400, 4)
    perm = np.random.default_rng(1).permutation(400)
    y = spmv_seq(rp, ci, v, x)
    srp, sci, sv = symmetric_permutation(rp, ci, v, perm)
    yp = spmv_seq(srp, sci, sv, x[perm])
    if values == "int":
        assert np.array_equal(yp, y[perm])
    else:
        ye, s = spmv_exact(rp, ci, v, x)
        ok, _ = within_tolerance(yp, ye[perm], s[perm], 1e-14)
        assert ok


def test_laplace_closed_forms():
    """5-point Laplacian 64x64: x = 1 gives 5 - nnz_i; x_j = j gives 0 inside."""
    n = 64
    rp, ci, v = synth.laplace2d(n)
    N = n * n
    y = spmv_seq(rp, ci, v, np.ones(N))
    deg = np.diff(rp)
    assert np.array_equal(y, 5.0 - deg)
    assert (y == 0).sum() == (n - 2) ** 2 == 3844
    assert (y == 1).sum() == 4 * (n - 2) == 248
    assert (y == 2).sum() == 4
    assert y.sum() == 256
    y2 = spmv_seq(rp, ci, v, np.arange(N, dtype=np.float64))
    ii, jj = np.divmod(np.arange(N), n)
    interior = (ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1)
    assert np.all(y2[interior] == 0)


def test_stencil27_closed_form():
    """27-point box on 100^3 with 26 / -1: x = 1 gives 27 - nnz_i."""
    rp, ci, v = synth.stencil3d_27(100)
    assert len(ci) == 26463592
    y = spmv_seq(rp, ci, v, np.ones(10 ** 6))
    counts = {val: int((y == val).sum()) for val in (0.0, 9.0, 15.0, 19.0)}
    assert counts == {0.0: 98 ** 3, 9.0: 6 * 98 ** 2, 15.0: 12 * 98, 19.0: 8}
