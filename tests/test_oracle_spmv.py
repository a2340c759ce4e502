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


# ---------------------------------------------------------------- Dot2
# The full-size accuracy reference (numpy and C) is Ogita-Rump-Oishi Dot2.
# Pins: the exact rational row sum within its published bound, exactness
# on integer data, and ill-conditioned rows where the plain sum loses every
# digit.
from oracle.spmv import spmv_dot2  # noqa: E402

U = 2.0 ** -53


def exact_rows(rp, ci, v, x):
    out = []
    for i in range(len(rp) - 1):
        out.append(sum((Fraction(float(v[k])) * Fraction(float(x[ci[k]]))
                        for k in range(rp[i], rp[i + 1])), Fraction(0)))
    return out


def dot2_bound_holds(y, scale, exact, rp):
    for i, tot in enumerate(exact):
        L = int(rp[i + 1] - rp[i])
        g = L * U / (1 - L * U)
        err = abs(Fraction(float(y[i])) - tot)
        assert err <= Fraction(U) * abs(tot) + Fraction(g * g) * Fraction(float(scale[i])) * 2, i


@pytest.mark.parametrize("impl", ["numpy", "c"])
def test_dot2_within_published_bound(impl):
    """|Dot2 - exact| <= u |exact| + gamma_L^2 sum|a||x| against Fractions,
    on wide-range values where plain summation is visibly worse."""
    f = spmv_dot2 if impl == "numpy" else cref.dot2
    for (rp, ci, v), m, rng in random_cases(40, seed=23):
        x = rng.uniform(-1, 1, size=m) * 10.0 ** rng.integers(-12, 12, size=m)
        y, sc = f(rp, ci, v, x)
        dot2_bound_holds(y, sc, exact_rows(rp, ci, v, x), rp)


@pytest.mark.parametrize("impl", ["numpy", "c"])
def test_dot2_ill_conditioned_rows(impl):
    """Rows whose terms cancel to far below their size: the plain sum is off
    by about the largest term, Dot2 recovers the exact (representable) sum."""
    f = spmv_dot2 if impl == "numpy" else cref.dot2
    rows = [[1e16, 1.0, -1e16], [2.0 ** 60, 3.0, -(2.0 ** 60), 5.0],
            [1.0, 1e100, 1.0, -1e100], [0.1, 0.2, -0.3]]
    rp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    v = np.concatenate([np.asarray(r) for r in rows])
    ci = np.concatenate([np.arange(len(r)) for r in rows]).astype(np.int32)
    x = np.ones(4)
    y, sc = f(rp, ci, v, x)
    exact = exact_rows(rp, ci, v, x)
    assert y[0] == 1.0 and y[1] == 8.0 and y[2] == 2.0
    assert y[3] == float(exact[3])          # 0.1 + 0.2 - 0.3 in exact rationals
    assert spmv_seq(rp, ci, v, x)[0] == 0.0  # the plain sum loses the 1
    assert sc[0] == 2e16 + 1.0


def test_dot2_integer_rows_exact_and_agree():
    """Integer data: Dot2 is exact; numpy and C give the same bits on a
    power-law matrix with long rows (same operations in the same order)."""
    for (rp, ci, v), m, rng in random_cases(30, seed=29):
        if not np.all(v == np.round(v)):
            continue
        x = rng.integers(-1024, 1025, size=m).astype(np.float64)
        y, _ = spmv_dot2(rp, ci, v, x)
        assert np.array_equal(y, dense(rp, ci, v, m) @ x)
    rp, ci, v = synth.powerlaw(3000, 109, 1500, seed=6)
    x = synth.vector(3000, 6)
    yn, sn = spmv_dot2(rp, ci, v, x)
    yc, sc = cref.dot2(rp, ci, v, x)
    assert np.array_equal(yn, yc)
    rows = np.arange(0, 3000, 11)
    ye, se = spmv_exact(rp, ci, v, x, rows)
    assert np.array_equal(yn[rows], ye) or np.all(np.abs(yn[rows] - ye) <= U * np.abs(ye))
    np.testing.assert_allclose(sn[rows], se, rtol=1e-12)


def test_seq_parallel_c_matches_sequential():
    rp, ci, v = synth.powerlaw(3000, 109, 1500, seed=8)
    x = synth.vector(3000, 8)
    assert np.array_equal(cref.seq(rp, ci, v, x), spmv_seq(rp, ci, v, x))
