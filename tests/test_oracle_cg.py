"""Pins of the CG oracle: direct solves, the exact-arithmetic iteration bound,
distinct-eigenvalue counts and the true residual at exit."""
import numpy as np

import synth
from oracle.cg import cg_ref
from oracle.spmv import spmv_seq


def dense_csr(A):
    rp, ci, v = [0], [], []
    for row in A:
        nz = np.nonzero(row)[0]
        ci.extend(nz.tolist())
        v.extend(row[nz].tolist())
        rp.append(len(ci))
    return np.array(rp), np.array(ci), np.array(v)


def test_laplacian_solution_matches_direct_solve():
    rp, ci, v = synth.laplace2d(8)
    n = 64
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    b = synth.vector(n, 3)
    x, it, res, _ = cg_ref(rp, ci, v, b, rtol=1e-13)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    assert it <= n and res <= 1e-13


def test_diagonal_with_three_distinct_eigenvalues_takes_three_steps():
    d = np.array([1.0, 4.0, 9.0] * 7)
    rp, ci, v = dense_csr(np.diag(d))
    b = synth.vector(21, 4)
    x, it, res, _ = cg_ref(rp, ci, v, b, rtol=1e-12)
    assert it == 3
    assert np.allclose(x, b / d, rtol=1e-12)


def test_random_spd_converges_within_n_plus_slack():
    rng = np.random.default_rng(5)
    M = rng.normal(size=(30, 30))
    A = M @ M.T + 30 * np.eye(30)
    rp, ci, v = dense_csr(A)
    b = rng.normal(size=30)
    x, it, res, hist = cg_ref(rp, ci, v, b, rtol=1e-12)
    assert it <= 30 + 5
    true = np.linalg.norm(b - spmv_seq(rp, ci, v, x)) / np.linalg.norm(b)
    assert true <= 1e-11
    assert hist[0] == 1.0 and hist[-1] == res


def test_zero_rhs_and_max_iters():
    rp, ci, v = synth.laplace2d(6)
    x, it, res, _ = cg_ref(rp, ci, v, np.zeros(36))
    assert it == 0 and not x.any()
    _, it, res, _ = cg_ref(rp, ci, v, synth.vector(36, 1), max_iters=2, rtol=1e-14)
    assert it == 2 and res > 1e-14
