"""Determinism and structural properties of the seeded generators."""
import numpy as np
import pytest

import synth


def check_csr(rp, ci, n_cols):
    assert rp.dtype == np.int32 and ci.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == len(ci) and np.all(np.diff(rp) >= 0)
    assert len(ci) == 0 or (ci.min() >= 0 and ci.max() < n_cols)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    d = np.diff(ci.astype(np.int64))
    same = rows[1:] == rows[:-1]
    assert np.all(d[same] > 0)


def test_hash_scalar_matches_vector():
    idx = np.array([0, 1, 2, 10 ** 9, 2 ** 40], dtype=np.int64)
    h = synth.hash_array(7, 3, idx)
    for i, v in zip(idx, h):
        assert int(v) == synth.h_int(7, 3, int(i))
    # SplitMix64 finaliser of 0 is 0; of the golden gamma a known constant
    assert synth.fmix_int(0) == 0


def test_splitmix_reference_sequence():
    """Published SplitMix64 with state 0: first outputs of next()."""
    state, out = 0, []
    for _ in range(3):
        state = (state + synth.G) & synth.MASK
        out.append(synth.fmix_int(state))
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("spec", synth.class_matrices(scale=500) + [synth.small_laplace()]
                         + [synth.sweep_spec(s, n_max=2e4) for s in range(1000, 1012)])
def test_families_valid_and_deterministic(spec):
    a = spec.build()
    b = spec.build()
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    n = len(a[0]) - 1
    check_csr(a[0], a[1], max(n, 1))
    assert np.all(np.abs(a[2]) <= 26)


def test_strata_one_column_per_stratum():
    rp, ci, _ = synth.uniform_random(500, 1000, 8, seed=3)
    for i in range(500):
        c = ci[rp[i]:rp[i + 1]]
        for j, col in enumerate(c):
            assert j * 1000 // 8 <= col < (j + 1) * 1000 // 8


def test_stencil_sizes():
    assert len(synth.laplace2d(64)[1]) == 5 * 64 * 64 - 4 * 64
    assert len(synth.stencil3d_7(10)[1]) == 7 * 1000 - 6 * 100
    assert len(synth.stencil2d_9(10)[1]) == 9 * 100 - 3 * 2 * 10 * 2 + 4


def test_pareto_lengths_exact_definition():
    rp, _, _ = synth.powerlaw(20000, 109, 5000, seed=3, force_long=False)
    L = np.diff(rp)
    k = (synth.hash_array(3, synth.ST_LEN, np.arange(20000)) >> np.uint64(32)).astype(np.int64)
    rhs = 109 ** 3 << 52
    for i in range(0, 20000, 37):
        kk = int(k[i]) + 1
        l = int(L[i])
        if 1 < l < 5000:
            assert l ** 3 * kk * kk <= rhs < (l + 1) ** 3 * kk * kk
        elif l == 1:
            assert 2 ** 3 * kk * kk > rhs
        else:
            assert l == 5000 and 5000 ** 3 * kk * kk <= rhs


def test_powerlaw_forced_row():
    spec = synth.class_matrices(scale=100)[2]
    rp, _, _ = spec.build()
    assert np.diff(rp).max() == 2000


def test_he_uniform_bounds():
    p = synth.he_uniform_params(0)
    assert p.dtype == np.float32 and len(p) == 5382
    assert np.abs(p[:768]).max() <= np.sqrt(0.5) and np.all(p[768:832] == 0)
