"""Device features are bit-identical to the oracle's (GPU)."""
import json
import os

import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.features import features_ref, row_quantities

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import make_plan  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def acc_words(acc):
    m = (1 << 64) - 1
    return [acc["nnz_min"], acc["nnz_max"], None, acc["S_L2"], acc["S_bw"], acc["S_bw2"] & m,
            acc["S_bw2"] >> 64, acc["S_q"], acc["S_q2"] & m, acc["S_q2"] >> 64,
            acc["S_miss"] & m, acc["NNZ"]]


MATS = {
    "laplace64": (lambda: synth.laplace2d(64), 4096),
    "stencil27_20": (lambda: synth.stencil3d_27(20), 8000),
    "random_4000x8": (lambda: synth.uniform_random(4000, 100000, 8, seed=2), 100000),
    "powerlaw_20000": (lambda: synth.powerlaw(20000, 109, 4000, seed=3), 20000),
    "shortrows": (lambda: synth.short_rows(9999, seed=4), 9999),
    "banded": (lambda: synth.banded(5000, 500, 3000, seed=5), 5000),
    "sweep_1001": (lambda: synth.sweep_spec(1001, n_max=3e4).build(), None),
    "sweep_1003": (lambda: synth.sweep_spec(1003, n_max=3e4).build(), None),
}


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32])
@pytest.mark.parametrize("name", list(MATS))
def test_features_bit_exact(name, dtype):
    build, m = MATS[name]
    rp, ci, v = build()
    m = m or (len(rp) - 1)
    xb = 8 if dtype == S.SPMV_F64 else 4
    want, acc = features_ref(rp, ci, m, val_bytes=8 if dtype == S.SPMV_F64 else 4, x_bytes=xb,
                             y_bytes=xb)
    plan = make_plan(rp, ci, v, m, dtype)
    got, words = plan.features()
    assert got == want, (name, got, want)
    exp = acc_words(acc)
    for i, w in enumerate(exp):
        if w is not None:
            assert words[i] == w, (i, words[i], w)
    _, bw, _, _ = row_quantities(rp, ci, xb)
    assert words[2] == (int(bw.max()) if len(bw) else 0)
    plan.close()


def test_laplace64_golden_values():
    gold = json.load(open(os.path.join(GOLDEN, "laplace64_features.json")))
    rp, ci, v = synth.laplace2d(64)
    plan = make_plan(rp, ci, v, 4096)
    f, w = plan.features()
    assert f[0] == 4096 and f[1] == gold["NNZ"] and f[2] == 79 / 16
    assert w[4] == gold["S_bw"] and w[10] == gold["S_miss"]
    assert f[4] == gold["nnz_max"] and f[5] == gold["nnz_min"]
    plan.close()


def test_features_row_permutation_invariant():
    rp, ci, v = synth.banded(3000, 300, 100, seed=9)
    perm = np.random.default_rng(0).permutation(3000)
    L = np.diff(rp)[perm]
    prp = np.zeros(3001, np.int32)
    prp[1:] = np.cumsum(L)
    pci = np.concatenate([ci[rp[p]:rp[p + 1]] for p in perm])
    a = make_plan(rp, ci, v, 3000)
    b = make_plan(prp, pci, v, 3000)
    assert a.features() == b.features()
    a.close()
    b.close()
