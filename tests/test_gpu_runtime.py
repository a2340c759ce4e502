"""Plan lifetime on the GPU: released device blocks are reused by later plans.

Derived formats of one plan land in blocks that held another plan's data;
every variant must still match the oracle (no kernel may rely on fresh or
zeroed memory), also after the kept blocks are given back.
"""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.spmv import spmv_exact

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import make_plan, run  # noqa: E402

MATS = [
    ("powerlaw_20000", lambda: synth.powerlaw(20000, 109, 6000, seed=5), 20000),
    ("random_3000x8", lambda: synth.uniform_random(3000, 5000, 8, seed=4), 5000),
    ("stencil27_12", lambda: synth.stencil3d_27(12, seed=3), 1728),
]


def check_all_variants(rp, ci, v, m, seed):
    x = synth.random_values(m, seed)
    y_ref, scale = spmv_exact(rp, ci, v, x)
    plan = make_plan(rp, ci, v, m)
    mask = plan.mask()
    for var in range(6):
        if (mask >> var) & 1:
            y = run(plan, var, x)
            assert np.all(np.abs(y - y_ref) <= 1e-12 * scale), S.VARIANTS[var]
    plan.close()


def test_reused_blocks_give_oracle_results():
    for rounds in range(2):
        for i, (name, build, m) in enumerate(MATS):
            rp, ci, v = build()
            print(f"round {rounds} {name}", flush=True)
            check_all_variants(rp, ci, v, m, seed=10 + i)
    S.spmv_release_cached_blocks()
    rp, ci, v = MATS[0][1]()
    check_all_variants(rp, ci, v, MATS[0][2], seed=20)
