"""The allocation-free merge-path entry point against the plan path.

spmv_merge_path_noalloc keeps its splits and carries in a static device
array shared by every call on the GPU; two calls in a row, the second on a
smaller matrix, must each give exactly what spmv_execute with MERGE_PATH
gives on the same data (same kernels), and lie within the oracle's
tolerance of the correctly rounded product.
"""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.spmv import spmv_exact, within_tolerance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import DEV, make_plan, upload_csr, x_tensor  # noqa: E402

TOL = {S.SPMV_F64: 1e-12, S.SPMV_F32: 1e-5, S.SPMV_BF16: 1e-2}


def plan_merge(rp, ci, v, m, dtype, x):
    plan = make_plan(rp, ci, v, m, dtype)
    plan.set_variant(S.V_MERGE_PATH)
    tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
    y = torch.full((max(len(rp) - 1, 1),), float("nan"), dtype=tdt, device=DEV)
    plan.execute(x_tensor(x, dtype), y)
    torch.cuda.synchronize()
    plan.close()
    return y[:len(rp) - 1].cpu().numpy()


def noalloc(rp, ci, v, m, dtype, x):
    r, c, vt = upload_csr(rp, ci, v, dtype)
    xt = x_tensor(x, dtype)
    tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
    n = len(rp) - 1
    y = torch.full((max(n, 1),), float("nan"), dtype=tdt, device=DEV)
    S.spmv_merge_path_noalloc(n, m, len(ci), r, c, vt, dtype, xt, y)
    torch.cuda.synchronize()
    return y[:n].cpu().numpy()


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16])
def test_noalloc_two_calls_match_plan_path(dtype):
    big = synth.powerlaw(30000, 109, 12000, seed=31)     # a long row across many tiles
    small = synth.random_rows(2500, 96, seed=32)         # fewer tiles on the second call
    for (rp, ci, v) in (big, small):
        n = len(rp) - 1
        x = synth.vector(n, 33)
        got = noalloc(rp, ci, v, n, dtype, x)
        want = plan_merge(rp, ci, v, n, dtype, x)
        assert np.array_equal(got, want), "allocation-free result differs from the plan path"
        y_ref, scale = spmv_exact(rp, ci, v, x)
        ok, worst = within_tolerance(got.astype(np.float64), y_ref, scale, TOL[dtype])
        assert ok, worst


def test_noalloc_edge_cases():
    # empty rows, a matrix with no nonzeros, and N = 0
    rp = np.array([0, 0, 3, 3, 5, 5], np.int32)
    ci = np.array([0, 2, 5, 1, 4], np.int32)
    v = np.array([1.0, -2.0, 3.0, 0.5, 4.0])
    x = synth.vector(6, 1)
    got = noalloc(rp, ci, v, 6, S.SPMV_F64, x)
    assert np.array_equal(got, plan_merge(rp, ci, v, 6, S.SPMV_F64, x))
    assert got[0] == 0 and got[2] == 0 and got[4] == 0
    rp0 = np.zeros(9, np.int32)
    got0 = noalloc(rp0, np.zeros(0, np.int32), np.zeros(0), 4, S.SPMV_F64, np.ones(4))
    assert np.array_equal(got0, np.zeros(8))
    S.spmv_merge_path_noalloc(0, 0, 0, torch.zeros(1, dtype=torch.int32, device=DEV), None, None,
                              S.SPMV_F64, None, None)
