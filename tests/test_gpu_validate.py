"""CSR validation statuses (GPU)."""
import numpy as np
import pytest

import paper_1511_02494_amd as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import upload_csr  # noqa: E402

GOOD = (np.array([0, 2, 3, 5], np.int32), np.array([0, 2, 1, 0, 3], np.int32),
        np.arange(5, dtype=np.float64))


def status_of(rp, ci, v, m=4, n=None, nnz=None):
    r, c, vt = upload_csr(rp, ci, v)
    n = len(rp) - 1 if n is None else n
    nnz = len(ci) if nnz is None else nnz
    try:
        h = S.spmv_plan_create(n, m, nnz, r, c, vt, S.SPMV_F64)
    except S.SpmvError as e:
        return e.status
    S.spmv_plan_destroy(h)
    return S.SPMV_OK


def test_good_matrix():
    assert status_of(*GOOD) == S.SPMV_OK


@pytest.mark.parametrize("rp", [[1, 2, 3, 5], [0, 2, 3, 4], [0, 3, 2, 5], [0, 2, 7, 5], [0, -1, 3, 5]])
def test_bad_rowptr(rp):
    assert status_of(np.array(rp, np.int32), GOOD[1], GOOD[2]) == S.SPMV_ERR_CSR_ROWPTR


@pytest.mark.parametrize("ci", [[0, 4, 1, 0, 3], [-1, 2, 1, 0, 3], [0, 2, 1, 0, 99]])
def test_bad_column_range(ci):
    assert status_of(GOOD[0], np.array(ci, np.int32), GOOD[2]) == S.SPMV_ERR_CSR_COL_RANGE


@pytest.mark.parametrize("ci", [[2, 0, 1, 0, 3], [0, 2, 1, 3, 3], [1, 1, 1, 0, 3]])
def test_unsorted_or_duplicate(ci):
    assert status_of(GOOD[0], np.array(ci, np.int32), GOOD[2]) == S.SPMV_ERR_CSR_UNSORTED


def test_row_start_descent_is_allowed():
    # column drops across row boundaries only
    rp = np.array([0, 3, 3, 5, 6], np.int32)
    ci = np.array([1, 2, 3, 0, 1, 0], np.int32)
    assert status_of(rp, ci, np.ones(6), m=4) == S.SPMV_OK


def test_skip_validate_trusts_input():
    r, c, vt = upload_csr(np.array([0, 2, 3, 5], np.int32), np.array([2, 0, 1, 0, 3], np.int32),
                          np.ones(5))
    h = S.spmv_plan_create(3, 4, 5, r, c, vt, S.SPMV_F64, None, S.SPMV_SKIP_VALIDATE)
    S.spmv_plan_destroy(h)
