"""Property tests through the C ABI: generated tiny integer-valued CSR
matrices (Hypothesis) give the dense product exactly in every feasible
variant, both delta16 layouts, both delta16 code widths (columns spread so
that codes escape) and every x-block slice count (GPU)."""
import numpy as np
import pytest

import paper_1511_02494_amd as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402
from gpu_util import make_plan, run  # noqa: E402
from test_oracle_properties import csr, spread_csr  # noqa: E402


@settings(max_examples=25, deadline=None, derandomize=True)
@given(csr(max_rows=150, max_cols=300))
def test_every_variant_gives_the_dense_product(A):
    rowptr, colind, val, m, dense, x = A
    want = dense @ x  # integers: every summation order is exact
    plan = make_plan(rowptr, colind, val, m)
    mask = S.spmv_variant_mask(plan.handle)
    for v in range(6):
        if (mask >> v) & 1:
            assert np.array_equal(run(plan, v, x), want), S.VARIANTS[v]
    if (mask >> S.V_DELTA16) & 1:
        for layout, srt in ((0, -1), (1, 0), (1, 1)):
            S.spmv_set_delta16_layout(plan.handle, layout)
            S.spmv_set_delta16_sort(plan.handle, srt)
            assert np.array_equal(run(plan, S.V_DELTA16, x), want), (layout, srt)
    for slices in (2, 8):
        S.spmv_set_xblock_slices(plan.handle, slices)
        assert np.array_equal(run(plan, S.V_XBLOCK_LDS, x), want), slices
    plan.close()


@settings(max_examples=25, deadline=None, derandomize=True)
@given(spread_csr())
def test_delta16_code_widths_give_the_dense_product(A):
    rowptr, colind, val, m, dense, x, xs = A
    want = dense @ x  # integers: exact
    plan = make_plan(rowptr, colind, val, m)
    if (S.spmv_variant_mask(plan.handle) >> S.V_DELTA16) & 1:
        S.spmv_set_delta16_layout(plan.handle, 1)
        for srt in (0, 1):
            S.spmv_set_delta16_sort(plan.handle, srt)
            for bits in (8, 16, 0):
                S.spmv_set_delta16_offset_bits(plan.handle, bits)
                assert np.array_equal(run(plan, S.V_DELTA16, xs), want), (srt, bits)
    plan.close()
