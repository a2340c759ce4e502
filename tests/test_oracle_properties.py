"""Property tests of the oracle on generated tiny CSR matrices (Hypothesis).

Each property is a definition written out independently of the oracle's own
code: the dense product, the layouts' slot formulas read back, the merge of
row ends and nonzeros, the column-sliced CSR put back together.
"""
import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from oracle.encode import (delta8_codes_ref, delta16_ref, delta16_sliced_ref, merge_search_ref,
                           merge_walk_ref, slice_csr_ref)
from oracle.spmv import spmv_seq

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True)


@st.composite
def csr(draw, max_rows=70, max_cols=50):
    n = draw(st.integers(0, max_rows))
    m = draw(st.integers(1, max_cols))
    density = draw(st.sampled_from([0.0, 0.03, 0.2, 0.6, 1.0]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    mask = rng.random((n, m)) < density
    dense = np.where(mask, rng.integers(-8, 9, (n, m)), 0).astype(np.float64)
    mask &= dense != 0
    rowptr = np.concatenate([[0], np.cumsum(mask.sum(axis=1))]).astype(np.int64)
    colind = np.nonzero(mask)[1].astype(np.int64)
    val = dense[mask]
    x = rng.integers(-8, 9, m).astype(np.float64)
    return rowptr, colind, val, m, dense, x


@st.composite
def spread_csr(draw):
    """A csr() matrix with its columns spread k apart (k = 1, 97 or 301), so
    that consecutive columns of a row are often 255 or more apart; xs is x
    placed at the spread columns (zeros between), so A_spread xs = dense x."""
    rowptr, colind, val, m, dense, x = draw(csr(max_rows=150, max_cols=60))
    k = draw(st.sampled_from([1, 97, 301]))
    xs = np.zeros(m * k)
    xs[::k] = x
    return rowptr, colind * k, val, m * k, dense, x, xs


@SETTINGS
@given(csr())
def test_sequential_spmv_is_the_dense_product(A):
    rowptr, colind, val, m, dense, x = A
    assert np.array_equal(spmv_seq(rowptr, colind, val, x), dense @ x)  # integers: exact


@SETTINGS
@given(csr(), st.sampled_from([1, 2, 5, 256]))
def test_delta16_offsets_rebuild_the_columns(A, H):
    rowptr, colind, val, m, dense, x = A
    ok, base, off = delta16_ref(rowptr, colind, H)
    assert ok
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    assert np.array_equal(base[rows // H].astype(np.int64) + off, colind)


@SETTINGS
@given(csr())
def test_sliced_layout_reads_back_as_the_matrix(A):
    rowptr, colind, val, m, dense, x = A
    n = len(rowptr) - 1
    L = delta16_sliced_ref(rowptr, colind, val)
    back = np.zeros_like(dense)
    for i in range(n):
        s, lane = divmod(i, 64)
        for k in range(L["width"][s]):
            slot = 128 * L["units"][s] + 128 * (k // 2) + 2 * lane + k % 2
            if L["kind"][s]:
                if (L["mask"][i] >> k) & 1:
                    back[i, i + L["diag"][32 * s + k]] += L["vals"][slot]
            elif k < rowptr[i + 1] - rowptr[i]:
                back[i, L["base"][s] + L["off"][slot]] += L["vals"][slot]
            else:
                assert L["vals"][slot] == 0
    assert np.array_equal(back, dense)


@SETTINGS
@given(csr(), st.sampled_from([1, 3, 8, 64]))
def test_merge_split_search_equals_walk(A, T):
    rowptr = A[0]
    si, sj = merge_search_ref(rowptr, T)
    wi, wj = merge_walk_ref(rowptr, T)
    assert np.array_equal(si, wi) and np.array_equal(sj, wj)


@SETTINGS
@given(csr(), st.sampled_from([1, 2, 4, 8]))
def test_column_slices_put_back_the_matrix(A, S):
    rowptr, colind, val, m, dense, x = A
    n = len(rowptr) - 1
    rps, cis = slice_csr_ref(rowptr, colind, m, S)
    width = (m + S - 1) // S
    back = np.zeros((n, m), dtype=bool)
    start = 0
    for s in range(S):
        rp = np.asarray(rps[s])
        for i in range(n):
            for c in cis[start + rp[i]:start + rp[i + 1]]:
                assert c // width == s and not back[i, c]
                back[i, c] = True
        start += rp[n]
    assert start == len(colind) and np.array_equal(back, dense != 0)


@SETTINGS
@given(spread_csr())
def test_delta8_codes_read_back_as_the_columns(A):
    """Walking a row's 8-bit codes from the slice's reference column, adding
    each code or taking the lane's next escape entry on code 255, at the
    documented places (code k of lane l of slice s at 128 (u_s + s) +
    256 (k // 4) + 4 l + k % 4, escape e at 64 (eunits_s + e) + l), gives
    the row's columns; a row uses at most E_s escapes."""
    rowptr, colind, val, m, dense, x, xs = A
    L = delta16_sliced_ref(rowptr, colind, val)
    C = delta8_codes_ref(rowptr, colind, L)
    for i in range(len(rowptr) - 1):
        s, lane = divmod(i, 64)
        if L["kind"][s]:
            continue
        c, e = int(L["base"][s]), 0
        for k in range(rowptr[i + 1] - rowptr[i]):
            code = int(C["codes"][128 * (int(L["units"][s]) + s) + 256 * (k // 4) + 4 * lane + k % 4])
            if code == 255:
                c = int(C["esc"][64 * (int(C["eunits"][s]) + e) + lane])
                e += 1
            else:
                c += code
            assert c == colind[rowptr[i] + k], (i, k)
        assert e <= C["E"][s]
