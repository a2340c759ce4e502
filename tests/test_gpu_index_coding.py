"""The index-coding axis: 16-bit column codes inside merge-path tiles, x-block
slice blocks and the rows-streamed layout (spmv_set_index_coding).

Checked through the C ABI against the oracle: the feasibility of every coded
form and the variant mask under the request, the stored references and
codes byte for byte, the coded results bit for bit equal to the same
variant on int32 columns (and within the oracle's tolerance of the correctly
rounded product), and the statuses of forms that do not exist.
"""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.encode import delta16_ref, merge_codes_ref, xblock_codes_ref
from oracle import cref
from oracle.spmv import spmv_exact, spmv_seq, within_tolerance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import make_plan, run  # noqa: E402

TOL = {S.SPMV_F64: 1e-12, S.SPMV_F32: 1e-5, S.SPMV_BF16: 1e-2}


def with_empty_rows():
    rp, ci, v = synth.banded(6000, 128, 700, seed=21)
    keep = np.ones(len(ci), bool)
    L = np.diff(rp)
    for i in range(0, len(L), 7):            # every 7th row empty
        keep[rp[i]:rp[i + 1]] = False
        L[i] = 0
    rp2 = np.zeros(len(rp), np.int32)
    rp2[1:] = np.cumsum(L)
    return rp2, ci[keep], v[keep]


MATS = {
    "banded_20k": (lambda: synth.banded(20000, 160, 300, seed=11), None),
    "powerlaw_30k": (lambda: synth.powerlaw(30000, 109, 12000, seed=31), None),
    "stencil27_24": (lambda: synth.stencil3d_27(24), None),
    "shortrows_50k": (lambda: synth.short_rows(50000, seed=12), None),
    "random_wide": (lambda: synth.uniform_random(20000, 300000, 6, seed=13), 300000),
    "empty_rows": (with_empty_rows, None),
}


def expected_mask(plan, rp, ci, m):
    n = len(rp) - 1
    bits = 0
    if plan.query(9):
        bits |= (1 << S.V_DELTA16) | (1 << S.V_SHORT_ROW)
    if merge_codes_ref(rp, ci)[0]:
        bits |= 1 << S.V_MERGE_PATH
    if plan.query(12) > 0 and xblock_codes_ref(rp, ci, m, plan.query(7), plan.query(25))[0]:
        bits |= 1 << S.V_XBLOCK_LDS
    return bits


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16])
@pytest.mark.parametrize("name", list(MATS))
def test_coded_forms_equal_int32_forms(name, dtype):
    build, m = MATS[name]
    rp, ci, v = build()
    n = len(rp) - 1
    m = m or n
    x = synth.vector(m, 5)
    y_ref, scale = spmv_exact(rp, ci, v, x)
    plan = make_plan(rp, ci, v, m, dtype)
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
    mask = plan.mask()
    assert mask == expected_mask(plan, rp, ci, m), (name, bin(mask))
    # the stored references and codes, byte for byte
    ok_m, base_m, off_m, _ = merge_codes_ref(rp, ci)
    assert plan.query(23) == int(ok_m)
    if ok_m:
        assert np.array_equal(S.spmv_plan_copy_format(plan.handle, 18, len(base_m)), base_m)
        assert np.array_equal(S.spmv_plan_copy_format(plan.handle, 19, len(ci)), off_m)
    if (mask >> S.V_XBLOCK_LDS) & 1:
        ok_x, base_x, off_x, _ = xblock_codes_ref(rp, ci, m, plan.query(7), plan.query(25))
        assert np.array_equal(S.spmv_plan_copy_format(plan.handle, 20, len(base_x)), base_x)
        assert np.array_equal(S.spmv_plan_copy_format(plan.handle, 21, len(off_x)), off_x)
    seq = spmv_seq(rp, ci, v, x) if dtype == S.SPMV_F64 else None
    for var in (S.V_MERGE_PATH, S.V_XBLOCK_LDS, S.V_SHORT_ROW):
        if not (mask >> var) & 1:
            with pytest.raises(S.SpmvError) as e:
                S.spmv_set_variant(plan.handle, var)
            assert e.value.status == S.SPMV_ERR_INFEASIBLE
            continue
        S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
        yc = run(plan, var, x, dtype)
        assert plan.query(22) == 1
        S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_I32)
        yi = run(plan, var, x, dtype)
        assert plan.query(22) == 0
        assert np.array_equal(yc, yi), (name, S.VARIANTS[var])
        ok, worst = within_tolerance(yc, y_ref, scale, TOL[dtype])
        assert ok, (name, S.VARIANTS[var], worst)
        if seq is not None and plan.query(21) == 1:
            assert np.array_equal(yc, seq), (name, S.VARIANTS[var])
    plan.close()


def test_coding_statuses():
    rp, ci, v = synth.banded(3000, 160, 200, seed=14)
    plan = make_plan(rp, ci, v, 3000)
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
    for var in (S.V_CSR_SCALAR, S.V_CSR_VECTOR):
        with pytest.raises(S.SpmvError) as e:
            S.spmv_set_variant(plan.handle, var)
        assert e.value.status == S.SPMV_ERR_INFEASIBLE
    S.spmv_set_variant(plan.handle, S.V_DELTA16)            # coded either way
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_I32)
    with pytest.raises(S.SpmvError) as e:
        S.spmv_set_variant(plan.handle, S.V_DELTA16)
    assert e.value.status == S.SPMV_ERR_INFEASIBLE
    assert not (plan.mask() >> S.V_DELTA16) & 1
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_AUTO)
    assert (plan.mask() >> S.V_DELTA16) & 1
    with pytest.raises(S.SpmvError) as e:
        S.spmv_set_index_coding(plan.handle, 2)
    assert e.value.status == S.SPMV_ERR_ARG
    plan.close()


def test_coded_bytes():
    """Algorithmic bytes: 2 instead of 4 per column index plus 4 per
    reference column (tile, slice block, row block)."""
    rp, ci, v = synth.banded(20000, 160, 300, seed=11)
    n, nnz = 20000, len(ci)
    plan = make_plan(rp, ci, v, n)
    plain = {var: plan.bytes(var) for var in (S.V_MERGE_PATH, S.V_XBLOCK_LDS, S.V_SHORT_ROW)}
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
    tiles = (n + nnz + 2047) // 2048
    assert plan.bytes(S.V_MERGE_PATH) == plain[S.V_MERGE_PATH] - 2 * nnz + 4 * tiles
    H, ns = plan.query(25), plan.query(7)
    assert plan.bytes(S.V_XBLOCK_LDS) == plain[S.V_XBLOCK_LDS] - 2 * nnz + 4 * ns * (-(-n // H))
    ok, base, _ = delta16_ref(rp, ci, plan.query(11))
    assert ok
    assert plan.bytes(S.V_SHORT_ROW) == plain[S.V_SHORT_ROW] - 2 * nnz + 4 * len(base)
    plan.close()


def with_empty_row_blocks():
    """A band of 1.2M rows whose 256-row blocks 1, 2 (mod 4) are empty, and
    the last block too: with more blocks than the workgroups that fit, the
    runs of a phased workgroup hold empty blocks between nonempty ones and
    at their end."""
    rp, ci, v = synth.banded(1_200_000, 80, 300, seed=23)
    L = np.diff(rp)
    n = len(L)
    blk = np.arange(n) // 256
    empty = (blk % 4 == 1) | (blk % 4 == 2) | (blk == (n - 1) // 256)
    keep = np.repeat(~empty, L)
    L = np.where(empty, 0, L)
    rp2 = np.zeros(len(rp), np.int32)
    rp2[1:] = np.cumsum(L)
    return rp2, ci[keep], v[keep]


@pytest.mark.parametrize("slices", [2, 4, 8])
def test_phased_coded_runs_over_empty_row_blocks(slices):
    """The phased x-block kernel streams a workgroup's row blocks as one run
    per slice; with 16-bit codes each position takes the reference column of
    the block that holds it, passing over empty blocks.  Coded equals int32
    bit for bit and both equal Algorithm 1's sequential sum (FP64), in every
    forced slice count."""
    rp, ci, v = with_empty_row_blocks()
    n = len(rp) - 1
    x = synth.vector(n, 6)
    seq = cref.seq(rp, ci, v, x)
    plan = make_plan(rp, ci, v, n)
    S.spmv_set_xblock_slices(plan.handle, slices)
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
    assert (plan.mask() >> S.V_XBLOCK_LDS) & 1
    yc = run(plan, S.V_XBLOCK_LDS, x)
    assert plan.query(22) == 1 and plan.query(16) > 1  # coded, phased, runs of blocks
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_I32)
    yi = run(plan, S.V_XBLOCK_LDS, x)
    assert plan.query(22) == 0 and plan.query(16) > 0
    assert np.array_equal(yc, yi), slices
    assert np.array_equal(yc, seq), slices
    plan.close()
