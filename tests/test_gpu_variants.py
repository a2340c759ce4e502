"""Parity of the six SpMV variants with the oracle (GPU, through the C ABI)."""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.encode import delta8_codes_ref, delta16_offset_bits_ref, delta16_sliced_ref
from oracle.spmv import spmv_exact, spmv_seq, within_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import make_plan, run  # noqa: E402

TOL = {S.SPMV_F64: 1e-12, S.SPMV_F32: 1e-5, S.SPMV_BF16: 1e-2}
SEQ_ORDER = {S.V_CSR_SCALAR, S.V_SHORT_ROW, S.V_DELTA16}  # sum in column order


def one_long_row(n_cols=100_000, seed=0, values="random"):
    rp = np.array([0, n_cols], np.int32)
    ci = np.arange(n_cols, dtype=np.int32)
    v = synth.random_values(n_cols, seed) if values == "random" else synth.int_values(n_cols, seed)
    return rp, ci, v


def empty_rows_mix(seed=1):
    rng = np.random.default_rng(seed)
    return synth.tiny_random_csr(rng, 300, 200, 0.02, int_valued=False)


def ragged(seed=2, values="random"):
    # row lengths 0..3000 cycling through chunk and tile boundaries
    L = np.array([0, 1, 7, 8, 9, 255, 256, 257, 2047, 2048, 2049, 3000, 0, 0, 5] * 20)
    rp = np.zeros(len(L) + 1, np.int64)
    rp[1:] = np.cumsum(L)
    ci = synth.strata_columns(rp, np.zeros(len(L), np.int64), np.full(len(L), 4000, np.int64), seed)
    nnz = int(rp[-1])
    v = synth.random_values(nnz, seed) if values == "random" else synth.int_values(nnz, seed)
    return rp.astype(np.int32), ci, v


CASES = {
    "laplace64": (lambda v: synth.laplace2d(64, values="const" if v == "random" else "int"), 4096),
    "stencil27_12": (lambda v: synth.stencil3d_27(12, seed=3, values=v), 1728),
    "random_3000x8": (lambda v: synth.uniform_random(3000, 5000, 8, seed=4, values=v), 5000),
    "powerlaw_20000": (lambda v: synth.powerlaw(20000, 109, 6000, seed=5, values=v), 20000),
    "shortrows_5000": (lambda v: synth.short_rows(5000, seed=6, values=v), 5000),
    "banded_4000": (lambda v: synth.banded(4000, 160, 40, seed=7, values=v), 4000),
    "narrowband_3000": (lambda v: synth.banded(3000, 960, 32, seed=8, values=v), 3000),
    "ragged": (lambda v: ragged(values=v), 4000),
    "one_long_row": (lambda v: one_long_row(values=v), 100_000),
    "empty_rows": (lambda v: empty_rows_mix(), 200),
}


def expected_mask(plan):
    return S.spmv_variant_mask(plan.handle)


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16])
@pytest.mark.parametrize("case", list(CASES))
def test_variants_within_tolerance(case, dtype):
    build, m = CASES[case]
    rp, ci, v = build("random")
    x = synth.vector(m, 11)
    y_ref, scale = spmv_exact(rp, ci, v, x)
    y_seq = spmv_seq(rp, ci, v, x)
    plan = make_plan(rp, ci, v, m, dtype)
    mask = expected_mask(plan)
    print(f"case={case} dtype={dtype} n={len(rp) - 1} nnz={len(ci)} mask={mask:06b}", flush=True)
    for var in range(6):
        if not (mask >> var) & 1:
            with pytest.raises(S.SpmvError) as e:
                S.spmv_set_variant(plan.handle, var)
            assert e.value.status == S.SPMV_ERR_INFEASIBLE
            continue
        y = run(plan, var, x, dtype)
        ok, worst = within_tolerance(y, y_ref, scale, TOL[dtype])
        assert ok, (S.VARIANTS[var], worst)
        if dtype == S.SPMV_F64 and var in SEQ_ORDER:
            assert np.array_equal(y, y_seq), S.VARIANTS[var]
        y2 = run(plan, var, x, dtype)
        assert np.array_equal(y, y2), f"{S.VARIANTS[var]} not deterministic"
    plan.close()


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16])
@pytest.mark.parametrize("case", ["laplace64", "stencil27_12", "random_3000x8", "shortrows_5000",
                                  "banded_4000", "narrowband_3000", "ragged", "empty_rows"])
def test_delta16_both_layouts(case, dtype):
    """delta16 rows streamed, sliced with rows in order and sliced with rows
    sorted by length: FP64 in Algorithm 1's order bit for bit, FP32/BF16
    (Kahan on the ragged case's rows above 256) within tolerance,
    integer-valued inputs exact in every dtype."""
    build, m = CASES[case]
    rp, ci, v = build("random")
    x = synth.vector(m, 15)
    y_ref, scale = spmv_exact(rp, ci, v, x)
    y_seq = spmv_seq(rp, ci, v, x)
    ri, cii, vi = build("int")
    xi = synth.int_vector(m, 16)
    yi_seq = spmv_seq(ri, cii, vi, xi)
    for layout, srt in ((0, -1), (1, 0), (1, 1)):
        plan = make_plan(rp, ci, v, m, dtype)
        if not (plan.mask() >> S.V_DELTA16) & 1:
            plan.close()
            pytest.skip("delta16 infeasible")
        S.spmv_set_delta16_layout(plan.handle, layout)
        S.spmv_set_delta16_sort(plan.handle, srt)
        y = run(plan, S.V_DELTA16, x, dtype)
        assert S.spmv_plan_query(plan.handle, 14) == layout
        assert S.spmv_plan_query(plan.handle, 26) == max(srt, 0)
        ok, worst = within_tolerance(y, y_ref, scale, TOL[dtype])
        assert ok, (layout, srt, worst)
        if dtype == S.SPMV_F64:
            assert np.array_equal(y, y_seq), (layout, srt)
        assert np.array_equal(y, run(plan, S.V_DELTA16, x, dtype))
        plan.close()
        if case == "empty_rows":  # its generator has no integer-valued form
            continue
        plan = make_plan(ri, cii, vi, m, dtype)
        S.spmv_set_delta16_layout(plan.handle, layout)
        S.spmv_set_delta16_sort(plan.handle, srt)
        assert np.array_equal(run(plan, S.V_DELTA16, xi, dtype), yi_seq), (layout, srt)
        plan.close()


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16])
@pytest.mark.parametrize("case", ["narrowband_3000", "empty_rows", "banded_4000", "ragged",
                                  "random_3000x8", "powerlaw_20000", "stencil27_12", "laplace64"])
def test_delta16_code_widths_agree(case, dtype):
    """8-bit delta codes (escapes included) and 16-bit offsets decode to the
    same columns, so the kernels gather the same x entries and sum in the
    same order: identical results, FP64 equal to the sequential sum.  The
    stencil and the Laplacian have diagonal slices only (no codes stored),
    where forcing 8 bits must change nothing.  The same with rows sorted by
    length (offset slices only, every case then stores codes)."""
    build, m = CASES[case]
    rp, ci, v = build("random")
    x = synth.vector(m, 19)
    y_ref, scale = spmv_exact(rp, ci, v, x)
    y_seq = spmv_seq(rp, ci, v, x)
    plan = make_plan(rp, ci, v, m, dtype)
    S.spmv_set_delta16_layout(plan.handle, 1)
    for srt in (0, 1):
        S.spmv_set_delta16_sort(plan.handle, srt)
        S.spmv_set_delta16_offset_bits(plan.handle, 0)
        y_auto = run(plan, S.V_DELTA16, x, dtype)
        bits = S.spmv_plan_query(plan.handle, 17)
        L = delta16_sliced_ref(rp, ci, v, sort_rows=bool(srt))
        C = delta8_codes_ref(rp, ci, L)
        print(f"case={case} dtype={dtype} sorted={srt} automatic bits={bits} "
              f"escapes={C['escapes']}", flush=True)
        assert bits == delta16_offset_bits_ref(L["nnz_offset"], int(C["E"].sum()))
        assert within_tolerance(y_auto, y_ref, scale, TOL[dtype])[0]
        if dtype == S.SPMV_F64:
            assert np.array_equal(y_auto, y_seq), srt
        for req in (16, 8):
            S.spmv_set_delta16_offset_bits(plan.handle, req)
            assert S.spmv_plan_query(plan.handle, 17) == req
            assert np.array_equal(run(plan, S.V_DELTA16, x, dtype), y_auto), (srt, req)
    plan.close()


def test_delta16_layout_change_rebuilds():
    rp, ci, v = CASES["stencil27_12"][0]("random")
    x = synth.vector(1728, 17)
    y_seq = spmv_seq(rp, ci, v, x)
    plan = make_plan(rp, ci, v, 1728)
    run(plan, S.V_DELTA16, x)
    for layout, srt in ((0, -1), (1, -1), (-1, -1), (0, -1), (1, 1), (1, 0), (-1, 1), (-1, -1)):
        S.spmv_set_delta16_layout(plan.handle, layout)  # active variant: rebuilt at once
        S.spmv_set_delta16_sort(plan.handle, srt)
        xt = torch.from_numpy(np.asarray(x, np.float64)).to("cuda:0")
        y = torch.full((plan.n,), float("nan"), dtype=torch.float64, device="cuda:0")
        plan.execute(xt, y)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), y_seq), (layout, srt)
        assert S.spmv_plan_query(plan.handle, 26) == (1 if srt == 1 and layout != 0 else 0)
    plan.close()


@pytest.mark.parametrize("dtype", [S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16])
@pytest.mark.parametrize("case", ["laplace64", "stencil27_12", "random_3000x8", "powerlaw_20000",
                                  "shortrows_5000", "ragged", "one_long_row"])
def test_integer_valued_bit_exact(case, dtype):
    """|a|, |x| <= 8 and partial sums below 2^24: every order is exact."""
    build, m = CASES[case]
    rp, ci, v = build("int")
    x = synth.int_vector(m, 12)
    y_seq = spmv_seq(rp, ci, v, x)
    assert np.max(np.abs(y_seq), initial=0) < 2 ** 24
    plan = make_plan(rp, ci, v, m, dtype)
    mask = expected_mask(plan)
    for var in range(6):
        if (mask >> var) & 1:
            y = run(plan, var, x, dtype)
            assert np.array_equal(y, y_seq), (case, S.VARIANTS[var])
    plan.close()


@pytest.mark.parametrize("n,m", [(0, 0), (0, 5), (7, 0), (10, 10)])
def test_degenerate_empty(n, m):
    rp = np.zeros(n + 1, np.int32)
    plan = make_plan(rp, np.zeros(0, np.int32), np.zeros(0), m)
    f, _ = plan.features()
    if n == 0:
        assert f == [0.0] * 12
    else:
        assert f[0] == n and f[1:11] == [0.0] * 10
    for var in range(6):
        if (S.spmv_variant_mask(plan.handle) >> var) & 1:
            y = run(plan, var, np.zeros(m), S.SPMV_F64)
            assert np.all(y == 0) and len(y) == n
    plan.close()


def test_default_variant_is_csr_scalar():
    rp, ci, v = synth.laplace2d(16)
    plan = make_plan(rp, ci, v, 256)
    assert plan.variant == S.V_CSR_SCALAR
    plan.close()


def test_copy_inputs_flag():
    rp, ci, v = synth.banded(1000, 128, 20, seed=1)
    x = synth.vector(1000, 2)
    from gpu_util import upload_csr
    r, c, vt = upload_csr(rp, ci, v)
    plan = S.Plan(r, c, vt, 1000, flags=S.SPMV_COPY_INPUTS, nnz=len(ci))
    c.zero_()
    vt.zero_()
    y = run(plan, S.V_CSR_VECTOR, x)
    y_ref, s = spmv_exact(rp, ci, v, x)
    assert within_tolerance(y, y_ref, s, 1e-12)[0]
    plan.close()


@pytest.mark.parametrize("slices", [1, 2, 4, 8])
@pytest.mark.parametrize("case", ["stencil27_12", "random_3000x8", "powerlaw_20000", "ragged",
                                  "one_long_row", "empty_rows", "shortrows_5000"])
def test_xblock_every_slice_count(case, slices):
    """x blocking with each forced slice count (small matrices pick 1 slice by
    themselves): row-streaming and merge-path slice kernels, both dtypes paths."""
    build, m = CASES[case]
    rp, ci, v = build("random")
    x = synth.vector(m, 13)
    y_ref, scale = spmv_exact(rp, ci, v, x)
    for dtype in (S.SPMV_F64, S.SPMV_F32):
        plan = make_plan(rp, ci, v, m, dtype)
        S.spmv_set_xblock_slices(plan.handle, slices)
        y = run(plan, S.V_XBLOCK_LDS, x, dtype)
        assert S.spmv_plan_query(plan.handle, 7) == slices
        ok, worst = within_tolerance(y, y_ref, scale, TOL[dtype])
        assert ok, (slices, dtype, worst)
        assert np.array_equal(y, run(plan, S.V_XBLOCK_LDS, x, dtype))
        plan.close()


def skewed_long_rows(seed=21):
    """4000 x 40000: ten rows of 3000 nonzeros all in the first 5000 columns,
    ten of 3000 spread over every column (23% of the nonzeros), the rest 40 to
    60 nonzeros; integer values and x, so every summation order gives the
    exact product."""
    rng = np.random.default_rng(seed)
    n, m = 4000, 40000
    rows = []
    for i in range(n):
        if i % 400 == 7:
            c = rng.choice(5000, 3000, replace=False)
        elif i % 400 == 207:
            c = rng.choice(m, 3000, replace=False)
        else:
            c = rng.choice(m, rng.integers(40, 61), replace=False)
        rows.append(np.sort(c))
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    v = rng.integers(-8, 9, len(ci)).astype(np.float64)
    return rp, ci, v, m


def test_xblock_long_rows_in_one_slice_and_across_all():
    """Long rows cut into chunks at the slice boundaries: chunks of one slice
    only (most chunk workgroups of the other slices idle) and of every slice;
    exact with integer data at each slice count, and deterministic."""
    rp, ci, v, m = skewed_long_rows()
    x = np.random.default_rng(22).integers(-8, 9, m).astype(np.float64)
    dense = np.zeros(len(rp) - 1)
    for i in range(len(rp) - 1):
        dense[i] = float(np.dot(v[rp[i]:rp[i + 1]], x[ci[rp[i]:rp[i + 1]]]))
    for slices in (2, 4, 8):
        plan = make_plan(rp, ci, v, m)
        S.spmv_set_xblock_slices(plan.handle, slices)
        y = run(plan, S.V_XBLOCK_LDS, x)
        nlong = S.spmv_plan_query(plan.handle, 13)
        print(f"slices={slices} long rows={nlong}", flush=True)
        assert nlong == 20
        assert np.array_equal(y, dense), slices
        assert np.array_equal(y, run(plan, S.V_XBLOCK_LDS, x))
        plan.close()


@pytest.mark.parametrize("case", ["laplace64", "stencil27_12", "random_3000x8", "shortrows_5000",
                                  "banded_4000", "empty_rows", "powerlaw_20000", "ragged"])
def test_xblock_phased_walk_is_sequential(case):
    """Without long rows the slices are walked in order by one thread per
    row (no partial y): FP64 results are Algorithm 1's sums bit for bit."""
    build, m = CASES[case]
    rp, ci, v = build("random")
    x = synth.vector(m, 18)
    y_seq = spmv_seq(rp, ci, v, x)
    for slices in (1, 2, 4, 8):
        plan = make_plan(rp, ci, v, m)
        S.spmv_set_xblock_slices(plan.handle, slices)
        y = run(plan, S.V_XBLOCK_LDS, x)
        phased, nlong, rows = (S.spmv_plan_query(plan.handle, k) for k in (16, 13, 12))
        print(f"case={case} slices={slices} phased J={phased} long rows={nlong} rows/block={rows}", flush=True)
        assert (phased > 0) == (nlong == 0 and rows > 0)
        if phased:
            assert np.array_equal(y, y_seq), slices
        plan.close()


def slice_count_rule(n, m, nnz):
    """The automatic x-block slice count restated: double from 1 while a
    slice would hold more than 256 Ki columns and a slice row would keep at
    least 0.9 nonzeros on average, up to 8."""
    ns = 1
    while ns < 8 and m > 262144 * ns and 10 * nnz >= 9 * 2 * ns * n:
        ns *= 2
    return ns


@pytest.mark.parametrize("n,m,per,want", [(300_000, 1_200_000, 2, 2), (300_000, 1_200_000, 4, 4),
                                          (300_000, 2_200_000, 8, 8), (300_000, 200_000, 8, 1)])
def test_xblock_automatic_slice_count(n, m, per, want):
    rp, ci, v = synth.uniform_random(n, m, per, seed=9)
    assert slice_count_rule(n, m, len(ci)) == want
    plan = make_plan(rp, ci, v, m)
    S.spmv_set_variant(plan.handle, S.V_XBLOCK_LDS)
    assert S.spmv_plan_query(plan.handle, 7) == want
    plan.close()


def test_xblock_slice_count_change_rebuilds():
    rp, ci, v = CASES["powerlaw_20000"][0]("int")
    x = synth.int_vector(20000, 14)
    y_seq = spmv_seq(rp, ci, v, x)
    plan = make_plan(rp, ci, v, 20000)
    y1 = run(plan, S.V_XBLOCK_LDS, x)
    for k in (8, 2, 0, 4):
        S.spmv_set_xblock_slices(plan.handle, k)  # active variant: rebuilt at once
        xt = torch.from_numpy(np.asarray(x, np.float64)).to("cuda:0")
        y = torch.full((plan.n,), float("nan"), dtype=torch.float64, device="cuda:0")
        plan.execute(xt, y)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), y_seq), k
    assert np.array_equal(y1, y_seq)
    with pytest.raises(S.SpmvError) as e:
        S.spmv_set_xblock_slices(plan.handle, 3)
    assert e.value.status == S.SPMV_ERR_ARG
    plan.close()


NONFINITE = {
    "stencil27_12": CASES["stencil27_12"],        # diagonal slices, x shared across lanes
    "narrowband_3000": CASES["narrowband_3000"],  # offset slices, x window in LDS
    "shortrows_5000": CASES["shortrows_5000"],
}


@pytest.mark.parametrize("case", list(NONFINITE))
def test_nonfinite_x_reaches_only_the_rows_that_use_it(case):
    """x holds +inf, -inf and NaN at a few columns.  In every variant (both
    delta16 layouts) a row with no nonzero in those columns stays finite and
    within tolerance; the others are NaN or an infinity of the sign the
    column-order sum gives, whatever the order (kernels that read neighbour
    lanes' x, or a window of x around the row's columns, must drop what the
    row does not hold)."""
    build, m = NONFINITE[case]
    rp, ci, v = build("random")
    x = synth.vector(m, 11)
    rng = np.random.default_rng(12)
    bad = rng.choice(m, size=6, replace=False)
    x[bad[:2]] = np.inf
    x[bad[2:4]] = -np.inf
    x[bad[4:]] = np.nan
    with np.errstate(invalid="ignore"):
        want = spmv_seq(rp, ci, v, x)
    finite_x = x.copy()
    finite_x[bad] = 0.0
    touched = np.zeros(len(rp) - 1, bool)
    for i in range(len(rp) - 1):
        touched[i] = np.isin(ci[rp[i]:rp[i + 1]], bad).any()
    yr, s = spmv_exact(rp, ci, v, finite_x)
    plan = make_plan(rp, ci, v, m)
    mask = expected_mask(plan)
    runs = [(var, None) for var in range(6) if (mask >> var) & 1]
    if (mask >> S.V_DELTA16) & 1:
        runs += [(S.V_DELTA16, 0), (S.V_DELTA16, 1), (S.V_DELTA16, 2)]  # 2: sliced, rows sorted
    for var, layout in runs:
        if layout is not None:
            S.spmv_set_delta16_layout(plan.handle, min(layout, 1))
            S.spmv_set_delta16_sort(plan.handle, 1 if layout == 2 else 0)
        y = run(plan, var, x)
        name = (S.VARIANTS[var], layout)
        assert np.array_equal(np.isnan(y), np.isnan(want)), name
        assert np.array_equal(np.isinf(y), np.isinf(want)), name
        inf = np.isinf(want)
        assert np.array_equal(np.sign(y[inf]), np.sign(want[inf])), name
        assert np.all(np.isfinite(y[~touched])), name
        ok, _ = within_tolerance(y[~touched], yr[~touched], s[~touched], 1e-12)
        assert ok, name
    plan.close()
