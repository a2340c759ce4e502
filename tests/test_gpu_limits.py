"""Matrices at the size limits of the boundary, over M = 2^31 - 1 columns
(the largest column count), rows of 1024 nonzeros, one of 1023, then 64
empty rows:

* NNZ = 2^31 - 2^16 - 1, the largest a plan takes (2^21 rows), in two
  patterns:
  - spread: row i holds columns a_i + k 2^21 (k < 1024), a_i in
    [0, 2^21 - 2], so every row reaches across all of x and row 0 ends at
    column M - 1;
  - band: row i holds columns B + 252 i + k, B chosen so that the last
    nonempty row ends at column M - 1; 256-row blocks span 65283 columns,
    so delta16 takes it (rows streamed: the sliced layout needs NNZ < 2^30
    and reports infeasible) and 16-bit index codes fit;
* NNZ = 2^30 - 1, the largest the sliced delta16 layout takes (2^20 + 64
  rows), the band pattern: both layouts and both code widths.

Values and x are small integers (v = (i + 3k) mod 7 - 3, x_j = 5j mod 11 - 5),
so every row sum and every partial sum is an integer below 2^24: exact in
FP64, FP32 and BF16 in any order.  Hence every variant, dtype and index
coding must give the same y bit for bit, over all rows; sampled rows (the
first and last 256, and 512 seeded random ones) equal the oracle's
sequential sum of the same products.  The device arrays are generated with
torch from the closed forms above and checked against the same closed forms
in NumPy at the sampled rows.  The twelve features are compared bit for bit
with the oracle's sums of the per-row quantities over the kinds of rows
(rows of 1024, the row of 1023, empty rows), each kind's quantities computed
by the oracle on one row of it.  A last case takes the largest row count.
"""
from collections import namedtuple

import numpy as np
import pytest

import paper_1511_02494_amd as S
from oracle import cref
from oracle.features import finalize, row_quantities, row_sums_of_kinds

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import DEV  # noqa: E402

M = 2 ** 31 - 1
STRIDE = 1 << 21
A_MOD = (1 << 21) - 1

# rows [0, full) hold 1024 nonzeros, row full 1023, rows (full, n) none
Case = namedtuple("Case", "pattern n full")
CASES = [Case("spread", 1 << 21, (1 << 21) - 65), Case("band", 1 << 21, (1 << 21) - 65),
         Case("band", (1 << 20) + 64, (1 << 20) - 1)]
IDS = ["spread_nnz_2^31-2^16-1", "band_nnz_2^31-2^16-1", "band_nnz_2^30-1"]

TDT = {S.SPMV_F64: torch.float64, S.SPMV_F32: torch.float32, S.SPMV_BF16: torch.bfloat16}
DNAME = {S.SPMV_F64: "f64", S.SPMV_F32: "f32", S.SPMV_BF16: "bf16"}


def nnz_of(cs):
    return cs.full * 1024 + 1023


def band0(cs):
    return M - 1 - (252 * cs.full + 1022)


def row_len(cs, i):
    i = np.asarray(i, np.int64)
    return np.where(i < cs.full, 1024, np.where(i == cs.full, 1023, 0))


def cols_np(cs, i, k):
    """Column of position k of row i (int64, NumPy)."""
    if cs.pattern == "spread":
        return (A_MOD - 1) - (i * 40503) % A_MOD + k * STRIDE
    return band0(cs) + 252 * i + k


def vals_np(i, k):
    return ((i + 3 * k) % 7 - 3).astype(np.float64)


def x_np(j):
    return ((5 * np.asarray(j, np.int64)) % 11 - 5).astype(np.float64)


def sample_rows(cs):
    rng = np.random.default_rng(2024)
    rows = np.concatenate([np.arange(256), np.arange(cs.n - 256, cs.n),
                           rng.integers(256, cs.n - 256, 512)])
    return np.unique(rows)


def rowptr_dev(cs):
    i = torch.arange(cs.n + 1, dtype=torch.int64, device=DEV)
    rp = torch.clamp(i, max=cs.full) * 1024 + torch.where(i > cs.full, 1023, 0)
    return rp.to(torch.int32)


def matrix_dev(cs, dtype):
    """colind and values of the whole matrix on the device, in row chunks."""
    nnz = nnz_of(cs)
    ci = torch.empty(nnz, dtype=torch.int32, device=DEV)
    v = torch.empty(nnz, dtype=TDT[dtype], device=DEV)
    k = torch.arange(1024, dtype=torch.int64, device=DEV)[None, :]
    ch = 1 << 15
    for r0 in range(0, cs.full + 1, ch):
        r1 = min(r0 + ch, cs.full + 1)
        i = torch.arange(r0, r1, dtype=torch.int64, device=DEV)[:, None]
        if cs.pattern == "spread":
            c = (A_MOD - 1) - (i * 40503) % A_MOD + k * STRIDE
        else:
            c = band0(cs) + 252 * i + k
        vv = (i + 3 * k) % 7 - 3
        c, vv = c.reshape(-1), vv.reshape(-1)
        if r1 == cs.full + 1:  # row full holds 1023
            c, vv = c[:-1], vv[:-1]
        p0 = r0 * 1024
        ci[p0:p0 + c.numel()] = c.to(torch.int32)
        v[p0:p0 + c.numel()] = vv.to(TDT[dtype])
        del c, vv
    if dtype == S.SPMV_BF16:
        v = v.view(torch.int16)
    return ci, v


@pytest.fixture(scope="module")
def xs():
    x64 = torch.empty(M, dtype=torch.float64, device=DEV)
    ch = 1 << 28
    for j0 in range(0, M, ch):
        j = torch.arange(j0, min(j0 + ch, M), dtype=torch.int64, device=DEV)
        x64[j0:j0 + j.numel()] = ((5 * j) % 11 - 5).to(torch.float64)
        del j
    x32 = x64.to(torch.float32)
    yield {S.SPMV_F64: x64, S.SPMV_F32: x32, S.SPMV_BF16: x32}
    del x64, x32
    torch.cuda.empty_cache()


def expected(cs, rows):
    """The oracle's sequential sums of the sampled rows, and their CSR pieces
    (columns in the original numbering, values) for the device check."""
    L = row_len(cs, rows)
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    i = np.repeat(rows, L)
    k = np.arange(rp[-1]) - np.repeat(rp[:-1], L)
    c = cols_np(cs, i, k)
    v = vals_np(i, k)
    # x restricted to the columns the rows use, renumbered in increasing
    # order (the order inside each row is kept)
    uc, inv = np.unique(c, return_inverse=True)
    y = cref.seq(rp.astype(np.int32), inv.astype(np.int32), v, x_np(uc))
    return y, rp, c, v


def expected_features(cs, dtype):
    """Features of the whole matrix from the oracle's per-row quantities of
    one row of each kind, repeated over the rows of that kind."""
    xb = 8 if dtype == S.SPMV_F64 else 4
    vb = {S.SPMV_F64: 8, S.SPMV_F32: 4, S.SPMV_BF16: 2}[dtype]
    kinds = [0, cs.full, cs.n - 1]  # 1024, 1023 and 0 nonzeros
    counts = [cs.full, 1, cs.n - cs.full - 1]
    L = row_len(cs, kinds)
    rp = np.concatenate([[0], np.cumsum(L)])
    c = np.concatenate([cols_np(cs, r, np.arange(row_len(cs, r))) for r in kinds])
    per = row_quantities(rp, c, xb)
    return finalize(row_sums_of_kinds(*per, counts), M, vb, xb, xb)


def run_into(plan, x, n):
    y = torch.full((n,), float("nan"), dtype=x.dtype, device=DEV)
    plan.execute(x, y)
    torch.cuda.synchronize()
    return y.to(torch.float64)


@pytest.mark.parametrize("cs", CASES, ids=IDS)
def test_largest_matrices_every_variant(cs, xs):
    nnz = nnz_of(cs)
    sliced_ok = nnz < 2 ** 30
    rows = sample_rows(cs)
    y_exp, rp_s, c_s, v_s = expected(cs, rows)
    assert c_s.max() == M - 1  # the sampled rows hold the last column
    rp = rowptr_dev(cs)
    rows_t = torch.from_numpy(rows).to(DEV)
    y_first = None
    print(f"\n{cs.pattern}: n={cs.n} m={M} nnz={nnz}", flush=True)

    def check(y, name):
        nonlocal y_first
        assert not torch.isnan(y).any(), name
        got = y[rows_t].cpu().numpy()
        bad = np.flatnonzero(got != y_exp)
        assert len(bad) == 0, (name, rows[bad[:5]].tolist(), got[bad[:5]].tolist(),
                               y_exp[bad[:5]].tolist())
        if y_first is None:
            y_first = y
        else:
            assert torch.equal(y, y_first), (name, "differs from the first run")
        print(f"  {name}: {len(rows)} sampled rows equal the oracle, all rows equal the first run",
              flush=True)

    for dtype in (S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16):
        ci, v = matrix_dev(cs, dtype)
        if dtype == S.SPMV_F64:
            # the device input is the closed form at the sampled rows
            lens = torch.from_numpy(row_len(cs, rows)).to(DEV)
            first = torch.cumsum(lens, 0) - lens
            idx = (torch.repeat_interleave(rp[rows_t].to(torch.int64), lens)
                   + torch.arange(int(lens.sum()), device=DEV)
                   - torch.repeat_interleave(first, lens))
            assert np.array_equal(ci[idx].cpu().numpy(), c_s), "device columns"
            assert np.array_equal(v[idx].cpu().numpy(), v_s), "device values"
            del idx
        x = xs[dtype]
        plan = S.Plan(rp, ci, v, M, dtype, nnz=nnz)
        assert plan.features()[0] == expected_features(cs, dtype), DNAME[dtype]
        mask = plan.mask()
        runs = [(var, S.SPMV_IDX_AUTO) for var in range(6) if (mask >> var) & 1]
        S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
        cmask = plan.mask()
        runs += [(var, S.SPMV_IDX_CODED) for var in (S.V_MERGE_PATH, S.V_XBLOCK_LDS, S.V_SHORT_ROW)
                 if (cmask >> var) & 1]
        want = (1 << S.V_CSR_SCALAR) | (1 << S.V_CSR_VECTOR) | (1 << S.V_MERGE_PATH) | \
            (1 << S.V_SHORT_ROW) | (1 << S.V_XBLOCK_LDS)
        if cs.pattern == "band":
            want |= 1 << S.V_DELTA16
            assert (cmask >> S.V_MERGE_PATH) & 1
        assert mask == want, bin(mask)
        for var, coding in runs:
            S.spmv_set_index_coding(plan.handle, coding)
            plan.set_variant(var)
            if coding == S.SPMV_IDX_CODED:
                assert plan.query(22) == 1
            name = f"{DNAME[dtype]}/{S.VARIANTS[var]}" + ("/coded" if coding == S.SPMV_IDX_CODED else "")
            check(run_into(plan, x, cs.n), name)
        if cs.pattern == "band":
            S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_AUTO)
            assert plan.query(14) == (1 if sliced_ok else 0)  # the layout the rule takes
            # the delta16 forms the rules did not pick
            for layout, bits in ((1, 8), (1, 16), (0, 0)):
                S.spmv_set_delta16_layout(plan.handle, layout)
                S.spmv_set_delta16_offset_bits(plan.handle, bits)
                if layout == 1 and not sliced_ok:
                    with pytest.raises(S.SpmvError) as e:
                        plan.set_variant(S.V_DELTA16)
                    assert e.value.status == S.SPMV_ERR_INFEASIBLE
                    continue
                plan.set_variant(S.V_DELTA16)
                assert plan.query(14) == layout and plan.query(17) == (bits or 16)
                check(run_into(plan, x, cs.n),
                      f"{DNAME[dtype]}/delta16 layout {layout} ({bits or 16}-bit codes)")
            S.spmv_set_delta16_layout(plan.handle, -1)
            S.spmv_set_delta16_offset_bits(plan.handle, 0)
        plan.close()
        del ci, v, plan
        torch.cuda.empty_cache()


# ---- the largest row count: N = 2^31 - 2 rows, the odd ones holding one
# nonzero on the diagonal (NNZ = 2^30 - 1, the last column N - 1 in use), the
# even ones empty.  Every variant, both delta16 layouts (the sliced one
# forced: 64-row slices of 32 rows with one diagonal), all dtypes.
TALL_N = 2 ** 31 - 2
TALL_NNZ = TALL_N // 2


def tall_expected(rows):
    L = rows % 2
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    r = rows[L == 1]
    y = cref.seq(rp.astype(np.int32), np.arange(len(r), dtype=np.int32), vals_np(r, 0),
                 x_np(r))
    return y


def tall_dev(dtype):
    rp = torch.empty(TALL_N + 1, dtype=torch.int32, device=DEV)
    ci = torch.empty(TALL_NNZ, dtype=torch.int32, device=DEV)
    v = torch.empty(TALL_NNZ, dtype=TDT[dtype], device=DEV)
    ch = 1 << 28
    for i0 in range(0, TALL_N + 1, ch):
        i = torch.arange(i0, min(i0 + ch, TALL_N + 1), dtype=torch.int64, device=DEV)
        rp[i0:i0 + i.numel()] = (i // 2).to(torch.int32)  # odd rows below i
        del i
    for k0 in range(0, TALL_NNZ, ch):
        k = torch.arange(k0, min(k0 + ch, TALL_NNZ), dtype=torch.int64, device=DEV)
        r = 2 * k + 1  # the k-th odd row
        ci[k0:k0 + k.numel()] = r.to(torch.int32)
        v[k0:k0 + k.numel()] = (r % 7 - 3).to(TDT[dtype])
        del k, r
    if dtype == S.SPMV_BF16:
        v = v.view(torch.int16)
    return rp, ci, v


def test_largest_row_count_every_variant(xs):
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([np.arange(256), np.arange(TALL_N - 256, TALL_N),
                                     rng.integers(256, TALL_N - 256, 512)]))
    y_exp = tall_expected(rows)
    rows_t = torch.from_numpy(rows).to(DEV)
    y_first = None
    print(f"\ntall: n={TALL_N} m={TALL_N} nnz={TALL_NNZ}", flush=True)
    kinds = np.array([0, 1])  # an empty row, a row with its diagonal
    for dtype in (S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16):
        rp, ci, v = tall_dev(dtype)
        if dtype == S.SPMV_F64:
            assert np.array_equal(rp[rows_t].cpu().numpy(), rows // 2), "device row pointers"
            odd = torch.from_numpy(rows[rows % 2 == 1] // 2).to(DEV)
            assert np.array_equal(ci[odd].cpu().numpy(), rows[rows % 2 == 1]), "device columns"
            assert np.array_equal(v[odd].cpu().numpy(), vals_np(rows[rows % 2 == 1], 0))
        x = xs[dtype]
        plan = S.Plan(rp, ci, v, TALL_N, dtype, nnz=TALL_NNZ)
        xb = 8 if dtype == S.SPMV_F64 else 4
        vb = {S.SPMV_F64: 8, S.SPMV_F32: 4, S.SPMV_BF16: 2}[dtype]
        per = row_quantities(np.array([0, 0, 1]), np.array([1]), xb)
        want_f = finalize(row_sums_of_kinds(*per, [TALL_N // 2, TALL_N // 2]), TALL_N, vb, xb, xb)
        assert plan.features()[0] == want_f, DNAME[dtype]
        mask = plan.mask()
        assert mask == 0b111111, bin(mask)
        runs = [(var, -1) for var in range(6)] + [(S.V_DELTA16, 1)]
        for var, layout in runs:
            if layout >= 0:
                S.spmv_set_delta16_layout(plan.handle, layout)
            plan.set_variant(var)
            name = f"{DNAME[dtype]}/{S.VARIANTS[var]}" + (f" layout {plan.query(14)}"
                                                          if var == S.V_DELTA16 else "")
            y = run_into(plan, x, TALL_N)
            assert not torch.isnan(y).any(), name
            got = y[rows_t].cpu().numpy()
            bad = np.flatnonzero(got != y_exp)
            assert len(bad) == 0, (name, rows[bad[:5]].tolist(), got[bad[:5]].tolist(),
                                   y_exp[bad[:5]].tolist())
            if y_first is None:
                y_first = y
            else:
                assert torch.equal(y, y_first), (name, "differs from the first run")
            del y
            print(f"  {name}: {len(rows)} sampled rows equal the oracle, all rows equal the "
                  f"first run", flush=True)
        assert plan.query(14) == 1
        plan.close()
        del rp, ci, v, plan
        torch.cuda.empty_cache()
