"""Full-size parity: the four FP64 class matrices at the sizes bench.py times.

Inputs come from the seeded CPU generator (never from the library).  Every
feasible variant runs in the bench's launch configuration (the plan's own
parameters), and EVERY row of y is compared with the oracle:

* against the accuracy reference y_ref (Ogita-Rump-Oishi Dot2 of the
  original FP64 data, as accurate as a twice-precision sum rounded once):
  |y_i - y_ref,i| <= tol * sum_j |a_ij| |x_j| with tol 1e-12 (FP64 values),
  1e-5 (FP32 values), 1e-2 (BF16 values), and y_i = 0 where that scale is 0;
* variants that sum every row in column order from +0 (plan query 21) equal
  Algorithm 1's sequential sum bit for bit in FP64.

The twelve features and their exact accumulators are compared bit for bit
with the oracle's on the same matrices, for FP64 and FP32 plans (the miss
feature and the working-set test depend on the x and value sizes), and on
the 2M-row band of the code-width report.
"""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle import cref
from oracle.encode import to_bf16_bits_ref, to_f32_ref
from oracle.features import features_ref, row_quantities

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import DEV, dev  # noqa: E402

TOL = {S.SPMV_F64: 1e-12, S.SPMV_F32: 1e-5, S.SPMV_BF16: 1e-2}
DNAME = {S.SPMV_F64: "f64", S.SPMV_F32: "f32", S.SPMV_BF16: "bf16"}
SPECS = synth.class_matrices(scale=1)
ACC_KEYS = ["nnz_min", "nnz_max", None, "S_L2", "S_bw", "S_bw2", None, "S_q", "S_q2", None,
            "S_miss", "NNZ"]


def upload_values(v, dtype):
    if dtype == S.SPMV_F64:
        return dev(v)
    if dtype == S.SPMV_F32:
        return dev(to_f32_ref(v))
    return dev(to_bf16_bits_ref(v).view(np.int16))


def check_whole_vector(y, y_ref, scale, tol, what):
    """Every row within tol * scale of the reference; exact zeros where the
    scale is zero.  Returns the largest |y - y_ref| / scale."""
    y = np.asarray(y, np.float64)
    err = np.abs(y - y_ref)
    bad = np.flatnonzero(err > tol * scale)
    assert len(bad) == 0, (what, f"{len(bad)} rows out of tolerance, first {bad[:5].tolist()}",
                           y[bad[:3]].tolist(), y_ref[bad[:3]].tolist())
    zero = scale == 0
    assert np.all(y[zero] == 0), (what, "nonzero result on a row whose scale is 0")
    return float(np.max(np.where(scale > 0, err / np.where(scale > 0, scale, 1), 0.0))) if len(y) else 0.0


def check_features(plan, rp, ci, n_cols, dtype, what):
    vb = {S.SPMV_F64: 8, S.SPMV_F32: 4, S.SPMV_BF16: 2}[dtype]
    xb = 8 if dtype == S.SPMV_F64 else 4
    f_ref, acc_ref = features_ref(rp, ci, n_cols, val_bytes=vb, x_bytes=xb, y_bytes=xb)
    feats, acc = plan.features()
    assert feats == f_ref, (what, feats, f_ref)
    mask64 = (1 << 64) - 1
    for k, name in enumerate(ACC_KEYS):
        if name is None:
            continue
        want = acc_ref[name]
        if name in ("S_bw2", "S_q2"):  # u128 as (lo, hi) words
            assert acc[k] == want & mask64 and acc[k + 1] == want >> 64, (what, name)
        else:
            assert acc[k] == want, (what, name, acc[k], want)
    _, bw, _, _ = row_quantities(rp, ci, xb)
    assert acc[2] == (int(bw.max()) if len(bw) else 0), (what, "bw_max")


@pytest.mark.parametrize("spec", SPECS, ids=[s.name for s in SPECS])
def test_fullsize_variants(spec):
    rp, ci, v = spec.build()
    n = len(rp) - 1
    x = spec.x(n)
    y_ref, scale = cref.dot2(rp, ci, v, x)
    y_seq = cref.seq(rp, ci, v, x)
    r_t, c_t = dev(rp), dev(ci)
    print(f"\n{spec.name}: n={n} nnz={len(ci)} (every row compared)", flush=True)
    for dtype in (S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16):
        v_t = upload_values(v, dtype)
        x_t = dev(x) if dtype == S.SPMV_F64 else dev(x.astype(np.float32))
        tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
        plan = S.Plan(r_t, c_t, v_t, n, dtype, nnz=len(ci))
        check_features(plan, rp, ci, n, dtype, f"{spec.name}/{DNAME[dtype]}")
        mask = plan.mask()
        runs = [(var, None) for var in range(6) if (mask >> var) & 1]
        if (mask >> S.V_DELTA16) & 1:  # the layout the rule did not pick, forced
            runs.append((S.V_DELTA16, 1 - plan.query(14)))
            runs.append((S.V_DELTA16, 2))  # sliced with rows sorted by length
        for var, layout in runs:
            if layout is not None:
                S.spmv_set_delta16_layout(plan.handle, min(layout, 1))
                S.spmv_set_delta16_sort(plan.handle, 1 if layout == 2 else -1)
            plan.set_variant(var)
            y = torch.full((n,), float("nan"), dtype=tdt, device=DEV)
            plan.execute(x_t, y)
            y2 = torch.full((n,), float("nan"), dtype=tdt, device=DEV)
            plan.execute(x_t, y2)
            torch.cuda.synchronize()
            name = S.VARIANTS[var] + ("" if layout is None else f"/layout{layout}")
            assert torch.equal(y, y2), f"{name} not deterministic"
            ys = y.cpu().numpy().astype(np.float64)
            rel = check_whole_vector(ys, y_ref, scale, TOL[dtype], (name, DNAME[dtype]))
            seq = dtype == S.SPMV_F64 and plan.query(21) == 1
            if seq:
                diff = np.flatnonzero(ys != y_seq)
                assert len(diff) == 0, (name, "differs from the sequential sum on rows",
                                        diff[:5].tolist())
            print(f"  {DNAME[dtype]:>4s} {name:>18s} max |y - y_ref| / sum|a||x| = {rel:.3e}"
                  f"{'  (= sequential sum)' if seq else ''}", flush=True)
            del y, y2
        plan.close()
        del v_t, x_t
        torch.cuda.empty_cache()


@pytest.mark.parametrize("spec", SPECS, ids=[s.name for s in SPECS])
def test_fullsize_selected_matches_oracle(spec):
    """The variant chosen by the learned selector, as bench.py runs it."""
    import os
    if not os.path.exists(S.DEFAULT_MODEL):
        pytest.skip("no trained model")
    S.spmv_model_load(S.DEFAULT_MODEL)
    rp, ci, v = spec.build()
    n = len(rp) - 1
    x = spec.x(n)
    plan = S.Plan(dev(rp), dev(ci), dev(v), n, nnz=len(ci))
    info = plan.select(S.SEL_MLP)
    y = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    plan.execute(dev(x), y)
    torch.cuda.synchronize()
    y_ref, scale = cref.dot2(rp, ci, v, x)
    check_whole_vector(y.cpu().numpy(), y_ref, scale, 1e-12, S.VARIANTS[info["variant"]])
    plan.close()


def test_fullsize_delta_codes():
    """The code-width report's wider band at its size (2M rows, 30..90
    nonzeros per row, half width 200; the sliced layout forced as the report
    does): features bit-exact for FP64 and FP32 plans; 8-bit delta codes,
    taken automatically, and 16-bit offsets on every row against the
    accuracy reference, equal to the sequential sum in FP64, and the two
    widths giving the same y in every dtype."""
    rp, ci, v = synth.banded(2_000_000, 960, 200, seed=9)
    n = len(rp) - 1
    x = synth.vector(n, 10)
    y_ref, scale = cref.dot2(rp, ci, v, x)
    y_seq = cref.seq(rp, ci, v, x)
    r_t, c_t = dev(rp), dev(ci)
    print(f"\nband_2000000_d60_w200: nnz={len(ci)} (every row compared)", flush=True)
    for dtype in (S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16):
        v_t = upload_values(v, dtype)
        x_t = dev(x) if dtype == S.SPMV_F64 else dev(x.astype(np.float32))
        tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
        plan = S.Plan(r_t, c_t, v_t, n, dtype, nnz=len(ci))
        if dtype != S.SPMV_BF16:
            check_features(plan, rp, ci, n, dtype, f"band/{DNAME[dtype]}")
        S.spmv_set_delta16_layout(plan.handle, 1)
        ys = {}
        for req in (0, 16):
            S.spmv_set_delta16_offset_bits(plan.handle, req)
            plan.set_variant(S.V_DELTA16)
            bits = plan.query(17)
            y = torch.full((n,), float("nan"), dtype=tdt, device=DEV)
            plan.execute(x_t, y)
            torch.cuda.synchronize()
            got = y.cpu().numpy().astype(np.float64)
            rel = check_whole_vector(got, y_ref, scale, TOL[dtype], (bits, DNAME[dtype]))
            print(f"  {DNAME[dtype]:>4s} {bits}-bit codes (escapes {plan.query(20)}) "
                  f"max |y - y_ref| / sum|a||x| = {rel:.3e}", flush=True)
            if dtype == S.SPMV_F64:
                assert np.array_equal(got, y_seq), bits
            ys[bits] = y
        assert sorted(ys) == [8, 16]
        assert torch.equal(ys[8], ys[16])
        plan.close()
        del v_t, x_t, ys
        torch.cuda.empty_cache()


@pytest.mark.parametrize("spec", SPECS, ids=[s.name for s in SPECS])
def test_fullsize_coded_forms(spec):
    """16-bit column codes inside merge-path tiles, x-block slice blocks and
    the rows-streamed layout, where they fit, at full size in FP64: every
    row equal to the same variant on int32 columns and within 1e-12 of the
    accuracy reference."""
    rp, ci, v = spec.build()
    n = len(rp) - 1
    x = spec.x(n)
    y_ref, scale = cref.dot2(rp, ci, v, x)
    plan = S.Plan(dev(rp), dev(ci), dev(v), n, nnz=len(ci))
    x_t = dev(x)
    S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
    mask = plan.mask()
    print(f"\n{spec.name}: coded mask {bin(mask)}", flush=True)
    for var in (S.V_MERGE_PATH, S.V_XBLOCK_LDS, S.V_SHORT_ROW):
        if not (mask >> var) & 1:
            continue
        ys = []
        for coding in (S.SPMV_IDX_CODED, S.SPMV_IDX_I32):
            S.spmv_set_index_coding(plan.handle, coding)
            plan.set_variant(var)
            y = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
            plan.execute(x_t, y)
            torch.cuda.synchronize()
            ys.append(y.cpu().numpy())
        assert np.array_equal(ys[0], ys[1]), S.VARIANTS[var]
        rel = check_whole_vector(ys[0], y_ref, scale, 1e-12, S.VARIANTS[var] + "/coded")
        print(f"  {S.VARIANTS[var]:>10s} coded = int32, max |y - y_ref| / sum|a||x| = {rel:.3e}", flush=True)
    plan.close()
