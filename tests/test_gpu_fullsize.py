"""Full-size parity: the four FP64 class matrices at the sizes bench.py times.

Inputs come from the seeded CPU generator (never from the library); every
feasible variant runs in the bench's launch configuration (the plan's own
parameters) and sampled rows are compared with the correctly rounded FP64
reference computed row by row, plus whole-vector properties (no NaN, exact
zeros on empty rows, determinism).  The precision path (FP32 / BF16 values,
FP32 x and accumulation) is checked the same way against the FP64 reference
of the original data, and the error table is printed.
"""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.encode import to_bf16_bits_ref, to_f32_ref
from oracle.spmv import spmv_exact, spmv_seq_rows

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import DEV, dev  # noqa: E402

TOL = {S.SPMV_F64: 1e-12, S.SPMV_F32: 1e-5, S.SPMV_BF16: 1e-2}
SEQ_ORDER = {S.V_CSR_SCALAR, S.V_SHORT_ROW, S.V_DELTA16}  # sum in column order
SPECS = synth.class_matrices(scale=1)


def sample_rows(rp, rng, k=1500):
    n = len(rp) - 1
    L = np.diff(rp)
    rows = set(rng.choice(n, size=min(k, n), replace=False).tolist())
    rows |= {0, n - 1, int(np.argmax(L))}
    return np.array(sorted(rows))


def upload_values(v, dtype):
    if dtype == S.SPMV_F64:
        return dev(v)
    if dtype == S.SPMV_F32:
        return dev(to_f32_ref(v))
    return dev(to_bf16_bits_ref(v).view(np.int16))


@pytest.mark.parametrize("spec", SPECS, ids=[s.name for s in SPECS])
def test_fullsize_variants(spec):
    rp, ci, v = spec.build()
    n = len(rp) - 1
    x = spec.x(n)
    rng = np.random.default_rng(0)
    rows = sample_rows(rp, rng)
    y_ref, scale = spmv_exact(rp, ci, v, x, rows)
    y_seq = spmv_seq_rows(rp, ci, v, x, rows)
    r_t, c_t = dev(rp), dev(ci)
    print(f"\n{spec.name}: n={n} nnz={len(ci)} sampled rows={len(rows)}", flush=True)
    for dtype in (S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16):
        v_t = upload_values(v, dtype)
        x_t = dev(x) if dtype == S.SPMV_F64 else dev(x.astype(np.float32))
        tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
        plan = S.Plan(r_t, c_t, v_t, n, dtype, nnz=len(ci))
        mask = plan.mask()
        runs = [(var, None) for var in range(6) if (mask >> var) & 1]
        if (mask >> S.V_DELTA16) & 1:  # the layout the rule did not pick, forced
            runs.append((S.V_DELTA16, 1 - plan.query(14)))
        for var, layout in runs:
            if layout is not None:
                S.spmv_set_delta16_layout(plan.handle, layout)
            plan.set_variant(var)
            y = torch.full((n,), float("nan"), dtype=tdt, device=DEV)
            plan.execute(x_t, y)
            y2 = torch.empty_like(y)
            plan.execute(x_t, y2)
            torch.cuda.synchronize()
            assert not torch.isnan(y).any().item(), S.VARIANTS[var]
            assert torch.equal(y, y2), f"{S.VARIANTS[var]} not deterministic"
            ys = y.cpu().numpy()[rows].astype(np.float64)
            err = np.abs(ys - y_ref)
            rel = float(np.max(np.where(scale > 0, err / np.where(scale > 0, scale, 1), 0)))
            name = S.VARIANTS[var] + ("" if layout is None else f"/layout{layout}")
            print(f"  dtype={['f64', 'f32', 'bf16'][dtype]:>4s} {name:>18s} "
                  f"max |y - y_ref| / sum|a||x| = {rel:.3e}", flush=True)
            assert np.all(err <= TOL[dtype] * scale), (name, dtype, rel)
            assert np.all(ys[scale == 0] == 0)
            if dtype == S.SPMV_F64 and var in SEQ_ORDER:
                assert np.array_equal(ys, y_seq), name
            del y, y2
        plan.close()
        del v_t, x_t
        torch.cuda.empty_cache()


@pytest.mark.parametrize("spec", SPECS, ids=[s.name for s in SPECS])
def test_fullsize_selected_matches_oracle(spec):
    """The variant chosen by the learned selector, as bench.py runs it."""
    if S.DEFAULT_MODEL and not __import__("os").path.exists(S.DEFAULT_MODEL):
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
    rows = sample_rows(rp, np.random.default_rng(1), 800)
    y_ref, scale = spmv_exact(rp, ci, v, x, rows)
    ys = y.cpu().numpy()[rows]
    assert np.all(np.abs(ys - y_ref) <= 1e-12 * scale), S.VARIANTS[info["variant"]]
    plan.close()


def test_fullsize_delta_codes():
    """The code-width report's wider band at its size (2M rows, 30..90
    nonzeros per row, half width 200; the sliced layout forced as the report
    does): 8-bit delta codes, taken automatically, and 16-bit offsets on
    sampled rows against the correctly rounded reference, equal to the
    sequential sum in FP64, and the two widths giving the same y in every
    dtype."""
    rp, ci, v = synth.banded(2_000_000, 960, 200, seed=9)
    n = len(rp) - 1
    x = synth.vector(n, 10)
    rows = sample_rows(rp, np.random.default_rng(2))
    y_ref, scale = spmv_exact(rp, ci, v, x, rows)
    y_seq = spmv_seq_rows(rp, ci, v, x, rows)
    r_t, c_t = dev(rp), dev(ci)
    print(f"\nband_2000000_d60_w200: nnz={len(ci)} sampled rows={len(rows)}", flush=True)
    for dtype in (S.SPMV_F64, S.SPMV_F32, S.SPMV_BF16):
        v_t = upload_values(v, dtype)
        x_t = dev(x) if dtype == S.SPMV_F64 else dev(x.astype(np.float32))
        tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
        plan = S.Plan(r_t, c_t, v_t, n, dtype, nnz=len(ci))
        S.spmv_set_delta16_layout(plan.handle, 1)
        ys = {}
        for req in (0, 16):
            S.spmv_set_delta16_offset_bits(plan.handle, req)
            plan.set_variant(S.V_DELTA16)
            bits = plan.query(17)
            y = torch.full((n,), float("nan"), dtype=tdt, device=DEV)
            plan.execute(x_t, y)
            torch.cuda.synchronize()
            assert not torch.isnan(y).any().item(), bits
            got = y.cpu().numpy()[rows].astype(np.float64)
            err = np.abs(got - y_ref)
            rel = float(np.max(np.where(scale > 0, err / np.where(scale > 0, scale, 1), 0)))
            print(f"  dtype={['f64', 'f32', 'bf16'][dtype]:>4s} {bits}-bit codes "
                  f"(escapes {plan.query(20)}) max |y - y_ref| / sum|a||x| = {rel:.3e}", flush=True)
            assert np.all(err <= TOL[dtype] * scale), (bits, dtype, rel)
            if dtype == S.SPMV_F64:
                assert np.array_equal(got, y_seq), bits
            ys[bits] = y
        assert sorted(ys) == [8, 16]
        assert torch.equal(ys[8], ys[16])
        plan.close()
        del v_t, x_t, ys
        torch.cuda.empty_cache()
