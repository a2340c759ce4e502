"""Derived formats and value rounding are byte-identical to the oracle (GPU)."""
import struct

import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.encode import (delta8_codes_ref, delta16_layout_ref, delta16_offset_bits_ref,
                           delta16_ref, delta16_sliced_auto_ref, delta16_sliced_ref,
                           merge_search_ref, merge_walk_ref, partition_ref, sliced_max_span_ref,
                           xblock_split_ref, to_bf16_bits_ref, to_f32_ref)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import dev, make_plan  # noqa: E402

MATS = [
    ("laplace64", lambda: synth.laplace2d(64), 4096),
    ("powerlaw", lambda: synth.powerlaw(30000, 109, 7000, seed=2), 30000),
    ("shortrows", lambda: synth.short_rows(20000, seed=3), 20000),
    ("banded", lambda: synth.banded(6000, 300, 200, seed=4), 6000),
    ("stencil27", lambda: synth.stencil3d_27(16), 4096),
    # rows of 30..65 nonzeros inside a 65-column band: 8-bit offsets
    ("narrowband", lambda: synth.banded(6000, 960, 32, seed=5), 6000),
]


@pytest.mark.parametrize("name,build,m", MATS)
def test_formats_match_oracle(name, build, m):
    rp, ci, v = build()
    n, nnz = len(rp) - 1, len(ci)
    plan = make_plan(rp, ci, v, m)
    h = plan.handle
    H16 = S.spmv_plan_query(h, 11)
    ok, base, off = delta16_ref(rp, ci, H16)
    if not ok and H16 != 256:
        pytest.fail("delta16 should have retried with 256-row blocks")
    assert S.spmv_plan_query(h, 9) == int(ok)
    if ok:
        L, srt = delta16_sliced_auto_ref(rp, ci, v)  # the row order the rule takes
        print(f"case={name} sorted={srt} slots={L['slots']}", flush=True)
        assert S.spmv_plan_query(h, 14) == delta16_layout_ref(True, L["slots"], nnz, n,
                                                              sliced_max_span_ref(L))
        assert S.spmv_plan_query(h, 15) == L["slots"]
        S.spmv_set_delta16_layout(h, 0)
        assert S.spmv_plan_query(h, 14) == 0
        assert S.spmv_plan_query(h, 26) == 0
        assert np.array_equal(S.spmv_plan_copy_format(h, 0, len(base)), base)
        assert np.array_equal(S.spmv_plan_copy_format(h, 1, nnz), off)
        S.spmv_set_delta16_layout(h, 1)
        bits = check_sliced(h, rp, ci, L, np.float64, srt=srt)
        assert S.spmv_bytes(h, S.V_DELTA16) == sliced_bytes(L, delta8_codes_ref(rp, ci, L), bits,
                                                            n, m, nnz, srt)
        for mode in (1 - int(srt), int(srt)):  # the other order forced, then this one
            S.spmv_set_delta16_sort(h, mode)
            Lm = delta16_sliced_ref(rp, ci, v, sort_rows=bool(mode))
            bits = check_sliced(h, rp, ci, Lm, np.float64, srt=bool(mode))
            assert S.spmv_bytes(h, S.V_DELTA16) == sliced_bytes(Lm, delta8_codes_ref(rp, ci, Lm),
                                                                bits, n, m, nnz, bool(mode))
        S.spmv_set_delta16_sort(h, -1)
        assert S.spmv_plan_query(h, 26) == int(srt)
    else:
        assert S.spmv_plan_query(h, 14) == -1
    T = S.spmv_plan_query(h, 3)
    tiles = S.spmv_plan_query(h, 4)
    si, sj = merge_search_ref(rp, T)
    assert len(si) == tiles + 1
    assert np.array_equal(S.spmv_plan_copy_format(h, 2, tiles + 1), si)
    assert np.array_equal(S.spmv_plan_copy_format(h, 3, tiles + 1), sj)
    if n + nnz < 200000:
        wi, wj = merge_walk_ref(rp, T)
        assert np.array_equal(wi, si) and np.array_equal(wj, sj)
    for forced in (0, 8, 2):
        S.spmv_set_xblock_slices(h, forced)
        nsl = S.spmv_plan_query(h, 7)
        assert forced == 0 or nsl == forced
        lr, rps, cx = xblock_split_ref(rp, ci, m, nsl)
        assert S.spmv_plan_query(h, 13) == len(lr)
        assert np.array_equal(S.spmv_plan_copy_format(h, 7, len(lr)), lr)
        assert np.array_equal(S.spmv_plan_copy_format(h, 4, nsl * (n + 1)), rps.reshape(-1))
        assert np.array_equal(S.spmv_plan_copy_format(h, 5, len(cx)), cx)
        tiles = sum((n + int(r[-1]) + T - 1) // T for r in rps)
        assert S.spmv_plan_query(h, 6) == tiles
    parts = S.spmv_plan_query(h, 8)
    assert np.array_equal(S.spmv_plan_copy_format(h, 6, parts + 1), partition_ref(rp, parts))
    plan.close()


def sliced_bytes(L, C, bits, n, m, nnz, srt=False):
    """Compulsory bytes: no codes in diagonal slices, their diagonals once;
    a column span per offset slice; 8-bit codes add their escaped columns
    and a first escape unit per offset slice; sorted rows a row index each."""
    ns = len(L["width"])
    n_off = ns - int(np.count_nonzero(L["kind"]))
    codes = L["nnz_offset"] * (1 if bits == 8 else 2) + (4 * C["escapes"] + 4 * n_off if bits == 8 else 0)
    return (4 * (n + 1) + 8 * nnz + codes + 8 * m + 8 * n + 16 * ns + 4 * n_off
            + 128 * int(np.count_nonzero(L["kind"])) + (4 * n if srt else 0))


def check_sliced(h, rp, ci, L, vdtype, bits=None, srt=False):
    """The plan's sliced arrays against the oracle; returns the code width."""
    ns = len(L["width"])
    assert S.spmv_plan_query(h, 26) == int(srt)
    if srt:
        assert np.array_equal(S.spmv_plan_copy_format(h, 22, len(L["perm"])), L["perm"])
    else:
        assert len(S.spmv_plan_copy_format(h, 22, 0)) == 0
    C = delta8_codes_ref(rp, ci, L)
    if bits is None:
        bits = delta16_offset_bits_ref(L["nnz_offset"], int(C["E"].sum()))
    assert S.spmv_plan_query(h, 17) == bits
    spans = L["span"][L["kind"] == 0]
    assert S.spmv_plan_query(h, 18) == (int(spans.max()) if len(spans) else 0)
    if bits == 8:
        assert S.spmv_plan_query(h, 19) == int(C["E"].sum())
        assert S.spmv_plan_query(h, 20) == C["escapes"]
        got = S.spmv_plan_copy_format(h, 11, len(C["codes"]))
        assert got.dtype == np.uint8 and np.array_equal(got, C["codes"])
        assert np.array_equal(S.spmv_plan_copy_format(h, 16, len(C["esc"])), C["esc"])
        assert np.array_equal(S.spmv_plan_copy_format(h, 17, ns), C["eunits"])
    else:
        assert S.spmv_plan_query(h, 19) == 0 and S.spmv_plan_query(h, 20) == 0
        assert np.all(L["off"] < 65536)
        got = S.spmv_plan_copy_format(h, 11, L["slots"])
        assert got.dtype == np.uint16 and np.array_equal(got, L["off"].astype(np.uint16))
        assert len(S.spmv_plan_copy_format(h, 17, 0)) == 0
    kinds = S.spmv_plan_copy_format(h, 13, ns)
    assert np.array_equal(kinds, np.where(L["kind"] > 0, 1 + L["ndiag"], 0))
    assert np.array_equal(S.spmv_plan_copy_format(h, 14, 32 * ns), L["diag"])
    assert np.array_equal(S.spmv_plan_copy_format(h, 15, len(L["mask"])), L["mask"])
    assert np.array_equal(S.spmv_plan_copy_format(h, 8, ns), L["width"])
    assert np.array_equal(S.spmv_plan_copy_format(h, 9, ns), L["units"])
    assert np.array_equal(S.spmv_plan_copy_format(h, 10, ns), L["base"])
    got = S.spmv_plan_copy_format(h, 12, L["slots"], vdtype)
    assert np.array_equal(got, L["vals"].astype(vdtype))
    return bits


@pytest.mark.parametrize("dtype", [S.SPMV_F32, S.SPMV_BF16])
def test_delta16_sliced_low_precision_values(dtype):
    """The sliced slots hold the plan's own FP32 / BF16 values."""
    rp, ci, v = synth.stencil3d_27(9, seed=2, values="random")
    plan = make_plan(rp, ci, v, 729, dtype)
    S.spmv_set_delta16_layout(plan.handle, 1)
    if dtype == S.SPMV_F32:
        q = to_f32_ref(v).astype(np.float64)
        L = delta16_sliced_ref(rp, ci, q)
        check_sliced(plan.handle, rp, ci, L, np.float32)
    else:
        bits = to_bf16_bits_ref(v)
        L = delta16_sliced_ref(rp, ci, bits.astype(np.float64))  # bit patterns as numbers
        L["vals"] = L["vals"].astype(np.uint16)
        check_sliced(plan.handle, rp, ci, L, np.uint16)
    plan.close()


def ragged_gaps(n=1024):
    """Rows of 40 columns 7 apart; in every slice row 5 jumps 300 columns once
    (one escape) and row 130 of every 256 twice."""
    rows = []
    for i in range(n):
        c = i + 7 * np.arange(40)
        if i % 64 == 5:
            c[20:] += 300
        if i % 256 == 130:
            c[10:] += 300
            c[30:] += 300
        rows.append(c)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    return rp, np.concatenate(rows).astype(np.int32)


@pytest.mark.parametrize("srt", [False, True])
@pytest.mark.parametrize("name", ["narrowband", "wideband", "random", "ragged_gaps"])
def test_delta16_code_widths(name, srt):
    """Automatic width, then 16 and 8 forced: codes, escapes and bytes as the
    oracle's.  The narrow and the wide band (half width 200, slices spanning
    about 460 columns) need no escape; on the random matrix every gap escapes
    and the rule keeps 16 bits; the last case mixes rows of small gaps with
    rows whose gaps escape.  Each with rows in order and sorted by length."""
    if name == "narrowband":
        rp, ci, v = synth.banded(6000, 960, 32, seed=5)
        m = 6000
    elif name == "wideband":
        rp, ci, v = synth.banded(6000, 300, 200, seed=4)
        m = 6000
    elif name == "random":
        rp, ci, v = synth.uniform_random(3000, 5000, 8, seed=4)
        m = 5000
    else:
        rp, ci = ragged_gaps()
        v = synth.random_values(len(ci), 6)
        m = 2000
    n, nnz = len(rp) - 1, len(ci)
    L = delta16_sliced_ref(rp, ci, v, sort_rows=srt)
    C = delta8_codes_ref(rp, ci, L)
    auto = delta16_offset_bits_ref(L["nnz_offset"], int(C["E"].sum()))
    print(f"case={name} sorted={srt} escapes={C['escapes']} E={int(C['E'].sum())} "
          f"automatic bits={auto}", flush=True)
    assert auto == (16 if name == "random" else 8)
    # sorted bands: a slice's rows come from a 256-row window, so a row can
    # start more than 254 columns above the slice's smallest column
    assert (C["escapes"] > 0) == (name in ("random", "ragged_gaps") or (srt and "band" in name))
    plan = make_plan(rp, ci, v, m)
    h = plan.handle
    S.spmv_set_delta16_layout(h, 1)
    S.spmv_set_delta16_sort(h, int(srt))
    for req in (0, 16, 8, 0):
        S.spmv_set_delta16_offset_bits(h, req)
        bits = check_sliced(h, rp, ci, L, np.float64, bits=req or auto, srt=srt)
        assert S.spmv_bytes(h, S.V_DELTA16) == sliced_bytes(L, C, bits, n, m, nnz, srt)
    with pytest.raises(S.SpmvError) as e:
        S.spmv_set_delta16_offset_bits(h, 4)
    assert e.value.status == S.SPMV_ERR_ARG
    with pytest.raises(S.SpmvError) as e:
        S.spmv_set_delta16_sort(h, 2)
    assert e.value.status == S.SPMV_ERR_ARG
    plan.close()


def test_delta16_layouts_and_row_orders_by_rule():
    """The stencil: sliced, diagonal slices, rows in order.  Rows of 2 to 6
    (mean 4): streamed.  Rows of 4 to 12 in half width 30 (1.5 slots per
    nonzero, mean 8): sliced, in order.  Rows of 10 to 30 in half width 400:
    sliced and sorted by length (the slices stage no x either way); forced
    in order, sliced with 1.5 slots per nonzero."""
    rp, ci, v = synth.stencil3d_27(16)
    plan = make_plan(rp, ci, v, 4096)
    assert S.spmv_plan_query(plan.handle, 14) == 1
    assert S.spmv_plan_query(plan.handle, 26) == 0  # diagonal slices are kept
    plan.close()
    rp, ci, v = synth.banded(6000, 64, 30, seed=4)
    plan = make_plan(rp, ci, v, 6000)
    L, srt = delta16_sliced_auto_ref(rp, ci, v)
    assert not srt and delta16_layout_ref(True, L["slots"], len(ci), 6000, sliced_max_span_ref(L)) == 0
    assert S.spmv_plan_query(plan.handle, 14) == 0
    assert S.spmv_plan_query(plan.handle, 26) == 0
    with pytest.raises(S.SpmvError) as e:
        S.spmv_plan_copy_format(plan.handle, 8, 1)
    assert e.value.status == S.SPMV_ERR_ARG
    with pytest.raises(S.SpmvError):
        S.spmv_set_delta16_layout(plan.handle, 2)
    plan.close()
    rp, ci, v = synth.banded(6000, 128, 30, seed=4)
    plan = make_plan(rp, ci, v, 6000)
    L, srt = delta16_sliced_auto_ref(rp, ci, v)
    assert not srt and delta16_layout_ref(True, L["slots"], len(ci), 6000, sliced_max_span_ref(L)) == 1
    assert S.spmv_plan_query(plan.handle, 14) == 1
    assert S.spmv_plan_query(plan.handle, 26) == 0
    assert S.spmv_plan_query(plan.handle, 15) == L["slots"]
    plan.close()
    rp, ci, v = synth.banded(6000, 320, 400, seed=4)
    plan = make_plan(rp, ci, v, 6000)
    L, srt = delta16_sliced_auto_ref(rp, ci, v)
    assert srt and delta16_layout_ref(True, L["slots"], len(ci), 6000, sliced_max_span_ref(L)) == 1
    assert S.spmv_plan_query(plan.handle, 14) == 1
    assert S.spmv_plan_query(plan.handle, 26) == 1
    assert S.spmv_plan_query(plan.handle, 15) == L["slots"]
    S.spmv_set_delta16_sort(plan.handle, 0)
    plain = delta16_sliced_ref(rp, ci, v)
    assert S.spmv_plan_query(plan.handle, 14) == delta16_layout_ref(True, plain["slots"], len(ci), 6000,
                                                                       sliced_max_span_ref(plain))
    assert S.spmv_plan_query(plan.handle, 26) == 0
    assert S.spmv_plan_query(plan.handle, 15) == plain["slots"]
    plan.close()


@pytest.mark.parametrize("d16,w", [(64, 30), (128, 30), (128, 400), (320, 400), (480, 20),
                                   (480, 200), (640, 2000)])
def test_delta16_rules_agree_with_oracle(d16, w):
    """The automatic layout and row order, and the slots and spans they give,
    equal the oracle's rules on bands of rows d/2 to 3d/2 long (d = d16/16)."""
    rp, ci, v = synth.banded(6000, d16, w, seed=7)
    plan = make_plan(rp, ci, v, 6000)
    h = plan.handle
    L, srt = delta16_sliced_auto_ref(rp, ci, v)
    layout = delta16_layout_ref(True, L["slots"], len(ci), 6000, sliced_max_span_ref(L))
    print(f"d16={d16} w={w} sorted={srt} layout={layout} slots/nnz={L['slots'] / len(ci):.3f}",
          flush=True)
    assert S.spmv_plan_query(h, 14) == layout
    assert S.spmv_plan_query(h, 26) == (int(srt) if layout == 1 else 0)
    S.spmv_set_delta16_layout(h, 1)  # the sliced arrays of the automatic row order
    assert S.spmv_plan_query(h, 26) == int(srt)
    assert S.spmv_plan_query(h, 15) == L["slots"]
    assert S.spmv_plan_query(h, 18) == sliced_max_span_ref(L)
    plan.close()


def test_delta16_infeasible_on_wide_rows():
    rp, ci, v = synth.uniform_random(3000, 2_000_000, 8, seed=2)
    plan = make_plan(rp, ci, v, 2_000_000)
    assert S.spmv_plan_query(plan.handle, 9) == 0
    assert not (plan.mask() >> S.V_DELTA16) & 1
    with pytest.raises(S.SpmvError) as e:
        plan.set_variant(S.V_DELTA16)
    assert e.value.status == S.SPMV_ERR_INFEASIBLE
    plan.close()


def rounding_cases():
    rng = np.random.default_rng(0)
    vals = [rng.uniform(-1, 1, 20000),
            rng.uniform(-1, 1, 4000) * 2.0 ** rng.integers(-140, 130, 4000)]
    ties = []
    for b in rng.integers(0x0100, 0x7F00, 2000):
        lo = struct.unpack("<f", struct.pack("<I", int(b) << 16))[0]
        hi = struct.unpack("<f", struct.pack("<I", (int(b) + 1) << 16))[0]
        mid = (lo + hi) / 2
        ties += [mid, np.nextafter(mid, 1e300), np.nextafter(mid, -1e300)]
    ties = np.array(ties)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, 1e300, -1e300, 3.4e38, 5e-324, 1e-45])
    return np.concatenate(vals + [ties, -ties, specials])


def test_quantize_bit_exact():
    v = rounding_cases()
    src = dev(v)
    out32 = torch.empty(len(v), dtype=torch.float32, device="cuda:0")
    out16 = torch.empty(len(v), dtype=torch.int16, device="cuda:0")
    S.spmv_quantize(src, out32, len(v), S.SPMV_F32)
    S.spmv_quantize(src, out16, len(v), S.SPMV_BF16)
    torch.cuda.synchronize()
    assert np.array_equal(out32.cpu().numpy().view(np.uint32), to_f32_ref(v).view(np.uint32))
    assert np.array_equal(out16.cpu().numpy().view(np.uint16), to_bf16_bits_ref(v))
