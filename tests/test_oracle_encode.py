"""Pins of the oracle encoders against definitions written out independently."""
import struct
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle.encode import (bf16_bits_to_f64, code_slot_ref, delta8_codes_ref, delta8_decode_ref,
                           delta16_sort_ref, delta16_sliced_auto_ref, sell_perm_ref,
                           sliced_stages_x_ref, staged_nnz_ref,
                           delta16_layout_ref, delta16_offset_bits_ref, delta16_ref,
                           delta16_sliced_ref, merge_search_ref, merge_walk_ref,
                           partition_ref, slice_csr_ref, to_bf16_bits_ref, to_f32_ref)
from oracle.spmv import spmv_seq


def cases(seed=3, count=40):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(0, 60))
        m = int(rng.integers(1, 70))
        yield synth.tiny_random_csr(rng, n, m, float(rng.choice([0, .02, .2, .7, 1.0])))


@pytest.mark.parametrize("H", [1, 3, 256])
def test_delta16_roundtrip_and_feasibility(H):
    for rp, ci, _ in cases():
        ok, base, off = delta16_ref(rp, ci, H)
        assert ok
        n = len(rp) - 1
        rows = np.repeat(np.arange(n), np.diff(rp))
        blk = rows // H
        assert np.array_equal(base[blk].astype(np.int64) + off, ci)
        for b in range(len(base)):
            seg = ci[rp[b * H]:rp[min(n, (b + 1) * H)]]
            assert base[b] == (seg.min() if len(seg) else 0)
    # a block spanning 65536 columns is infeasible, 65535 is feasible
    assert delta16_ref([0, 2], [0, 65535])[0]
    assert not delta16_ref([0, 2], [0, 65536])[0]
    assert delta16_ref([0, 1, 2], [0, 65536], 1)[0]
    assert not delta16_ref([0, 1, 2], [0, 65536], 2)[0]


def test_delta16_random_2m_infeasible_stencil_feasible():
    rp, ci, _ = synth.uniform_random(20000, 2_000_000, 8, seed=2)
    assert not delta16_ref(rp, ci)[0]
    rp, ci, _ = synth.stencil3d_27(30)
    assert delta16_ref(rp, ci)[0]


def test_delta16_sliced_laplacian_closed_form():
    """5-point Laplacian on a 64 x 64 grid: slice s is grid line s.

    Every slice is diagonal: lines 1..62 use the diagonals -64, -1, 0, 1, 64
    (width 6), line 0 lacks -64 and line 63 lacks 64 (width 4).  Rows at the
    ends of a line lack -1 or 1, so their masks miss that bit and its slot
    stays empty.
    """
    rp, ci, v = synth.laplace2d(64)
    L = delta16_sliced_ref(rp, ci, v)
    assert L["kind"].tolist() == [1] * 64
    assert L["width"].tolist() == [4] + [6] * 62 + [4]
    assert L["units"].tolist() == [0] + [2 + 3 * (s - 1) for s in range(1, 64)]
    assert L["slots"] == 64 * (4 + 6 * 62 + 4) == 24320
    assert len(ci) == 20224 and L["nnz_offset"] == 0
    assert delta16_layout_ref(True, L["slots"], len(ci), 4096) == 1  # 1.2025 slots per nonzero
    d = L["diag"].reshape(64, 32)
    assert d[0, :4].tolist() == [-1, 0, 1, 64] and d[63, :4].tolist() == [-64, -1, 0, 1]
    assert all(d[s_, :5].tolist() == [-64, -1, 0, 1, 64] for s_ in range(1, 63))
    assert not d[:, 5:].any() and not L["off"].any()
    m = L["mask"].reshape(64, 64)
    assert m[0].tolist() == [14] + [15] * 62 + [11]
    assert m[63].tolist() == [13] + [15] * 62 + [7]
    assert all(m[s_].tolist() == [29] + [31] * 62 + [23] for s_ in range(1, 63))
    for s_, j in ((1, 1), (17, 40), (62, 62), (5, 0), (9, 63)):
        present = [k for k in range(5) if (m[s_, j] >> k) & 1]
        for k in range(6):
            slot = 128 * (2 + 3 * (s_ - 1)) + 128 * (k // 2) + 2 * j + k % 2
            want = (4.0 if k == 2 else -1.0) if k in present else 0.0
            assert L["vals"][slot] == want, (s_, j, k)


def test_delta16_sliced_layout_rule():
    def csr(lens):
        lens = np.asarray(lens)
        rp = np.concatenate([[0], np.cumsum(lens)])
        ci = np.concatenate([np.arange(i, i + lens[i]) for i in range(len(lens))])
        return rp, ci, delta16_sliced_ref(rp, ci, np.ones(len(ci)))
    # rows of 1 and 2 nonzeros: width 2, 128 slots per 96 nonzeros -> sliced
    rp, ci, L = csr([1 + (i % 2) for i in range(128)])
    assert L["slots"] == 256 and len(ci) == 192
    assert delta16_layout_ref(True, L["slots"], len(ci), 128) == 1
    # rows of 1 and 3: width 4, 256 slots per 128 nonzeros -> streamed
    rp, ci, L = csr([1 + 2 * (i % 2) for i in range(64)])
    assert L["slots"] == 256 and len(ci) == 128
    assert delta16_layout_ref(True, L["slots"], len(ci), 64) == 0
    assert delta16_layout_ref(False, 0, 0, 0) == -1
    # one row of 30 among rows of 20: 1920 slots per 1290 nonzeros (1.49),
    # and one row of 14 among rows of 10: 896 per 644 (1.39), sliced because
    # rows average at least 8 nonzeros; one row of 7 among rows of 5: 512 per
    # 322 (1.59), streamed because they average 5; one row of 14 among rows
    # of 8: 896 per 518 (1.73), streamed
    rp, ci, L = csr([30] + [20] * 63)
    assert L["slots"] == 1920 and len(ci) == 1290
    assert delta16_layout_ref(True, L["slots"], len(ci), 64) == 1
    rp, ci, L = csr([14] + [10] * 63)
    assert L["slots"] == 896 and len(ci) == 644
    assert delta16_layout_ref(True, L["slots"], len(ci), 64) == 1
    rp, ci, L = csr([7] + [5] * 63)
    assert L["slots"] == 512 and len(ci) == 322
    assert delta16_layout_ref(True, L["slots"], len(ci), 64) == 0
    rp, ci, L = csr([14] + [8] * 63)
    assert L["slots"] == 896 and len(ci) == 518
    assert delta16_layout_ref(True, L["slots"], len(ci), 64) == 0
    # the 1.6 bound: a mean of 7.5 or more, and offset slices spanning
    # fewer than 8192 columns
    assert delta16_layout_ref(True, 150, 100, 13) == 1                 # mean 7.69
    assert delta16_layout_ref(True, 150, 100, 14) == 0                 # mean 7.14
    assert delta16_layout_ref(True, 160, 100, 13) == 1 and delta16_layout_ref(True, 161, 100, 13) == 0
    assert delta16_layout_ref(True, 150, 100, 13, 8191) == 1
    assert delta16_layout_ref(True, 150, 100, 13, 8192) == 0
    assert delta16_layout_ref(True, 135, 100, 50, 100000) == 1         # 1.35 holds at any span
    # equal odd rows of 27: 28 slots per 27 nonzeros -> sliced
    rp = np.arange(0, 27 * 128 + 1, 27)
    ci = np.concatenate([np.arange(27) + i for i in range(128)])
    L = delta16_sliced_ref(rp, ci, np.ones(len(ci)))
    assert L["width"].tolist() == [28, 28] and L["slots"] == 64 * 56
    assert delta16_layout_ref(True, L["slots"], len(ci), 128) == 1
    # 70 such rows: the second slice pads 58 empty lanes -> 1.9 slots per
    # nonzero, streamed
    L = delta16_sliced_ref(rp[:71], ci[:27 * 70], np.ones(27 * 70))
    assert L["slots"] == 64 * 56
    assert delta16_layout_ref(True, L["slots"], 27 * 70, 70) == 0


def dense_band(n, w):
    """Row i holds every column of [i - w, i + w] inside [0, n)."""
    cols = [np.arange(max(0, i - w), min(n, i + w + 1)) for i in range(n)]
    rp = np.concatenate([[0], np.cumsum([len(c) for c in cols])])
    return rp, np.concatenate(cols)


@pytest.mark.parametrize("w", [20, 96, 200, 1000])
def test_delta8_dense_band(w):
    """A dense band of half-width w has 2w + 1 > 32 diagonals, so every slice
    stores codes.  Row r holds columns max(0, r - w) .. min(n - 1, r + w):
    consecutive columns differ by 1, and the first lies max(0, r - w) -
    max(0, 64 s - w) <= 63 past the slice's reference column, so no code
    escapes, whatever the band's width, and the matrix takes 8 bits."""
    n = 640
    rp, ci = dense_band(n, w)
    L = delta16_sliced_ref(rp, ci, np.ones(len(ci)))
    ns = n // 64
    assert L["kind"].tolist() == [0] * ns
    span = [min(n - 1, 64 * s + 63 + w) - max(0, 64 * s - w) for s in range(ns)]
    assert L["span"].tolist() == span
    C = delta8_codes_ref(rp, ci, L)
    assert C["E"].tolist() == [0] * ns and C["escapes"] == 0 and len(C["esc"]) == 0
    assert delta16_offset_bits_ref(L["nnz_offset"], int(C["E"].sum())) == 8
    for r in range(n):
        s, lane = divmod(r, 64)
        length = rp[r + 1] - rp[r]
        for k in range(length):
            slot = 128 * (L["units"][s] + s) + 256 * (k // 4) + 4 * lane + k % 4
            want = max(0, r - w) - max(0, 64 * s - w) if k == 0 else 1
            assert C["codes"][slot] == want, (r, k)
    # every byte is a code or padding: the nonzero codes are exactly the
    # nonzeros' (each at least 1 after a row's first)
    assert len(C["codes"]) == L["slots"] + 128 * ns


def test_delta8_escape_closed_form():
    """Row l of a 64-row matrix holds columns 3 l and 3 l + 254 + (l mod 2):
    128 diagonals, one offset slice with reference column 0.  Codes: 3 l, then
    254 (even l) or the escape (odd l, a gap of 255), whose column goes to
    esc[l]; E = 1, 32 escapes.  8 bits would need 256 escape bytes for 128
    codes, so the matrix keeps 16 bits."""
    rp = np.arange(0, 129, 2)
    ci = np.array([c for l in range(64) for c in (3 * l, 3 * l + 254 + l % 2)])
    L = delta16_sliced_ref(rp, ci, np.ones(128))
    assert L["kind"].tolist() == [0] and L["width"].tolist() == [2] and L["base"].tolist() == [0]
    C = delta8_codes_ref(rp, ci, L)
    assert len(C["codes"]) == 256  # width 2 plus the spare unit: one group of four
    assert C["codes"][0:256:4].tolist() == [3 * l for l in range(64)]
    assert C["codes"][1:256:4].tolist() == [254 + l % 2 for l in range(64)]
    assert not C["codes"][2:256:4].any() and not C["codes"][3:256:4].any()
    assert code_slot_ref(0, 0, 5, 1) == 21 and code_slot_ref(3, 2, 0, 6) == 128 * 5 + 256 + 2
    assert C["E"].tolist() == [1] and C["eunits"].tolist() == [0] and C["escapes"] == 32
    assert C["esc"].tolist() == [3 * l + 255 if l % 2 else 0 for l in range(64)]
    assert delta16_offset_bits_ref(L["nnz_offset"], 1) == 16


def test_delta8_decode_round_trip():
    """Decoding the codes gives back every offset-slice row's columns."""
    mats = [c for c in cases(seed=13)]
    mats += [synth.banded(700, 48, 300, seed=3), synth.uniform_random(200, 70000, 9, seed=4),
             synth.powerlaw(900, 109, 400, seed=5)]
    for rp, ci, v in mats:
        rp, ci = np.asarray(rp), np.asarray(ci)
        L = delta16_sliced_ref(rp, ci, np.ones(len(ci)))
        C = delta8_codes_ref(rp, ci, L)
        L = dict(L, eunits=C["eunits"])
        rows = delta8_decode_ref(C["codes"], C["esc"], L, np.diff(rp))
        for i in range(len(rp) - 1):
            if not L["kind"][i // 64]:
                assert rows[i] == ci[rp[i]:rp[i + 1]].tolist(), i
        n_esc = sum(1 for i in range(len(rp) - 1) if not L["kind"][i // 64]
                    for j in range(rp[i], rp[i + 1])
                    if ci[j] - (ci[j - 1] if j > rp[i] else L["base"][i // 64]) >= 255)
        assert C["escapes"] == n_esc


def test_delta16_offset_bits_rule():
    assert delta16_offset_bits_ref(0, 0) == 16          # nothing to store
    assert delta16_offset_bits_ref(100, 0) == 8
    assert delta16_offset_bits_ref(512, 1) == 8          # 256 escape bytes = half the saving
    assert delta16_offset_bits_ref(511, 1) == 16
    # a tridiagonal matrix has only diagonal slices: 16 bits
    rp, ci = dense_band(200, 1)
    L = delta16_sliced_ref(rp, ci, np.ones(len(ci)))
    assert L["nnz_offset"] == 0 and delta16_offset_bits_ref(0, 0) == 16


def test_delta16_sliced_places_every_nonzero_once():
    kinds = set()
    for rp, ci, v in list(cases(seed=11)) + [synth.stencil3d_27(5, seed=2, values="random"),
                                             synth.banded(300, 48, 3, seed=3)]:
        rp, ci, v = np.asarray(rp), np.asarray(ci), np.asarray(v)
        n = len(rp) - 1
        L = delta16_sliced_ref(rp, ci, v)
        seen = np.zeros(L["slots"], dtype=bool)
        for s_ in range(len(L["width"])):
            r0, r1 = 64 * s_, min(n, 64 * s_ + 64)
            rel = sorted({int(ci[j]) - i for i in range(r0, r1) for j in range(rp[i], rp[i + 1])})
            longest = max([rp[i + 1] - rp[i] for i in range(r0, r1)], default=0)
            diag = len(rel) <= 32 and len(rel) + len(rel) % 2 <= longest + longest % 2
            assert L["kind"][s_] == int(diag)
            kinds.add(int(diag))
            for i in range(r0, r1):
                lane = i - r0
                for k_row in range(rp[i + 1] - rp[i]):
                    j = rp[i] + k_row
                    k = rel.index(int(ci[j]) - i) if diag else k_row
                    assert k < L["width"][s_]
                    slot = 128 * L["units"][s_] + 128 * (k // 2) + 2 * lane + k % 2
                    assert not seen[slot]
                    seen[slot] = True
                    assert L["vals"][slot] == v[j]
                    if diag:
                        assert L["diag"][32 * s_ + k] == ci[j] - i and (L["mask"][i] >> k) & 1
                    else:
                        assert L["base"][s_] + L["off"][slot] == ci[j]
                if diag:
                    assert bin(int(L["mask"][i])).count("1") == rp[i + 1] - rp[i]
                else:
                    assert L["mask"][i] == 0
        assert not np.any(L["vals"][~seen]) and not np.any(L["off"][~seen])
    assert kinds == {0, 1}


def test_delta16_sliced_spmv_in_lane_order_is_sequential():
    """Summing each lane's positions in order from +0 (adding nothing for an
    empty position) is Algorithm 1's sum, in both kinds of slice."""
    rng = np.random.default_rng(5)
    mats = []
    for n in (1, 63, 64, 65, 200):
        lens = rng.integers(0, 40, n)
        lens[rng.integers(0, n)] = 0
        rp = np.concatenate([[0], np.cumsum(lens)])
        ci = np.concatenate([np.sort(rng.choice(300, l, replace=False)) for l in lens]).astype(np.int64)
        mats.append((rp, ci, rng.uniform(-1, 1, len(ci)), 300))
    rp, ci, v = synth.stencil3d_27(6, seed=4, values="random")
    mats.append((np.asarray(rp), np.asarray(ci), np.asarray(v), 216))
    for rp, ci, v, m in mats:
        n = len(rp) - 1
        x = rng.uniform(-1, 1, m)
        L = delta16_sliced_ref(rp, ci, v)
        y = np.zeros(n)
        for i in range(n):
            s_, lane = divmod(i, 64)
            acc = 0.0
            for k in range(L["width"][s_]):
                slot = 128 * L["units"][s_] + 128 * (k // 2) + 2 * lane + k % 2
                if L["kind"][s_]:
                    if (L["mask"][i] >> k) & 1:
                        acc = acc + L["vals"][slot] * x[i + L["diag"][32 * s_ + k]]
                elif k < rp[i + 1] - rp[i]:
                    acc = acc + L["vals"][slot] * x[L["base"][s_] + L["off"][slot]]
            y[i] = acc
        assert np.array_equal(y, spmv_seq(rp, ci, v, x))


@pytest.mark.parametrize("T", [1, 3, 7, 64, 2048])
def test_merge_search_equals_walk(T):
    for rp, ci, _ in cases(seed=T):
        a = merge_walk_ref(rp, T)
        b = merge_search_ref(rp, T)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_merge_split_properties():
    rp, _, _ = synth.powerlaw(2000, 109, 500, seed=1)
    T = 97
    si, sj = merge_search_ref(rp, T)
    n, nnz = len(rp) - 1, int(rp[-1])
    assert si[0] == 0 and sj[0] == 0 and si[-1] == n and sj[-1] == nnz
    for t in range(len(si)):
        d = min(t * T, n + nnz)
        i, j = int(si[t]), int(sj[t])
        assert i + j == d
        # every consumed nonzero belongs to a row < i or to row i itself
        assert j <= (rp[i + 1] if i < n else nnz)
        # every consumed row end lies at or before the nonzero cursor
        assert i == 0 or rp[i] <= j


def test_partition_equal_nnz():
    rp, _, _ = synth.powerlaw(5000, 109, 2000, seed=2)
    b = partition_ref(rp, 64)
    nnz = int(rp[-1])
    assert b[0] == 0 and b[-1] == 5000 and np.all(np.diff(b) >= 0)
    for p in range(1, 64):
        tgt = -((-p * nnz) // 64)
        assert rp[b[p]] >= tgt and (b[p] == 0 or rp[b[p] - 1] < tgt)


@pytest.mark.parametrize("S", [1, 3, 8])
def test_slice_csr_reassembles_matrix(S):
    for rp, ci, _ in cases(seed=5):
        m = int(ci.max()) + 1 if len(ci) else 1
        rps, cx = slice_csr_ref(rp, ci, m, S)
        n = len(rp) - 1
        width = (m + S - 1) // S
        off = np.concatenate([[0], np.cumsum(rps[:, -1])])
        assert off[-1] == len(ci)
        for i in range(n):
            parts = [cx[off[s] + rps[s, i]:off[s] + rps[s, i + 1]] for s in range(S)]
            for s, p in enumerate(parts):
                assert np.all(p // width == s)
            assert np.array_equal(np.concatenate(parts), ci[rp[i]:rp[i + 1]])


def bf16_by_fraction(x):
    """Round x to the nearest bfloat16 (ties to even) by scanning neighbours."""
    f32 = np.float32(x)
    # candidates: bf16 values around the float32 rounding of x
    b = struct.unpack("<I", struct.pack("<f", float(f32)))[0] >> 16
    best = None
    for c in range(max(0, b - 2), min(0xFFFF, b + 3)):
        v = struct.unpack("<f", struct.pack("<I", c << 16))[0]
        if v != v or abs(v) == float("inf"):
            continue
        if (v < 0) != (x < 0) and v != 0:
            continue
        d = abs(Fraction(v) - Fraction(x))
        key = (d, c & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


def test_bf16_round_to_nearest_even():
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.uniform(-1, 1, 3000),
                           rng.uniform(-1, 1, 500) * 2.0 ** rng.integers(-120, 120, 500)])
    # exact ties: bf16 value plus half an ulp, and a tie broken by a far bit
    ties = []
    for b in rng.integers(0x3C00, 0x4300, 200):
        lo = struct.unpack("<f", struct.pack("<I", int(b) << 16))[0]
        hi = struct.unpack("<f", struct.pack("<I", (int(b) + 1) << 16))[0]
        mid = (lo + hi) / 2
        ties += [mid, np.nextafter(mid, 10.0), np.nextafter(mid, -10.0)]
    vals = np.concatenate([vals, ties, -np.array(ties)])
    got = to_bf16_bits_ref(vals)
    for v, g in zip(vals, got):
        assert g == bf16_by_fraction(float(v)), v


def test_bf16_special_values():
    vals = np.array([0.0, -0.0, 1.0, -2.0, 3.0 * 2 ** 130, 2.0 ** -130, 2.0 ** -140, np.inf, -np.inf])
    got = to_bf16_bits_ref(vals)
    assert list(got[:4]) == [0x0000, 0x8000, 0x3F80, 0xC000]
    assert got[4] == 0x7F80                   # overflow -> +inf
    assert got[5] == 0x0008                   # 2^-130 = 8 units of 2^-133 (subnormal)
    assert got[6] == 0x0000                   # 2^-140 rounds to zero
    assert got[7] == 0x7F80 and got[8] == 0xFF80
    back = bf16_bits_to_f64(got[:4])
    assert list(back) == [0.0, -0.0, 1.0, -2.0]


def test_integers_exact_in_bf16_and_f32():
    v = np.arange(-256, 257, dtype=np.float64)
    assert np.array_equal(bf16_bits_to_f64(to_bf16_bits_ref(v)), v)
    assert np.array_equal(to_f32_ref(v).astype(np.float64), v)


def test_f32_rounding_matches_fractions():
    rng = np.random.default_rng(1)
    for x in rng.uniform(-1, 1, 500):
        f = float(to_f32_ref([x])[0])
        up = float(np.nextafter(np.float32(f), np.float32(2)))
        dn = float(np.nextafter(np.float32(f), np.float32(-2)))
        d = abs(Fraction(f) - Fraction(x))
        assert d <= abs(Fraction(up) - Fraction(x)) and d <= abs(Fraction(dn) - Fraction(x))


def test_xblock_split_takes_long_rows_out():
    from oracle.encode import slice_csr_ref, xblock_split_ref
    rng = np.random.default_rng(11)
    n, m = 400, 8000
    rows = []
    for i in range(n):
        if i in (17, 230):   # long: 700 columns inside slice 0 (width 2000)
            rows.append(np.sort(rng.choice(2000, 700, replace=False)))
        else:
            rows.append(np.sort(rng.choice(m, rng.integers(0, 30), replace=False)))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows)
    lr, rps, cols = xblock_split_ref(rp, ci, m, 4)
    assert lr.tolist() == [17, 230]
    for s in range(4):
        seg = np.diff(rps[s])
        assert seg[17] == 0 and seg[230] == 0 and seg.max() <= 128
    # short rows keep their slice segments unchanged
    full, _ = slice_csr_ref(rp, ci, m, 4)
    keep = np.setdiff1d(np.arange(n), lr)
    assert np.array_equal(np.diff(rps, axis=1)[:, keep], np.diff(full, axis=1)[:, keep])
    assert len(cols) + 1400 == len(ci)
    # brute force of the long-row rule
    width = 2000
    brute = [i for i in range(n) if max(np.bincount(rows[i] // width, minlength=4), default=0) > 128]
    assert brute == lr.tolist()
    # long rows above a quarter of the nonzeros: nothing is split
    lr2, rps2, _ = xblock_split_ref(rp, ci, m, 4, max_share=0.1)
    assert len(lr2) == 0 and np.array_equal(rps2, full)


# ---------------------------------------------------------------- 16-bit codes
# inside merge-path tiles and x-block slice blocks (the index-coding axis)
from oracle.encode import (merge_codes_ref, merge_walk_ref, range_codes_ref,  # noqa: E402
                           slice_csr_ref, xblock_codes_ref, xblock_split_ref)


def test_range_codes_definition_by_hand():
    """Hand-counted case: three ranges, one empty."""
    ci = np.array([7, 9, 12, 3, 100, 40], np.int32)
    ok, base, off, span = range_codes_ref(ci, [0, 3, 3, 6])
    assert ok and span == 97
    assert base.tolist() == [7, 0, 3]
    assert off.tolist() == [0, 2, 5, 0, 97, 37]
    ok, _, _, span = range_codes_ref(np.array([0, 65536], np.int32), [0, 2])
    assert not ok and span == 65536
    ok, _, _, span = range_codes_ref(np.array([5, 65540], np.int32), [0, 2])
    assert ok and span == 65535            # the widest span that fits 16 bits


def test_merge_codes_tridiagonal_closed_form():
    """Tridiagonal N = 3000 (row 0 has 2 nonzeros, row i >= 1 starts at
    nonzero 3 i - 1): 2048 items = 512 row ends + 1536 nonzeros, so tile t
    (t < 5) starts on row 512 t at nonzero 1536 t, that row's second nonzero,
    column 512 t, which is the tile's smallest column; its last nonzero is
    the first of row 512 (t + 1), column 512 (t + 1) - 1.  Every span is
    below 513 and the codes decode back to the columns."""
    n = 3000
    rows = [[j for j in (i - 1, i, i + 1) if 0 <= j < n] for i in range(n)]
    rp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    ci = np.concatenate([np.array(r) for r in rows]).astype(np.int32)
    ok, base, off, span = merge_codes_ref(rp, ci)
    si, sj = merge_walk_ref(rp, 2048)
    assert ok and len(base) == len(si) - 1
    assert si[:5].tolist() == [0, 512, 1024, 1536, 2048]
    assert sj[:5].tolist() == [0, 1536, 3072, 4608, 6144]
    assert base[:5].tolist() == [0, 512, 1024, 1536, 2048]
    assert span <= 512
    for t in range(len(base)):
        seg = ci[sj[t]:sj[t + 1]]
        assert np.array_equal(base[t] + off[sj[t]:sj[t + 1]].astype(np.int64), seg)
        if len(seg):
            assert off[sj[t]:sj[t + 1]].min() == 0     # the reference is attained


def test_merge_codes_wide_rows_infeasible():
    """A tile holding columns 0 and M - 1 with M > 65536 cannot be coded."""
    rp, ci, _ = synth.uniform_random(3000, 200000, 6, seed=4)
    ok, _, _, span = merge_codes_ref(rp, ci)
    assert not ok and span > 65535


@pytest.mark.parametrize("S,H", [(1, 256), (2, 256), (4, 512), (8, 256)])
def test_xblock_codes_round_trip(S, H):
    """Every slice-major column decodes from its block's reference; blocks
    are the rows [b H, (b+1) H) of each slice, in slice-major order."""
    rp, ci, _ = synth.banded(4000, 200, 400, seed=6)
    n = len(rp) - 1
    ok, base, off, span = xblock_codes_ref(rp, ci, n, S, H)
    long_rows, rps, cols = xblock_split_ref(rp, ci, n, S)
    assert ok
    nb = (n + H - 1) // H
    assert len(base) == S * nb
    start = 0
    for s in range(S):
        for b in range(nb):
            a = start + int(rps[s][b * H]) if b * H <= n else start
            e = start + int(rps[s][min((b + 1) * H, n)])
            seg = cols[a:e]
            got = base[s * nb + b] + off[a:e].astype(np.int64)
            assert np.array_equal(got, seg)
            if len(seg):
                assert seg.min() == base[s * nb + b]
        start += int(rps[s][n])
    assert start == len(cols)


def test_xblock_codes_span_bound():
    """Columns of a slice lie in a slice of ceil(M / S) columns, so a slice
    narrower than 65536 columns always codes, whatever the rows."""
    rp, ci, _ = synth.uniform_random(2000, 120000, 8, seed=7)
    ok2, _, _, span2 = xblock_codes_ref(rp, ci, 120000, 2, 256)   # slices of 60000 columns
    assert ok2 and span2 < 60000
    ok1, _, _, span1 = xblock_codes_ref(rp, ci, 120000, 1, 256)   # one slice of 120000
    assert not ok1 and span1 > 65535


# ------------------------------------------------ the length-sorted sliced layout
def test_sell_perm_by_hand():
    """Longest first inside each window, ties in row order."""
    rp = np.array([0, 1, 4, 6, 9])                      # lengths 1, 3, 2, 3
    assert sell_perm_ref(rp, 4).tolist() == [1, 3, 2, 0]
    assert sell_perm_ref(rp, 2).tolist() == [1, 0, 3, 2]
    lens = np.arange(600) % 7                            # windows of 256 rows, then a partial one
    rp = np.concatenate([[0], np.cumsum(lens)])
    perm = sell_perm_ref(rp)
    for w0 in (0, 256, 512):
        rows = perm[w0:w0 + 256]
        assert sorted(rows.tolist()) == list(range(w0, min(600, w0 + 256)))
        key = [(-lens[i], i) for i in rows]
        assert key == sorted(key)


def _slots_for(rp, perm):
    lens = np.diff(np.asarray(rp))[perm]
    w = [int(lens[k:k + 64].max()) for k in range(0, len(lens), 64)]
    return 64 * sum(x + x % 2 for x in w)


def test_sorted_rows_minimise_padding():
    """Sorting each window's rows by length gives the fewest slots of any
    order of the rows inside their windows (the sum of the 64-row maxima of
    a sorted sequence is minimal), and the layout's slot count is that sum."""
    rng = np.random.default_rng(21)
    for n in (64, 300, 700):
        lens = rng.integers(0, 50, n)
        rp = np.concatenate([[0], np.cumsum(lens)])
        ci = np.concatenate([np.sort(rng.choice(400, l, replace=False)) for l in lens]).astype(np.int64)
        L = delta16_sliced_ref(rp, ci, np.ones(len(ci)), sort_rows=True)
        assert L["slots"] == _slots_for(rp, L["perm"])
        assert not np.any(L["kind"])
        for _ in range(30):
            other = np.concatenate([rng.permutation(np.arange(w0, min(n, w0 + 256)))
                                    for w0 in range(0, n, 256)])
            assert L["slots"] <= _slots_for(rp, other)


def test_sorted_layout_places_every_nonzero_once_and_sums_in_order():
    """Every nonzero of the row at each position sits once at its slot with
    its offset; summing a lane's positions in order is Algorithm 1's sum of
    the row it holds; 8-bit codes decode back to every row."""
    rng = np.random.default_rng(22)
    mats = [synth.banded(700, 960, 32, seed=3), synth.short_rows(900, seed=4),
            synth.powerlaw(800, 109, 300, seed=5), synth.uniform_random(300, 70000, 9, seed=6)]
    for rp, ci, v in mats:
        rp, ci, v = np.asarray(rp), np.asarray(ci), np.asarray(v)
        n = len(rp) - 1
        L = delta16_sliced_ref(rp, ci, v, sort_rows=True)
        perm = L["perm"]
        assert sorted(perm.tolist()) == list(range(n))
        seen = np.zeros(L["slots"], dtype=bool)
        x = rng.uniform(-1, 1, int(ci.max()) + 1)
        y = np.zeros(n)
        for p in range(n):
            i, (s_, lane) = int(perm[p]), divmod(p, 64)
            acc = 0.0
            for k in range(rp[i + 1] - rp[i]):
                slot = 128 * L["units"][s_] + 128 * (k // 2) + 2 * lane + k % 2
                assert not seen[slot]
                seen[slot] = True
                assert L["vals"][slot] == v[rp[i] + k]
                assert L["base"][s_] + L["off"][slot] == ci[rp[i] + k]
                acc = acc + L["vals"][slot] * x[L["base"][s_] + L["off"][slot]]
            y[i] = acc
        assert not np.any(L["vals"][~seen]) and not np.any(L["off"][~seen])
        assert np.array_equal(y, spmv_seq(rp, ci, v, x))
        C = delta8_codes_ref(rp, ci, L)
        rows = delta8_decode_ref(C["codes"], C["esc"], dict(L, eunits=C["eunits"]), np.diff(rp))
        assert all(rows[i] == ci[rp[i]:rp[i + 1]].tolist() for i in range(n))


def test_delta16_sort_rule():
    n, nnz, ns = 1000, 20000, 16
    assert not delta16_sort_ref(21000, 20000, 0, ns, nnz, n)      # padding 5%: not worth it
    assert delta16_sort_ref(30000, 22000, 0, ns, nnz, n)          # saves 27% and 8 slots per row
    assert not delta16_sort_ref(30000, 28600, 0, ns, nnz, n)      # saves under 5%
    assert not delta16_sort_ref(30000, 22000, 1, ns, nnz, n)      # a diagonal slice in 16
    assert not delta16_sort_ref(3000, 1900, 0, ns, 1500, n)       # 1.1 slots per row saved (short rows)
    assert not delta16_sort_ref(30000, 22100, 0, ns, nnz, n)      # 7.9 slots per row saved
    assert delta16_sort_ref(30000, 22000, 0, ns, nnz, n, 20000, 10000, 20000)     # 8, half the staging kept
    assert not delta16_sort_ref(30000, 22000, 0, ns, nnz, n, 20000, 9999, 20000)  # staging lost
    assert delta16_sort_ref(30000, 26000, 0, ns, nnz, n, 9999, 0, 20000)      # 4 per row, little staged
    assert not delta16_sort_ref(30000, 26100, 0, ns, nnz, n, 9999, 0, 20000)  # 3.9 per row
    assert not delta16_sort_ref(30000, 26000, 0, ns, nnz, n, 10000, 0, 20000)  # half staged, lost


def test_x_staging_rule_by_hand():
    """A slice stages x when its span is under 512 columns and its 64 w
    gathers are at least twice the span + 1 entries it loads."""
    assert sliced_stages_x_ref(0, 2) and sliced_stages_x_ref(63, 2)
    assert not sliced_stages_x_ref(64, 2)                  # 130 entries > 128 gathers
    assert sliced_stages_x_ref(511, 16) and not sliced_stages_x_ref(512, 64)
    # one offset slice of two 40-wide rows spanning 100 columns, one of two
    # rows spanning 3000 (both with 64-row slices padded by empty rows)
    lens = np.zeros(128, np.int64)
    lens[[0, 1, 64, 65]] = 40
    ci = np.concatenate([np.arange(0, 100, 100 / 40).astype(np.int64)[:40] for _ in range(2)] +
                        [np.linspace(0, 3000, 40).astype(np.int64) for _ in range(2)])
    rp = np.concatenate([[0], np.cumsum(lens)])
    L = delta16_sliced_ref(rp, ci, np.ones(len(ci)))
    assert list(L["kind"]) == [0, 0] and list(L["span"]) == [97, 3000]
    assert staged_nnz_ref(rp, L) == 80


def test_automatic_row_order():
    """The automatic order keeps diagonal slices and evenly long rows plain
    and sorts rows of mixed lengths when that saves enough slots per row and
    keeps the x staging."""
    rp, ci, v = synth.stencil3d_27(8)
    L, sorted_ = delta16_sliced_auto_ref(rp, ci, v)
    assert not sorted_ and np.any(L["kind"]) and np.all(L["perm"] == np.arange(len(rp) - 1))
    rng = np.random.default_rng(23)
    lens = rng.choice([2, 40], 1024)                     # lengths mixed inside every slice
    rp = np.concatenate([[0], np.cumsum(lens)])
    ci = np.concatenate([np.sort(rng.choice(3000, l, replace=False)) for l in lens]).astype(np.int64)
    v = np.ones(len(ci))
    L, sorted_ = delta16_sliced_auto_ref(rp, ci, v)
    plain = delta16_sliced_ref(rp, ci, v)
    assert sorted_ and L["slots"] < 0.7 * plain["slots"]
    rp, ci, v = synth.banded(6000, 128, 400, seed=4)     # 4 to 12 per row: too little saved
    assert not delta16_sliced_auto_ref(rp, ci, v)[1]
    rp, ci, v = synth.banded(6000, 480, 200, seed=4)     # 15 to 45 per row, staging lost
    plain, srt = delta16_sliced_ref(rp, ci, v), delta16_sliced_ref(rp, ci, v, sort_rows=True)
    assert plain["slots"] - srt["slots"] >= 6 * 6000
    assert 2 * staged_nnz_ref(rp, srt) < staged_nnz_ref(rp, plain)
    assert not delta16_sliced_auto_ref(rp, ci, v)[1]
    rp, ci, v = synth.banded(6000, 480, 20, seed=4)      # the same rows, staged either way: sorted
    L, sorted_ = delta16_sliced_auto_ref(rp, ci, v)
    plain = delta16_sliced_ref(rp, ci, v)
    assert sorted_ and 2 * staged_nnz_ref(rp, L) >= staged_nnz_ref(rp, plain) > 0
    rp, ci, v = synth.banded(6000, 320, 400, seed=4)     # 10 to 30 per row, staged near the
    L, sorted_ = delta16_sliced_auto_ref(rp, ci, v)      # first columns only: sorted
    assert sorted_ and staged_nnz_ref(rp, delta16_sliced_ref(rp, ci, v)) < 0.05 * len(ci)
    lens = np.full(1024, 12)                             # equal lengths: no padding to save
    rp = np.concatenate([[0], np.cumsum(lens)])
    ci = np.concatenate([np.sort(rng.choice(3000, 12, replace=False)) for _ in lens]).astype(np.int64)
    assert not delta16_sliced_auto_ref(rp, ci, np.ones(len(ci)))[1]
