"""Derived formats of the optimisation pool (test infrastructure).

* ``delta16_ref``   column-index compression (Section 3.3, Table 2, class MB).
  The paper stores 8- or 16-bit deltas between consecutive column indices of
  a row, never mixing widths.  Reading used here: 16-bit deltas from one
  reference column per block of consecutive rows (the block's smallest
  column), which a GPU decodes with a single add and no in-row scan or row
  lookup.  Feasible iff no block spans more than 65536 columns.
* ``delta16_sliced_ref``  the second layout of the same 16-bit offsets, for
  matrices whose rows in a group of 64 have nearly equal lengths (stencils):
  64-row slices stored column-major in pairs, one row per lane of a
  wavefront, each slice with its own reference column; a slice whose rows
  share at most 32 diagonals stores those diagonals once and a bit mask per
  row instead of any column data.  A combination of the MB optimisation with
  a GPU storage order, in the spirit of the paper's closing remarks on wider
  pools and multi-level optimisation.  ``delta8_codes_ref`` is the paper's
  other width: 8-bit deltas between consecutive columns of a row, with an
  escape code for a gap that does not fit; ``delta16_offset_bits_ref``
  chooses the width.
* ``merge_splits_ref``  start coordinates of the nonzero-balanced merge-path
  tiles (Merrill and Garland, SC'16): the merge of the row-end list
  ``rowptr[1..N]`` with the nonzero indices ``0..NNZ-1``, where nonzero j is
  taken before row end i exactly when ``j < rowptr[i+1]``.
* ``slice_csr_ref``  the column-sliced CSR of x blocking (one slice per XCD);
  ``xblock_split_ref`` takes rows with a long slice segment out of it.
* ``range_codes_ref``  16-bit column codes inside the other variants' work
  units (Section 3.3's column-index compression combined with another
  optimisation, the multi-level pool of the Conclusions): each unit - a
  merge-path tile (``merge_codes_ref``) or a row block of an x-block column
  slice (``xblock_codes_ref``) - takes its smallest column as reference and
  stores every column as its offset from it; feasible iff no unit spans
  more than 65535 columns.
* ``partition_ref``  the paper's default static partition: contiguous row
  ranges with (as nearly as possible) equal nonzeros (Section 3.2.1).
* ``to_bf16_bits_ref`` / ``to_f32_ref``  value rounding for the precision
  path, round-to-nearest-even straight from FP64 (one rounding).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def delta16_ref(rowptr, colind, block_rows: int = 256):
    """(feasible, base int32[B], off uint16[NNZ]) for blocks of ``block_rows`` rows.

    Block b holds rows [b*block_rows, (b+1)*block_rows); its reference column
    base_b is the smallest column of the block's nonzeros (0 if it has none)
    and every nonzero of the block stores off_k = c_k - base_b.  Feasible iff
    every offset fits 16 bits (each block spans at most 65536 columns).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    n = len(rowptr) - 1
    nb = (n + block_rows - 1) // block_rows
    base = np.zeros(nb, dtype=np.int64)
    off = np.zeros(len(colind), dtype=np.int64)
    feasible = True
    for b in range(nb):
        a, e = rowptr[b * block_rows], rowptr[min(n, (b + 1) * block_rows)]
        if a < e:
            base[b] = colind[a:e].min()
            off[a:e] = colind[a:e] - base[b]
            if off[a:e].max() > 65535:
                feasible = False
    return feasible, base.astype(np.int32), (off & 0xFFFF).astype(np.uint16)


SLICE_ROWS = 64          # rows per slice: one per lane of a wavefront
SLICE_MAX_PAD = 1.35     # sliced layout only if its slots are at most this many per nonzero,
SLICE_MAX_PAD_LONG = 1.6  # or this many when the rows average at least
SLICE_LONG_MEAN = 7.5     # this many nonzeros
SLICE_MAX_SPAN_LONG = 8192  # and the offset slices span fewer columns than this
SORT_MIN_SAVED = 8        # slots per row that sorting rows by length must save,
SORT_MIN_SAVED_FREE = 4   # or this many where the plain layout stages little x


SELL_WINDOW = 256  # rows per window of the length-sorted sliced layout


def sell_perm_ref(rowptr, window: int = SELL_WINDOW):
    """Row order of the length-sorted sliced layout (sorting rows by length
    inside windows, as in Kreutzer et al.'s SELL-C-sigma, to cut a slice's
    padding): the rows of each window of ``window`` consecutive rows, longest
    first, ties in row order.  Position p of the layout holds row perm[p]."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = len(rowptr) - 1
    lens = rowptr[1:] - rowptr[:-1]
    perm = np.empty(n, dtype=np.int64)
    for w0 in range(0, n, window):
        rows = sorted(range(w0, min(n, w0 + window)), key=lambda i: (-int(lens[i]), i))
        perm[w0:w0 + len(rows)] = rows
    return perm


def delta16_sliced_ref(rowptr, colind, val, slice_rows: int = SLICE_ROWS, sort_rows: bool = False):
    """The sliced delta16 layout of a CSR matrix.

    Slice s holds rows [64 s, 64 s + 64) (lanes past the last row are empty
    rows).  With ``sort_rows`` it holds rows perm[64 s .. 64 s + 63] of
    ``sell_perm_ref`` instead (positions past the last row empty) and every
    slice is an offset slice; everything below then reads "the row at
    position p" for "row p".  Each slice is of one of two kinds:

    * diagonal (kind 1): U_s, the sorted distinct values of c - r over the
      slice's nonzeros, has at most 32 entries and, rounded up to an even
      count, is no wider than the slice's longest row rounded up to even.
      Position k of a row holds its nonzero on diagonal U_s[k], if any; the
      row's mask has bit k set for each diagonal it has.  Columns are not
      stored: the column at position k of row r is r + U_s[k].
    * offset (kind 0): position k of a row holds its k-th nonzero (from 0,
      in column order) and off[slot] = c - base_s, base_s being the smallest
      column among the slice's nonzeros (0 if none).

    The slice's width w_s is |U_s| or its longest row, rounded up to even,
    and its storage starts at unit u_s = sum_{t<s} w_t / 2, where one unit is
    128 slots (a pair of positions for each of the 64 lanes).  Position k of
    the row in lane l lives at

        slot = 128 u_s + 128 (k // 2) + 2 l + (k % 2)

    with vals[slot] = a; every other slot (and off[] of diagonal slices)
    holds 0.  Returns a dict with kind, ndiag (|U_s| of diagonal slices, else
    0), width, base, units, span (int32[S]; span_s is the largest column of
    the slice minus base_s, 0 if it has no nonzeros), diag
    (int32[32 S]: U_s zero-padded, zeros for offset slices), mask (uint32[N]:
    0 in offset slices), slots (64 sum w_s), off (int64[slots]; the caller
    checks they fit 16 bits), vals (float64[slots]), nnz_offset (the
    nonzeros of the offset slices) and perm (the row at each position: the
    identity unless sorted).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    n = len(rowptr) - 1
    perm = sell_perm_ref(rowptr) if sort_rows else np.arange(n, dtype=np.int64)
    ns = (n + slice_rows - 1) // slice_rows
    kind = np.zeros(ns, dtype=np.int64)
    ndiag = np.zeros(ns, dtype=np.int64)
    width = np.zeros(ns, dtype=np.int64)
    base = np.zeros(ns, dtype=np.int64)
    span = np.zeros(ns, dtype=np.int64)
    diag = np.zeros(32 * ns, dtype=np.int64)
    diag_sets = []
    for s in range(ns):
        rows = perm[s * slice_rows:min(n, (s + 1) * slice_rows)]
        lens = rowptr[rows + 1] - rowptr[rows]
        longest = int(lens.max()) if len(lens) else 0
        w_off = longest + (longest % 2)
        cols = np.concatenate([colind[rowptr[i]:rowptr[i + 1]] for i in rows]) if len(rows) else colind[:0]
        base[s] = cols.min() if len(cols) else 0
        span[s] = cols.max() - base[s] if len(cols) else 0
        rel = sorted({int(colind[j]) - int(i) for i in rows
                      for j in range(rowptr[i], rowptr[i + 1])})
        d_even = len(rel) + (len(rel) % 2)
        if not sort_rows and len(rel) <= 32 and d_even <= w_off:
            kind[s], ndiag[s], width[s] = 1, len(rel), d_even
            diag[32 * s:32 * s + len(rel)] = rel
        else:
            width[s] = w_off
        diag_sets.append(rel)
    units = np.zeros(ns, dtype=np.int64)
    for s in range(1, ns):
        units[s] = units[s - 1] + width[s - 1] // 2
    slots = int(slice_rows * width.sum())
    off = np.zeros(slots, dtype=np.int64)
    vals = np.zeros(slots, dtype=np.float64)
    mask = np.zeros(n, dtype=np.int64)
    nnz_offset = 0
    pair_stride = 2 * slice_rows
    for p in range(n):
        i = int(perm[p])
        s, lane = divmod(p, slice_rows)
        for k_row in range(rowptr[i + 1] - rowptr[i]):
            j = rowptr[i] + k_row
            if kind[s]:
                k = diag_sets[s].index(int(colind[j]) - i)
                mask[i] |= 1 << k
            else:
                k = k_row
                nnz_offset += 1
            slot = pair_stride * units[s] + pair_stride * (k // 2) + 2 * lane + (k % 2)
            if not kind[s]:
                off[slot] = colind[j] - base[s]
            vals[slot] = val[j]
    return dict(kind=kind.astype(np.int32), ndiag=ndiag.astype(np.int32),
                width=width.astype(np.int32),
                base=base.astype(np.int32), units=units.astype(np.int32),
                span=span.astype(np.int32),
                diag=diag.astype(np.int32), mask=mask.astype(np.uint32), slots=slots,
                off=off, vals=vals, nnz_offset=nnz_offset, perm=perm.astype(np.int32))


ESCAPE = 255  # 8-bit code of a column stored in full


def delta8_codes_ref(rowptr, colind, L, slice_rows: int = SLICE_ROWS):
    """8-bit delta coding of the offset slices of a sliced layout ``L``
    (Section 3.3: delta indexing of the column indices, Pooch and Nieder).

    In an offset slice s the k-th nonzero of the row in lane l, column c_k,
    gets the code d = c_k - c_{k-1}, with c_{-1} = base_s, when d <= 254;
    otherwise the escape code 255, and c_k itself goes to the slice's escape
    area: the e-th escape of lane l is esc[64 (eunits_s + e) + l], where E_s
    is the largest number of escapes of a row of the slice and eunits the
    exclusive prefix sums of E.  Codes go in groups of four positions per
    lane: code k of lane l of slice s is at

        128 (u_s + s) + 256 (k // 4) + 4 l + (k % 4)

    (u_s the slice's unit offset; one spare unit per slice covers a width
    that is not a multiple of 4), 128 (sum of widths / 2 + S) bytes in all.
    Every other code is 0 (so a padding position repeats the row's last
    column) and unused escape entries hold 0.  Diagonal slices have no codes
    and E_s = 0.  Returns a dict with codes (uint8), E and eunits
    (int32[S]), esc (int32[64 sum E]) and escapes (the escaped nonzeros).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    n = len(rowptr) - 1
    ns = len(L["width"])
    E = np.zeros(ns, dtype=np.int64)
    perm = L.get("perm", np.arange(n))
    row_escapes = []
    for p in range(n):
        i = int(perm[p])
        s, lane = divmod(p, slice_rows)
        if L["kind"][s]:
            row_escapes.append([])
            continue
        prev, esc_cols = int(L["base"][s]), []
        for j in range(rowptr[i], rowptr[i + 1]):
            if colind[j] - prev >= ESCAPE:
                esc_cols.append(int(colind[j]))
            prev = int(colind[j])
        row_escapes.append(esc_cols)
        E[s] = max(E[s], len(esc_cols))
    eunits = np.zeros(ns, dtype=np.int64)
    for s in range(1, ns):
        eunits[s] = eunits[s - 1] + E[s - 1]
    codes = np.zeros(L["slots"] + 2 * slice_rows * ns, dtype=np.uint8)
    esc = np.zeros(slice_rows * int(E.sum()), dtype=np.int64)
    escapes = 0
    for p in range(n):
        i = int(perm[p])
        s, lane = divmod(p, slice_rows)
        if L["kind"][s]:
            continue
        prev, e = int(L["base"][s]), 0
        for k in range(rowptr[i + 1] - rowptr[i]):
            c = int(colind[rowptr[i] + k])
            slot = code_slot_ref(L["units"][s], s, lane, k, slice_rows)
            if c - prev >= ESCAPE:
                codes[slot] = ESCAPE
                esc[slice_rows * (eunits[s] + e) + lane] = c
                e += 1
                escapes += 1
            else:
                codes[slot] = c - prev
            prev = c
    return dict(codes=codes, E=E.astype(np.int32), eunits=eunits.astype(np.int32),
                esc=esc.astype(np.int32), escapes=escapes)


def code_slot_ref(unit: int, s: int, lane: int, k: int, slice_rows: int = SLICE_ROWS) -> int:
    """Byte of 8-bit code k of lane ``lane`` of slice s (unit offset ``unit``)."""
    return 2 * slice_rows * (int(unit) + s) + 4 * slice_rows * (k // 4) + 4 * lane + k % 4


def delta8_decode_ref(codes, esc, L, row_lengths, slice_rows: int = SLICE_ROWS):
    """The columns of every offset-slice row back from its codes (the
    inverse of ``delta8_codes_ref``), as a list of lists (empty for rows of
    diagonal slices)."""
    n = len(row_lengths)
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(L.get("perm", np.arange(n)), dtype=np.int64)] = np.arange(n)
    out = []
    for i, length in enumerate(row_lengths):
        s, lane = divmod(int(pos[i]), slice_rows)
        cols = []
        if not L["kind"][s]:
            c, e = int(L["base"][s]), 0
            for k in range(length):
                d = int(codes[code_slot_ref(L["units"][s], s, lane, k, slice_rows)])
                if d == ESCAPE:
                    c = int(esc[slice_rows * (int(L["eunits"][s]) + e) + lane])
                    e += 1
                else:
                    c += d
                cols.append(c)
        out.append(cols)
    return out


def delta16_offset_bits_ref(nnz_offset: int, escape_units: int) -> int:
    """Bits per stored column code of the sliced layout (Section 3.3: deltas
    of 8 or 16 bits, one width per matrix, never both).

    16 bits are offsets c - base_s, which always fit (a slice spans at most
    65536 columns).  8 bits are the delta codes of ``delta8_codes_ref``; their
    escape area holds 64 int32 entries per unit of E.  The matrix takes 8
    bits when it has offsets to store and that area costs at most half of the
    byte the codes save per nonzero: 256 sum E <= nnz_offset / 2.
    """
    return 8 if nnz_offset > 0 and 512 * escape_units <= nnz_offset else 16


SELL_X_WINDOW = 512  # x entries an offset slice can stage in LDS


def sliced_stages_x_ref(span: int, width: int, slice_rows: int = SLICE_ROWS) -> bool:
    """Whether an offset slice reads x from a staged copy of its column
    window: its columns lie within SELL_X_WINDOW of its reference column and
    its gathers (64 per pair of positions) number at least twice the window
    it would load."""
    return span < SELL_X_WINDOW and 2 * (span + 1) <= slice_rows * width


def staged_nnz_ref(rowptr, L, slice_rows: int = SLICE_ROWS) -> int:
    """Nonzeros of the offset slices of layout L that stage x."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    lens = np.diff(rowptr)[np.asarray(L["perm"], dtype=np.int64)]
    total = 0
    for s in range(len(L["width"])):
        if L["kind"][s] == 0 and sliced_stages_x_ref(int(L["span"][s]), int(L["width"][s]), slice_rows):
            total += int(lens[s * slice_rows:(s + 1) * slice_rows].sum())
    return total


def delta16_sort_ref(slots: int, slots_sorted: int, ndiag: int, nslices: int, nnz: int, n: int,
                     staged: int = 0, staged_sorted: int = 0, nnz_offset: int = 0) -> bool:
    """Whether the sliced layout sorts its rows (``sell_perm_ref``).

    Sorting gives up diagonal slices, costs a 4-byte row index per row and
    scattered y stores (the kernel reads the row it owns and stores y
    there), and widens each slice's column span to its window's, so that a
    slice of a band may no longer stage x.  It is taken when the plain layout
    has at most 1% diagonal slices and over 5% of padding, sorting saves at
    least 5% of its slots, and either the plain layout stages x for under
    half of its ``nnz_offset`` offset-slice nonzeros and sorting saves
    SORT_MIN_SAVED_FREE slots per row, or sorting keeps at least half of the
    staging (``staged_sorted`` against ``staged``, the nonzeros of staging
    slices, ``staged_nnz_ref``) and saves SORT_MIN_SAVED slots per row."""
    if ndiag * 100 > nslices or slots * 100 <= 105 * nnz:
        return False
    saved = slots - slots_sorted
    if saved * 20 < slots:
        return False
    if 2 * staged < nnz_offset and saved >= SORT_MIN_SAVED_FREE * n:
        return True
    return 2 * staged_sorted >= staged and saved >= SORT_MIN_SAVED * n


def sliced_max_span_ref(L) -> int:
    """The largest column span of an offset slice of layout L (0 if none)."""
    spans = np.asarray(L["span"])[np.asarray(L["kind"]) == 0]
    return int(spans.max()) if len(spans) else 0


def delta16_sliced_auto_ref(rowptr, colind, val):
    """The sliced layout under the automatic row order: the plain layout, or
    the length-sorted one when ``delta16_sort_ref`` takes it.  Returns the
    layout and whether it is sorted."""
    L = delta16_sliced_ref(rowptr, colind, val)
    n, nnz, ns = len(rowptr) - 1, len(colind), len(L["width"])
    ndiag = int(np.count_nonzero(L["kind"]))
    if n == 0 or ndiag * 100 > ns or L["slots"] * 100 <= 105 * nnz:
        return L, False  # the rule declines before the sorted layout is needed
    Ls = delta16_sliced_ref(rowptr, colind, val, sort_rows=True)
    if delta16_sort_ref(L["slots"], Ls["slots"], ndiag, ns, nnz, n,
                        staged_nnz_ref(rowptr, L), staged_nnz_ref(rowptr, Ls), L["nnz_offset"]):
        return Ls, True
    return L, False


def delta16_layout_ref(block_feasible: bool, slots: int, nnz: int, n: int, max_span: int = 0) -> int:
    """Layout of the delta16 variant: -1 infeasible, 0 rows streamed, 1 sliced.

    A 64-row slice lies inside one block of the streamed layout, so it spans
    no more columns than that block: the sliced layout is feasible whenever
    the streamed one is.  It is taken when padding keeps its slots (in the
    row order ``delta16_sort_ref`` takes) at most 1.35 times the nonzero
    count, or 1.6 times when the rows of the n-row matrix average at least
    7.5 nonzeros and its offset slices span fewer than 8192 columns
    (``max_span``, the largest span of an offset slice), and NNZ < 2^30.
    """
    if not block_feasible:
        return -1
    if nnz >= 1 << 30:
        return 0
    ok = slots <= SLICE_MAX_PAD * nnz or (2 * nnz >= 2 * SLICE_LONG_MEAN * n and
                                          slots <= SLICE_MAX_PAD_LONG * nnz and
                                          max_span < SLICE_MAX_SPAN_LONG)
    return 1 if ok else 0


def merge_walk_ref(rowptr, items_per_tile: int):
    """Split coordinates by walking the whole merge sequentially.

    Returns (split_row, split_nnz), each int32[ntiles + 1], where tile t starts
    on diagonal min(t * items_per_tile, N + NNZ).
    """
    rowptr = [int(v) for v in rowptr]
    n = len(rowptr) - 1
    nnz = rowptr[-1]
    total = n + nnz
    ntiles = (total + items_per_tile - 1) // items_per_tile
    out_i, out_j = [0], [0]
    i = j = 0
    for d in range(1, total + 1):
        # consume one item: a nonzero if it belongs to the current row
        if j < nnz and (i == n or j < rowptr[i + 1]):
            j += 1
        else:
            i += 1
        if d % items_per_tile == 0 and d < total:
            out_i.append(i)
            out_j.append(j)
    while len(out_i) < ntiles + 1:
        out_i.append(i)
        out_j.append(j)
    return np.array(out_i, dtype=np.int32), np.array(out_j, dtype=np.int32)


def merge_search_ref(rowptr, items_per_tile: int):
    """The same split coordinates by binary search on each tile diagonal.

    On diagonal d the row coordinate is the smallest i in
    [max(0, d - NNZ), min(d, N)] with rowptr[i+1] > d - i - 1 (min(d, N) if
    there is none); the nonzero coordinate is d - i.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = len(rowptr) - 1
    nnz = int(rowptr[-1])
    total = n + nnz
    ntiles = (total + items_per_tile - 1) // items_per_tile
    si = np.zeros(ntiles + 1, dtype=np.int64)
    sj = np.zeros(ntiles + 1, dtype=np.int64)
    for t in range(ntiles + 1):
        d = min(t * items_per_tile, total)
        lo, hi = max(0, d - nnz), min(d, n)
        while lo < hi:
            mid = (lo + hi) // 2
            if rowptr[mid + 1] <= d - mid - 1:
                lo = mid + 1
            else:
                hi = mid
        si[t], sj[t] = lo, d - lo
    return si.astype(np.int32), sj.astype(np.int32)


def slice_csr_ref(rowptr, colind, n_cols: int, slices: int = 8):
    """Column-sliced CSR for x blocking.

    Columns are cut into ``slices`` slices of width ceil(M / slices) (column c
    lies in slice c // width).  Returns (rowptrs int32[slices, N+1],
    colind int32[NNZ]) where slice s keeps, row by row, the nonzeros of A whose
    columns fall in it, and the column array holds slice 0's nonzeros, then
    slice 1's, and so on.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    n = len(rowptr) - 1
    width = (n_cols + slices - 1) // slices if n_cols > 0 else 1
    rps = np.zeros((slices, n + 1), dtype=np.int64)
    parts = [[] for _ in range(slices)]
    for i in range(n):
        row = colind[rowptr[i]:rowptr[i + 1]]
        sl = row // width
        for s in range(slices):
            seg = row[sl == s]
            parts[s].append(seg)
            rps[s, i + 1] = rps[s, i] + len(seg)
    cols = [np.concatenate(p) if p else np.zeros(0, np.int64) for p in parts]
    return rps.astype(np.int32), np.concatenate(cols).astype(np.int32)


def xblock_split_ref(rowptr, colind, n_cols: int, slices: int, max_seg: int = 128,
                     max_share: float = 0.25):
    """The x-block split into short and long rows.

    A row is long when one of its slice segments (slice_csr_ref) has more
    than ``max_seg`` nonzeros.  When the long rows hold at most ``max_share``
    of the nonzeros they leave the slices (their segments become empty) and
    are summed from the original CSR instead; otherwise nothing is split.
    Returns (long row indices int32[L] in ascending order, slice row
    pointers int32[slices, N+1], slice-major columns int32) of the slices.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    n = len(rowptr) - 1
    rps, _ = slice_csr_ref(rowptr, colind, n_cols, slices)
    seg = np.diff(rps.astype(np.int64), axis=1)          # [slices, N]
    long_rows = np.nonzero(seg.max(axis=0, initial=0) > max_seg)[0] if n else np.zeros(0, np.int64)
    long_nnz = int(np.sum(rowptr[long_rows + 1] - rowptr[long_rows]))
    if len(long_rows) == 0 or long_nnz > max_share * len(colind):
        rps, cols = slice_csr_ref(rowptr, colind, n_cols, slices)
        return np.zeros(0, np.int32), rps, cols
    keep = np.ones(n, dtype=bool)
    keep[long_rows] = False
    L = np.diff(rowptr)
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum(np.where(keep, L, 0))
    ci2 = np.concatenate([colind[rowptr[i]:rowptr[i + 1]] for i in range(n) if keep[i]] or
                         [np.zeros(0, np.int64)])
    rps, cols = slice_csr_ref(rp2, ci2, n_cols, slices)
    return long_rows.astype(np.int32), rps, cols


def range_codes_ref(colind, bounds):
    """(feasible, base int32[R], off uint16[len(colind)], max span) for the
    ranges [bounds[k], bounds[k+1]) of a column array: base[k] is the range's
    smallest column (0 for an empty range) and off[j] = colind[j] - base[k]
    for j in range k.  Feasible iff every range spans at most 65535 columns
    (offsets are only filled in when feasible)."""
    colind = np.asarray(colind, dtype=np.int64)
    bounds = np.asarray(bounds, dtype=np.int64)
    R = len(bounds) - 1
    base = np.zeros(R, dtype=np.int64)
    span = 0
    for k in range(R):
        seg = colind[bounds[k]:bounds[k + 1]]
        if len(seg):
            base[k] = seg.min()
            span = max(span, int(seg.max() - seg.min()))
    feasible = span <= 65535
    off = np.zeros(len(colind), dtype=np.uint16)
    if feasible:
        for k in range(R):
            a, b = bounds[k], bounds[k + 1]
            off[a:b] = (colind[a:b] - base[k]).astype(np.uint16)
    return feasible, base.astype(np.int32), off, span


def merge_codes_ref(rowptr, colind, items_per_tile: int = 2048):
    """16-bit codes inside merge-path tiles: the ranges are the tiles' nonzero
    ranges [split_nnz[t], split_nnz[t+1]) of the sequential merge walk."""
    _, sj = merge_walk_ref(rowptr, items_per_tile)
    return range_codes_ref(colind, sj)


def xblock_codes_ref(rowptr, colind, n_cols: int, slices: int, block_rows: int,
                     max_seg: int = 128, max_share: float = 0.25):
    """16-bit codes inside the x-block slices: for every slice (of the split
    of ``xblock_split_ref``) and block b of ``block_rows`` rows, the range of
    the slice-major columns of rows [b H, min((b+1) H, N)).  Returns
    (feasible, base int32[slices * nblocks] (slice-major), off uint16 at the
    positions of the slice-major columns, max span)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = len(rowptr) - 1
    _, rps, cols = xblock_split_ref(rowptr, colind, n_cols, slices, max_seg, max_share)
    nb = (n + block_rows - 1) // block_rows
    bounds, start = [0], 0
    for s in range(slices):
        srp = rps[s].astype(np.int64)
        for b in range(nb):
            bounds.append(start + int(srp[min((b + 1) * block_rows, n)]))
        start += int(srp[n])
    # ranges are consecutive: slice s block b ends where block b+1 (or the
    # next slice's first block) starts
    return range_codes_ref(cols, bounds)


def partition_ref(rowptr, parts: int):
    """Row boundaries b[0..parts] of the equal-nonzero static partition.

    b_0 = 0, b_parts = N and, in between, b_p is the first row whose start
    offset reaches ceil(p * NNZ / parts).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = len(rowptr) - 1
    nnz = int(rowptr[-1])
    b = np.zeros(parts + 1, dtype=np.int64)
    for p in range(1, parts):
        target = -((-p * nnz) // parts)
        b[p] = int(np.searchsorted(rowptr, target, side="left"))
    b[parts] = n
    return b.astype(np.int32)


def to_f32_ref(val) -> np.ndarray:
    """FP64 -> FP32, round to nearest even (the C conversion)."""
    return np.asarray(val, dtype=np.float64).astype(np.float32)


def _bf16_bits_exact(x: float) -> int:
    """bfloat16 bits of x by exact rational rounding (half to even)."""
    if x != x:
        return 0x7FC0
    sign = 0x8000 if (x < 0 or (x == 0 and np.signbit(x))) else 0
    a = abs(x)
    if a == 0:
        return sign
    if a == float("inf"):
        return sign | 0x7F80
    fa = Fraction(a)
    e = fa.numerator.bit_length() - fa.denominator.bit_length()
    if Fraction(2) ** e > fa:
        e -= 1                      # now 2**e <= a < 2**(e+1)
    if e < -126:                    # subnormal: units of 2**-133
        s = round(fa * 2 ** 133)
        return sign | s             # s == 128 encodes the smallest normal
    s = round(fa * Fraction(2) ** (7 - e))   # 128 <= s <= 256
    if s == 256:
        s, e = 128, e + 1
    if e > 127:
        return sign | 0x7F80
    return sign | ((e + 127) << 7) | (s - 128)


def to_bf16_bits_ref(val) -> np.ndarray:
    """FP64 -> bfloat16 bit patterns (uint16), one round-to-nearest-even.

    Normal-range values are rounded on the FP64 bit pattern (keep 7 fraction
    bits, round on the next bit with the rest as sticky); zeros, subnormal
    results, overflow and non-finite values go through exact rational
    rounding.
    """
    v = np.ascontiguousarray(np.asarray(val, dtype=np.float64))
    bits = v.view(np.uint64)
    sign = ((bits >> np.uint64(63)) << np.uint64(15)).astype(np.uint64)
    exp = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    mant = bits & np.uint64((1 << 52) - 1)
    keep = mant >> np.uint64(45)                       # 7 fraction bits
    rbit = (mant >> np.uint64(44)) & np.uint64(1)
    sticky = (mant & np.uint64((1 << 44) - 1)) != 0
    up = (rbit == 1) & (sticky | ((keep & np.uint64(1)) == 1))
    body = ((exp + 127).astype(np.uint64) << np.uint64(7)) + keep + up.astype(np.uint64)
    out = (sign | body).astype(np.uint64)
    normal = (exp >= -126) & (exp <= 127)
    normal &= body < np.uint64(0x7F80)                 # no overflow to inf
    res = np.where(normal, out, np.uint64(0)).astype(np.uint16)
    for i in np.nonzero(~normal)[0]:
        res[i] = _bf16_bits_exact(float(v[i]))
    return res


def bf16_bits_to_f64(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)
