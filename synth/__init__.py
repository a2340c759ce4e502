"""Seeded synthetic CSR matrices and vectors.

This module only *generates inputs*: it holds none of the SpMV method's
arithmetic (no products, no features, no selection).  Both the CPU oracle
side (tests, reference runs) and the benchmark use it; the HIP library has
its own device generator, written separately from the same definitions
below, and the tests check that the two produce identical bytes.

Random numbers come from one counter-based generator: the SplitMix64
output function of Steele, Lea and Flood (OOPSLA 2014) applied to a
Weyl sequence, so element ``i`` of stream ``s`` for seed ``seed`` is

    key(seed, s) = fmix(seed * G + s * S + 1)
    h(seed, s, i) = fmix(key(seed, s) + (i + 1) * G)          (mod 2**64)

with ``G = 0x9E3779B97F4A7C15``, ``S = 0xD1B54A32D192ED03`` and ``fmix`` the
SplitMix64 finaliser.  Derived draws use only exact integer or exactly
representable floating-point operations, so any two implementations agree
bit for bit:

* ``u01(h)   = (h >> 11) * 2**-53``            (double in [0, 1))
* ``upm1(h)  = 2 * u01(h) - 1``                (double in [-1, 1))
* ``below(h, n) = ((h >> 32) * n) >> 32``      (integer in [0, n), n < 2**32)

Column sets are drawn "one per stratum": a row with ``L`` entries over the
column range ``[lo, hi)`` of size ``R >= L`` splits the range into ``L``
strata ``[lo + j*R//L, lo + (j+1)*R//L)`` and draws one column uniformly in
each, which yields sorted, distinct columns with no rejection.  The counter
of nonzero ``k`` (its global CSR position) selects its column and value.

Every family returns ``(rowptr int32[N+1], colind int32[NNZ], val float64[NNZ])``
with columns strictly increasing inside each row.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

G = 0x9E3779B97F4A7C15
S = 0xD1B54A32D192ED03
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1

# stream ids (shared with the device generator's definition)
ST_X = 1        # dense vector x
ST_VAL = 2      # nonzero values
ST_LEN = 3      # row lengths
ST_COL = 4      # column draws
ST_MISC = 5     # one-off draws (forced long row position)
ST_SWEEP = 100  # per-matrix parameters of the sweep families

_U64 = np.uint64


def fmix_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (mod 2**64)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def key_int(seed: int, stream: int) -> int:
    return fmix_int((seed * G + stream * S + 1) & MASK)


def h_int(seed: int, stream: int, i: int) -> int:
    return fmix_int((key_int(seed, stream) + (i + 1) * G) & MASK)


def u01_int(h: int) -> float:
    return (h >> 11) * 2.0 ** -53


def _fmix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> _U64(30)
        z *= _U64(M1)
        z ^= z >> _U64(27)
        z *= _U64(M2)
        z ^= z >> _U64(31)
    return z


def hash_array(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """h(seed, stream, i) for every i in ``idx`` (uint64 array)."""
    key = _U64(key_int(seed, stream))
    i = np.asarray(idx).astype(np.uint64)
    with np.errstate(over="ignore"):
        z = key + (i + _U64(1)) * _U64(G)
    return _fmix(z)


def u01(h: np.ndarray) -> np.ndarray:
    return (h >> _U64(11)).astype(np.float64) * (2.0 ** -53)


def upm1(h: np.ndarray) -> np.ndarray:
    return 2.0 * u01(h) - 1.0


def below(h: np.ndarray, n) -> np.ndarray:
    """Integer in [0, n) from the high 32 bits of ``h`` (n < 2**32)."""
    hi = (h >> _U64(32)).astype(np.uint64)
    n = np.asarray(n).astype(np.uint64)
    with np.errstate(over="ignore"):
        return ((hi * n) >> _U64(32)).astype(np.int64)


def vector(n: int, seed: int) -> np.ndarray:
    """x ~ U[-1, 1) from ``seed`` (stream ST_X)."""
    return upm1(hash_array(seed, ST_X, np.arange(n, dtype=np.int64)))


def int_vector(n: int, seed: int, amp: int = 8) -> np.ndarray:
    """Integer-valued x in [-amp, amp] (exact in BF16/FP32 for amp <= 256)."""
    h = hash_array(seed, ST_X, np.arange(n, dtype=np.int64))
    return (below(h, 2 * amp + 1) - amp).astype(np.float64)


# ----------------------------------------------------------------------------
# building blocks


def _rowptr_from_lengths(lengths: np.ndarray) -> np.ndarray:
    rp = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=rp[1:])
    if rp[-1] >= 2 ** 31:
        raise ValueError("nnz >= 2**31 is not supported")
    return rp


def strata_columns(rowptr: np.ndarray, lo: np.ndarray, hi: np.ndarray,
                   seed: int) -> np.ndarray:
    """One uniform column per stratum for every row (see module docstring)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = len(rowptr) - 1
    L = np.diff(rowptr)
    nnz = int(rowptr[-1])
    if nnz == 0:
        return np.zeros(0, dtype=np.int32)
    rows = np.repeat(np.arange(n, dtype=np.int64), L)
    k = np.arange(nnz, dtype=np.int64)
    j = k - rowptr[rows]
    Lr = L[rows]
    lo_r = np.asarray(lo, dtype=np.int64)[rows]
    R = np.asarray(hi, dtype=np.int64)[rows] - lo_r
    if np.any(R < Lr):
        raise ValueError("row has more entries than its column range")
    start = (j * R) // Lr
    width = ((j + 1) * R) // Lr - start
    col = lo_r + start + below(hash_array(seed, ST_COL, k), width)
    return col.astype(np.int32)


def random_values(nnz: int, seed: int) -> np.ndarray:
    return upm1(hash_array(seed, ST_VAL, np.arange(nnz, dtype=np.int64)))


def int_values(nnz: int, seed: int, amp: int = 8) -> np.ndarray:
    h = hash_array(seed, ST_VAL, np.arange(nnz, dtype=np.int64))
    return (below(h, 2 * amp + 1) - amp).astype(np.float64)


# ----------------------------------------------------------------------------
# stencils (natural ordering; the neighbour offsets come out column-sorted)


def _stencil(dims, offsets, diag_value, off_value, seed, values):
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    if n == 0:
        return (np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    coords = np.indices(dims).reshape(len(dims), -1).astype(np.int64)
    strides = np.array([int(np.prod(dims[a + 1:])) for a in range(len(dims))],
                       dtype=np.int64)
    cols, valid = [], []
    for off in sorted(offsets):
        c = coords + np.array(off, dtype=np.int64)[:, None]
        ok = np.all((c >= 0) & (c < np.array(dims)[:, None]), axis=0)
        cols.append(np.where(ok, (c * strides[:, None]).sum(axis=0), -1))
        valid.append(ok)
    cols = np.stack(cols, axis=1)          # [n, n_off] sorted by column
    valid = np.stack(valid, axis=1)
    L = valid.sum(axis=1)
    rowptr = _rowptr_from_lengths(L)
    colind = cols[valid].astype(np.int32)  # row-major: rows in order
    nnz = int(rowptr[-1])
    if values == "const":
        diag = (np.repeat(np.arange(n, dtype=np.int64), L) == colind)
        val = np.where(diag, float(diag_value), float(off_value))
    elif values == "random":
        val = random_values(nnz, seed)
    elif values == "int":
        val = int_values(nnz, seed)
    else:
        raise ValueError(values)
    return rowptr.astype(np.int32), colind, val.astype(np.float64)


def _offsets(ndim, kind):
    import itertools
    allo = list(itertools.product([-1, 0, 1], repeat=ndim))
    if kind == "star":
        return [o for o in allo if sum(abs(t) for t in o) <= 1]
    return allo  # full 3^ndim box


def laplace2d(n: int, seed: int = 0, values: str = "const"):
    """5-point Laplacian on an n x n grid: 4 on the diagonal, -1 off it."""
    return _stencil((n, n), _offsets(2, "star"), 4.0, -1.0, seed, values)


def stencil2d_9(n: int, seed: int = 0, values: str = "random"):
    """9-point 2D box (3 x 3) on an n x n grid: 8 on the diagonal, -1 off it."""
    return _stencil((n, n), _offsets(2, "box"), 8.0, -1.0, seed, values)


def stencil3d_7(n: int, seed: int = 0, values: str = "random"):
    """7-point 3D star on an n^3 grid: 6 on the diagonal, -1 off it."""
    return _stencil((n, n, n), _offsets(3, "star"), 6.0, -1.0, seed, values)


def stencil3d_27(n: int, seed: int = 0, values: str = "const"):
    """27-point 3D box on an n^3 grid: 26 on the diagonal, -1 off it."""
    return _stencil((n, n, n), _offsets(3, "box"), 26.0, -1.0, seed, values)


# ----------------------------------------------------------------------------
# random-pattern families


def uniform_random(n_rows: int, n_cols: int, per_row: int, seed: int,
                   values: str = "random"):
    """Every row has ``per_row`` entries, one per stratum over [0, n_cols)."""
    L = np.full(n_rows, min(per_row, n_cols), dtype=np.int64)
    rowptr = _rowptr_from_lengths(L)
    lo = np.zeros(n_rows, dtype=np.int64)
    hi = np.full(n_rows, n_cols, dtype=np.int64)
    col = strata_columns(rowptr, lo, hi, seed)
    nnz = int(rowptr[-1])
    val = random_values(nnz, seed) if values == "random" else int_values(nnz, seed)
    return rowptr.astype(np.int32), col, val


def banded_lengths(n_rows: int, d16: int, seed: int) -> np.ndarray:
    """L_i = max(1, round(d * (0.5 + u))) with d = d16 / 16, in integers.

    With u = v / 2**32 (v the high 32 hash bits) this is
    ``(d16 * (2**31 + v) + 2**35) >> 36``.
    """
    v = (hash_array(seed, ST_LEN, np.arange(n_rows, dtype=np.int64))
         >> _U64(32)).astype(np.int64)
    L = (int(d16) * (2 ** 31 + v) + 2 ** 35) >> 36
    return np.maximum(L, 1)


def banded(n: int, d16: int, half_width: int, seed: int, values: str = "random"):
    """Row i draws about d entries from [i - W, i + W] (clipped to [0, n))."""
    L = banded_lengths(n, d16, seed)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - half_width)
    hi = np.minimum(n, i + half_width + 1)
    L = np.minimum(L, hi - lo)
    rowptr = _rowptr_from_lengths(L)
    col = strata_columns(rowptr, lo, hi, seed)
    nnz = int(rowptr[-1])
    val = random_values(nnz, seed) if values == "random" else int_values(nnz, seed)
    return rowptr.astype(np.int32), col, val


def random_rows(n: int, d16: int, seed: int, values: str = "random"):
    """Banded lengths, columns drawn over the whole range [0, n)."""
    L = np.minimum(banded_lengths(n, d16, seed), n)
    rowptr = _rowptr_from_lengths(L)
    lo = np.zeros(n, dtype=np.int64)
    hi = np.full(n, n, dtype=np.int64)
    col = strata_columns(rowptr, lo, hi, seed)
    nnz = int(rowptr[-1])
    val = random_values(nnz, seed) if values == "random" else int_values(nnz, seed)
    return rowptr.astype(np.int32), col, val


def pareto_lengths(n_rows: int, p16: int, cap: int, seed: int) -> np.ndarray:
    """Heavy-tailed row lengths with tail exponent 1.5.

    With a = p16 / 16 and v = (k + 1) / 2**32 (k the high 32 hash bits),
    L = clamp(floor(a * v**(-2/3)), 1, cap).  The floor is defined exactly as
    the largest integer l with ``l**3 * (k+1)**2 <= p16**3 * 2**52``.  A
    float estimate is used and every row whose estimate lies near an integer
    boundary is settled with exact Python integers.
    """
    k = (hash_array(seed, ST_LEN, np.arange(n_rows, dtype=np.int64))
         >> _U64(32)).astype(np.float64)
    a = p16 / 16.0
    t = a * np.power((k + 1.0) / 2.0 ** 32, -2.0 / 3.0)
    L = np.floor(t)
    near = (t - L < 1e-6) | (L + 1.0 - t < 1e-6)
    L = L.astype(np.int64)
    rhs = (p16 ** 3) << 52
    for r in np.nonzero(near & (t < cap + 2))[0]:
        kk = int(k[r]) + 1
        lo_, hi_ = 0, cap + 1  # largest l in [0, cap+1] with l^3 kk^2 <= rhs
        while lo_ < hi_:
            mid = (lo_ + hi_ + 1) // 2
            if mid ** 3 * kk * kk <= rhs:
                lo_ = mid
            else:
                hi_ = mid - 1
        L[r] = lo_
    return np.clip(L, 1, cap)


def powerlaw(n: int, p16: int, cap: int, seed: int, force_long: bool = True,
             values: str = "random"):
    """Pareto(1.5) row lengths, columns one per stratum over [0, n).

    If ``force_long`` one row (chosen by a seeded draw) gets exactly ``cap``
    entries.
    """
    L = np.minimum(pareto_lengths(n, p16, cap, seed), n)
    if force_long and n > 0:
        r = int(below(np.array([h_int(seed, ST_MISC, 0)], dtype=np.uint64), n)[0])
        L[r] = min(cap, n)
    rowptr = _rowptr_from_lengths(L)
    lo = np.zeros(n, dtype=np.int64)
    hi = np.full(n, n, dtype=np.int64)
    col = strata_columns(rowptr, lo, hi, seed)
    nnz = int(rowptr[-1])
    val = random_values(nnz, seed) if values == "random" else int_values(nnz, seed)
    return rowptr.astype(np.int32), col, val


def short_rows(n: int, seed: int, values: str = "random"):
    """Diagonal plus (i, i+1) when the row's draw has its top bit clear."""
    h = hash_array(seed, ST_LEN, np.arange(n, dtype=np.int64))
    extra = ((h >> _U64(63)) == 0) & (np.arange(n) + 1 < n)
    L = 1 + extra.astype(np.int64)
    rowptr = _rowptr_from_lengths(L)
    rows = np.repeat(np.arange(n, dtype=np.int64), L)
    j = np.arange(int(rowptr[-1]), dtype=np.int64) - rowptr[rows]
    col = (rows + j).astype(np.int32)
    nnz = int(rowptr[-1])
    val = random_values(nnz, seed) if values == "random" else int_values(nnz, seed)
    return rowptr.astype(np.int32), col, val


# ----------------------------------------------------------------------------
# named workloads


@dataclass
class MatrixSpec:
    """A generator call: family name plus integer parameters."""
    family: str
    params: dict = field(default_factory=dict)
    seed: int = 0
    x_seed: int = 0
    name: str = ""

    def build(self, values: str | None = None):
        p = dict(self.params)
        if values is not None:
            p["values"] = values
        fn = FAMILIES[self.family]
        return fn(seed=self.seed, **p)

    def x(self, n_cols: int) -> np.ndarray:
        return vector(n_cols, self.x_seed)


FAMILIES = {
    "laplace2d": laplace2d,
    "stencil2d_9": stencil2d_9,
    "stencil3d_7": stencil3d_7,
    "stencil3d_27": stencil3d_27,
    "uniform_random": uniform_random,
    "banded": banded,
    "random_rows": random_rows,
    "powerlaw": powerlaw,
    "short_rows": short_rows,
}

# Pareto scale 6.8 written as a multiple of 1/16 (6.8125)
C13_P16 = 109


def small_laplace() -> MatrixSpec:
    """5-point Laplacian, 64 x 64 grid; x seed 0."""
    return MatrixSpec("laplace2d", {"n": 64, "values": "const"}, 0, 0,
                      "laplace2d_64")


def class_matrices(scale: int = 1) -> list[MatrixSpec]:
    """The four FP64 bottleneck-class matrices.

    ``scale`` divides the sizes (for fast tests); ``scale=1`` is full size:
    27-point 100^3, uniform random 2M x 8/row, Pareto 1M with a 200k row,
    short rows 8M.
    """
    n3 = max(4, round(100 / scale ** (1 / 3)))
    return [
        MatrixSpec("stencil3d_27", {"n": n3, "values": "const"}, 1, 1,
                   f"stencil27_{n3}^3"),
        MatrixSpec("uniform_random", {"n_rows": 2_000_000 // scale,
                                       "n_cols": 2_000_000 // scale,
                                       "per_row": 8}, 2, 2,
                   f"random_{2_000_000 // scale}x8"),
        MatrixSpec("powerlaw", {"n": 1_000_000 // scale, "p16": C13_P16,
                                "cap": max(1, 200_000 // scale)}, 3, 3,
                   f"powerlaw_{1_000_000 // scale}"),
        MatrixSpec("short_rows", {"n": 8_000_000 // scale}, 4, 4,
                   f"shortrows_{8_000_000 // scale}"),
    ]


def sweep_spec(seed: int, n_min: float = 1e4, n_max: float = 4e6,
               d_max: float = 64.0) -> MatrixSpec:
    """One matrix of the mixed selector sweep (host-side parameters).

    N = floor(10**U[log10 n_min, log10 n_max]), d = 10**U[0, log10 d_max];
    the pattern is chosen by ``seed % 5``: stencil (2D-5, 2D-9, 3D-7, 3D-27),
    banded with half width d * {1, 4, 16, 64}, random, power-law (Pareto
    1.5 scaled to mean d, longest row N/5), or short rows (the diagonal plus
    (i, i+1) for about half the rows; d unused).  Only these host-side
    parameters use transcendental functions; per-row draws are exact.
    """
    u = [u01_int(h_int(seed, ST_SWEEP, i)) for i in range(4)]
    n = int(math.floor(10 ** (math.log10(n_min)
                              + u[0] * (math.log10(n_max) - math.log10(n_min)))))
    d = 10 ** (u[1] * math.log10(d_max))
    kind = seed % 5
    sub = min(3, int(u[2] * 4))
    d16 = max(16, int(round(d * 16)))
    if kind == 0:
        fam = ["laplace2d", "stencil2d_9", "stencil3d_7", "stencil3d_27"][sub]
        side = max(2, int(round(n ** (0.5 if fam.startswith(("laplace", "stencil2d"))
                                      else 1 / 3))))
        return MatrixSpec(fam, {"n": side, "values": "random"}, seed, seed,
                          f"sweep{seed}_{fam}_{side}")
    if kind == 1:
        w = max(1, int(round(d * [1, 4, 16, 64][sub])))
        return MatrixSpec("banded", {"n": n, "d16": d16, "half_width": w},
                          seed, seed, f"sweep{seed}_banded_{n}_{w}")
    if kind == 2:
        return MatrixSpec("random_rows", {"n": n, "d16": d16}, seed, seed,
                          f"sweep{seed}_random_{n}")
    if kind == 4:
        return MatrixSpec("short_rows", {"n": n}, seed, seed, f"sweep{seed}_shortrows_{n}")
    p16 = max(1, int(round(16 * d / 3)))
    return MatrixSpec("powerlaw", {"n": n, "p16": p16, "cap": max(1, n // 5),
                                   "force_long": False},
                      seed, seed, f"sweep{seed}_powerlaw_{n}")


def tiny_random_csr(rng: np.random.Generator, n_rows: int, n_cols: int,
                    density: float, int_valued: bool = True, amp: int = 8):
    """Small random CSR for property tests (numpy Generator, not the hash)."""
    mask = rng.random((n_rows, n_cols)) < density
    L = mask.sum(axis=1)
    rowptr = _rowptr_from_lengths(L).astype(np.int32)
    colind = np.nonzero(mask)[1].astype(np.int32)
    if int_valued:
        val = rng.integers(-amp, amp + 1, size=len(colind)).astype(np.float64)
    else:
        val = rng.uniform(-1, 1, size=len(colind))
    return rowptr, colind, val


# ----------------------------------------------------------------------------
# MLP initial parameters and minibatch order (random draws of the learned
# selector's training, generated here so that every implementation starts
# from the same numbers)

ST_INIT = 200
ST_SHUFFLE = 201
MLP_DIMS = (12, 64, 64, 6)


def he_uniform_params(seed: int) -> np.ndarray:
    """Flat float32 parameters W1,b1,W2,b2,W3,b3 (row-major, out x in).

    W ~ U[-b, b) with b = sqrt(6 / fan_in); biases are zero.
    """
    chunks, off = [], 0
    for li in range(3):
        fi, fo = MLP_DIMS[li], MLP_DIMS[li + 1]
        b = math.sqrt(6.0 / fi)
        h = hash_array(seed, ST_INIT, np.arange(off, off + fi * fo, dtype=np.int64))
        chunks.append((b * upm1(h)).astype(np.float32))
        chunks.append(np.zeros(fo, dtype=np.float32))
        off += fi * fo
    return np.concatenate(chunks)


def epoch_order(n: int, seed: int, epoch: int) -> np.ndarray:
    """A permutation of range(n) for one epoch (sort by hash)."""
    h = hash_array(seed * 1000003 + epoch, ST_SHUFFLE, np.arange(n, dtype=np.int64))
    return np.argsort(h, kind="stable")
