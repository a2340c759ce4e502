"""Profiling-based classifier and class-to-optimisation map (test infrastructure).

Section 3.2.1: three micro-benchmarks modify baseline CSR SpMV — ``noxmiss``
(irregular accesses to x removed; the paper zeroes every column index, which
on a GPU makes every wavefront hit one cache line, so row i's indices are
mapped to i instead), ``inflate`` (64-bit row pointers and column indices) and ``balance`` (per-thread execution times and their
arithmetic mean, under the default static partition with equal nonzeros per
thread).  Each yields a speedup over baseline CSR, except ``inflate`` whose
slowdown (the inverse) is used.  The benchmarks are examined from the
highest score down; the first whose score exceeds its threshold names the
class (noxmiss -> CML, inflate -> MB, balance -> IMB); if none does, the
class is CMP.  The thresholds are not given in the paper (set empirically);
they are inputs here.

GPU reading of ``balance``: the per-partition durations d_p are taken on
the device clock inside the baseline runs, and the score is
max_p d_p / mean_p d_p (the statically partitioned kernel lasts about as
long as its slowest partition).  Ties in the descending order keep the
order (noxmiss, inflate, balance).  A score whose denominator is not
positive is 0.

Table 2 maps classes to optimisations; the GPU pool remaps them:
CML -> xblock_lds (x blocking by column slices) if feasible, else csr_vector;
MB  -> delta16 (16-bit column offsets) if feasible, else csr_vector;
IMB -> merge_path (nonzero-balanced merge-based CSR);
CMP -> short_row if nnz_avg <= theta[3], else csr_vector.
"""
from __future__ import annotations

CLASSES = ["CML", "MB", "IMB", "CMP"]
VARIANTS = ["csr_scalar", "csr_vector", "merge_path", "delta16",
            "xblock_lds", "short_row"]
V_CSR_SCALAR, V_CSR_VECTOR, V_MERGE_PATH, V_DELTA16, V_XBLOCK_LDS, V_SHORT_ROW = range(6)
K_CML, K_MB, K_IMB, K_CMP = range(4)


def _ratio(a: float, b: float) -> float:
    return a / b if b > 0 else 0.0


def profile_scores(meas) -> list[float]:
    """meas = (t_base, t_nox, t_inf, d_max, d_mean) -> (s_nox, s_inf, s_bal)."""
    t_base, t_nox, t_inf, d_max, d_mean = (float(v) for v in meas)
    return [_ratio(t_base, t_nox), _ratio(t_inf, t_base), _ratio(d_max, d_mean)]


def classify(scores, theta) -> int:
    """Descending threshold cascade over the three scores."""
    order = sorted(range(3), key=lambda b: -scores[b])  # stable: ties keep order
    for b in order:
        if scores[b] > theta[b]:
            return [K_CML, K_MB, K_IMB][b]
    return K_CMP


def class_to_variant(klass: int, features, theta, feasible_bits: int) -> int:
    def ok(v):
        return (feasible_bits >> v) & 1
    if klass == K_CML:
        return V_XBLOCK_LDS if ok(V_XBLOCK_LDS) else V_CSR_VECTOR
    if klass == K_MB:
        return V_DELTA16 if ok(V_DELTA16) else V_CSR_VECTOR
    if klass == K_IMB:
        return V_MERGE_PATH
    return V_SHORT_ROW if features[2] <= theta[3] else V_CSR_VECTOR


def decide_profile_ref(meas, features, theta, feasible_bits: int):
    """(variant, class) from the five measurements, features and thresholds."""
    k = classify(profile_scores(meas), theta)
    return class_to_variant(k, features, theta, feasible_bits), k
