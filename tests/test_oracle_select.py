"""Pins of the profiling cascade (Section 3.2.1) and the class map (Table 2)."""
import itertools

import pytest

from oracle.select import (K_CML, K_CMP, K_IMB, K_MB, V_CSR_VECTOR, V_DELTA16,
                           V_MERGE_PATH, V_SHORT_ROW, V_XBLOCK_LDS, classify,
                           decide_profile_ref, profile_scores)

THETA = [2.0, 1.2, 1.5, 4.0]
ALL = 0b111111
FEAT = [1000.0, 27000.0, 27.0] + [0.0] * 9
SHORT = [1000.0, 1500.0, 1.5] + [0.0] * 9


def meas(s_nox, s_inf, s_bal, t_base=1.0):
    # t_base/t_nox = s_nox, t_inf/t_base = s_inf, d_max/d_mean = s_bal
    return (t_base, t_base / s_nox, t_base * s_inf, s_bal * 3.0, 3.0)


def test_scores_definition():
    s = profile_scores((2.0, 0.5, 3.0, 9.0, 3.0))
    assert s == [4.0, 1.5, 3.0]
    assert profile_scores((1.0, 0.0, 1.0, 1.0, 0.0)) == [0.0, 1.0, 0.0]


@pytest.mark.parametrize("scores,klass", [
    ((3.0, 1.0, 1.0), K_CML),      # only noxmiss over its threshold
    ((1.0, 1.3, 1.0), K_MB),       # only inflate
    ((1.0, 1.0, 2.0), K_IMB),      # only balance
    ((1.9, 1.19, 1.49), K_CMP),    # none
    ((2.5, 1.0, 4.0), K_IMB),      # balance is highest and passes
    ((1.9, 1.0, 1.95), K_IMB),     # highest (balance) passes
    ((1.99, 1.0, 1.4), K_CMP),     # highest (noxmiss) fails, others fail
    ((1.9, 1.25, 1.0), K_MB),      # highest fails, second (inflate) passes
])
def test_cascade_branches(scores, klass):
    assert classify(list(scores), THETA) == klass


def test_ties_keep_benchmark_order():
    # equal scores above every threshold: noxmiss first, then inflate, balance
    assert classify([5.0, 5.0, 5.0], THETA) == K_CML
    assert classify([1.0, 5.0, 5.0], THETA) == K_MB
    # tie where the earlier benchmark fails its threshold: next one is tried
    assert classify([1.8, 1.8, 1.8], [2.0, 1.2, 1.5]) == K_MB


def test_class_to_variant_map():
    assert decide_profile_ref(meas(3, 1, 1), FEAT, THETA, ALL) == (V_XBLOCK_LDS, K_CML)
    assert decide_profile_ref(meas(3, 1, 1), FEAT, THETA, ALL & ~(1 << V_XBLOCK_LDS)) == (V_CSR_VECTOR, K_CML)
    assert decide_profile_ref(meas(1, 1.3, 1), FEAT, THETA, ALL) == (V_DELTA16, K_MB)
    assert decide_profile_ref(meas(1, 1.3, 1), FEAT, THETA, ALL & ~(1 << V_DELTA16)) == (V_CSR_VECTOR, K_MB)
    assert decide_profile_ref(meas(1, 1, 2), FEAT, THETA, ALL) == (V_MERGE_PATH, K_IMB)
    assert decide_profile_ref(meas(1, 1, 1), FEAT, THETA, ALL) == (V_CSR_VECTOR, K_CMP)
    assert decide_profile_ref(meas(1, 1, 1), SHORT, THETA, ALL) == (V_SHORT_ROW, K_CMP)


def test_cascade_exhaustive_against_definition():
    """Every ordering of scores above/below thresholds, written out directly."""
    grid = [0.5, 1.1, 1.3, 1.6, 2.5]
    for s in itertools.product(grid, repeat=3):
        order = sorted(range(3), key=lambda b: (-s[b], b))
        want = K_CMP
        for b in order:
            if s[b] > THETA[b]:
                want = [K_CML, K_MB, K_IMB][b]
                break
        assert classify(list(s), THETA) == want
