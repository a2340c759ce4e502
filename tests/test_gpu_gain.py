"""What the learned selectors gain over the method without them, on the 500
held-out matrices whose every variant was timed (data/labels_test.jsonl):
device inference of the installed models against the profiling cascade's
picks from the same records, scored by the recorded times."""
import json
import os
import time

import numpy as np
import pytest

import paper_1511_02494_amd as S

pytestmark = pytest.mark.gpu

DATA = os.path.join(os.path.dirname(S.__file__), "data", "labels_test.jsonl")


def records():
    with open(DATA) as f:
        return [json.loads(line) for line in f]


def score(recs, pick):
    hit, reg = [], []
    for r in recs:
        t = r["times"]
        best = min(x for x in t if x > 0)
        v = pick(r)
        hit.append(t[v] <= 1.05 * best)
        reg.append(t[v] / best - 1)
    return float(np.mean(hit)), float(np.mean(reg))


def profiling(r, theta):
    return S.spmv_profile_decide(r["meas"], r["features"], theta, r["mask"])[0]


def test_mlp_gain_over_profiling_cascade():
    if not os.path.exists(S.DEFAULT_MODEL):
        pytest.skip("no trained model")
    recs = records()
    theta = S.spmv_get_thresholds()
    S.spmv_model_load(S.DEFAULT_MODEL)

    def mlp(r):
        p = S.spmv_mlp_predict(r["features"], r["mask"])
        return profiling(r, theta) if p["fallback"] else p["variant"]
    try:
        hit_m, reg_m = score(recs, mlp)
        t0 = time.perf_counter()
        for _ in range(50):
            S.spmv_mlp_predict(recs[0]["features"], recs[0]["mask"])
        t_inf = (time.perf_counter() - t0) / 50
    finally:
        S.spmv_model_unload()
    hit_p, reg_p = score(recs, lambda r: profiling(r, theta))
    hit_v, _ = score(recs, lambda r: S.V_CSR_VECTOR)
    over = [(r["t_select"] if "t_select" in r else r["t_features"] + t_inf)
            / min(x for x in r["times"] if x > 0) for r in recs]
    print(f"\nheld-out: MLP {hit_m:.3f} within 5% (regret {reg_m:.3f}); profiling {hit_p:.3f} "
          f"({reg_p:.3f}); always csr_vector {hit_v:.3f}; median selection cost "
          f"{np.median(over):.1f} SpMVs of the fastest variant", flush=True)
    assert hit_m >= 0.90                      # the learned selector's target
    assert hit_m > hit_p + 0.2 and reg_m < reg_p
    assert np.median(over) <= 20


def test_cart_gain_over_profiling_cascade():
    if not os.path.exists(S.DTREE_MODEL):
        pytest.skip("no stored tree")
    assert "dtree" in S.load_classifiers()
    recs = records()
    theta = S.spmv_get_thresholds()

    def tree(r):
        p = S.spmv_classifier_predict(S.SPMV_CLF_DTREE, r["features"], r["mask"])
        return profiling(r, theta) if p["fallback"] else p["variant"]
    try:
        hit_t, reg_t = score(recs, tree)
    finally:
        S.spmv_classifier_unload(S.SPMV_CLF_DTREE)
        S.spmv_classifier_unload(S.SPMV_CLF_GNB)
    hit_p, reg_p = score(recs, lambda r: profiling(r, theta))
    print(f"\nheld-out: CART {hit_t:.3f} within 5% (regret {reg_t:.3f}); profiling {hit_p:.3f}", flush=True)
    assert hit_t >= 0.85 and hit_t > hit_p and reg_t < reg_p
