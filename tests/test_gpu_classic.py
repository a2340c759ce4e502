"""Device inference of the paper's feature classifiers (CART, Gaussian naive
Bayes) against the oracle, and their selectors through spmv_select."""
import json
import math
import os

import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.classic import cart_predict_ref, gnb_fit_ref, gnb_predict_ref
from oracle.mlp import raw_inputs
from oracle.select import class_to_variant, classify, profile_scores
from oracle.spmv import spmv_exact

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import make_plan, run  # noqa: E402

DATA = os.path.join(os.path.dirname(S.__file__), "data")


def records(name, limit=None):
    out = []
    with open(os.path.join(DATA, name)) as f:
        for line in f:
            out.append(json.loads(line))
            if limit and len(out) == limit:
                break
    return out


def as_ref_tree(t):
    return {k: (v.tolist() if k != "threshold" else [float(a) for a in v]) for k, v in t.items()}


@pytest.fixture(scope="module")
def data():
    train, test = records("labels_train.jsonl"), records("labels_test.jsonl", 300)
    X = np.array([r["features"] for r in train])
    y = np.array([r["label"] for r in train])
    theta = S.spmv_get_thresholds()
    yc = np.array([classify(profile_scores(r["meas"]), theta) for r in train])
    return dict(train=train, test=test, X=X, y=y, yc=yc, theta=theta)


@pytest.mark.parametrize("label_kind", [S.SPMV_LABEL_VARIANT, S.SPMV_LABEL_CLASS])
def test_tree_inference_matches_oracle(data, label_kind):
    C = 6 if label_kind == S.SPMV_LABEL_VARIANT else 4
    y = data["y"] if label_kind == S.SPMV_LABEL_VARIANT else data["yc"]
    tree = S.spmv_dtree_fit(data["X"], y, C, 10, 3)
    S.spmv_dtree_load(tree, label_kind)
    ref = as_ref_tree(tree)
    for r in data["test"]:
        feas = r["mask"] if label_kind == S.SPMV_LABEL_VARIANT else 0xF
        k, leaf, fb = cart_predict_ref(ref, r["features"], feas)
        p = S.spmv_classifier_predict(S.SPMV_CLF_DTREE, r["features"], r["mask"])
        assert (p["label"], p["leaf"], p["fallback"]) == (k, leaf, fb), r["name"]
        want = k if label_kind == S.SPMV_LABEL_VARIANT else \
            class_to_variant(k, r["features"], data["theta"], r["mask"])
        assert p["variant"] == want
    S.spmv_classifier_unload(S.SPMV_CLF_DTREE)


@pytest.mark.parametrize("label_kind", [S.SPMV_LABEL_VARIANT, S.SPMV_LABEL_CLASS])
def test_gnb_inference_is_bit_exact(data, label_kind):
    C = 6 if label_kind == S.SPMV_LABEL_VARIANT else 4
    y = data["y"] if label_kind == S.SPMV_LABEL_VARIANT else data["yc"]
    model = S.spmv_gnb_fit(data["X"], y, C)
    S.spmv_gnb_load(model, label_kind)
    ref = gnb_fit_ref(np.array([raw_inputs(f) for f in data["X"]]), y, C)
    for r in data["test"]:
        feas = r["mask"] if label_kind == S.SPMV_LABEL_VARIANT else 0xF
        k, sc, fb = gnb_predict_ref(ref, r["features"], feas)
        p = S.spmv_classifier_predict(S.SPMV_CLF_GNB, r["features"], r["mask"])
        assert (p["label"], p["fallback"]) == (k, fb), r["name"]
        for a, b in zip(p["scores"][:C], sc):
            assert a == b or (math.isinf(a) and math.isinf(b))
    S.spmv_classifier_unload(S.SPMV_CLF_GNB)


CASES = [
    ("stencil27_12", lambda: synth.stencil3d_27(12, seed=3, values="random"), 1728),
    ("random_3000x8", lambda: synth.uniform_random(3000, 5000, 8, seed=4, values="random"), 5000),
    ("powerlaw_20000", lambda: synth.powerlaw(20000, 109, 6000, seed=5, values="random"), 20000),
]


@pytest.mark.parametrize("selector,which", [(S.SEL_DTREE, S.SPMV_CLF_DTREE), (S.SEL_GNB, S.SPMV_CLF_GNB)])
def test_select_with_feature_classifiers(data, selector, which):
    if which == S.SPMV_CLF_DTREE:
        model = S.spmv_dtree_fit(data["X"], data["y"], 6, 10, 3)
        S.spmv_dtree_load(model)
    else:
        model = S.spmv_gnb_fit(data["X"], data["y"], 6)
        S.spmv_gnb_load(model)
    for name, build, m in CASES:
        rp, ci, v = build()
        x = synth.vector(m, 21)
        plan = make_plan(rp, ci, v, m)
        info = plan.select(selector)
        if which == S.SPMV_CLF_DTREE:
            k, _, fb = cart_predict_ref(as_ref_tree(model), info["features"], info["feasible"])
        else:
            ref = gnb_fit_ref(np.array([raw_inputs(f) for f in data["X"]]), data["y"], 6)
            k, _, fb = gnb_predict_ref(ref, info["features"], info["feasible"])
        assert bool(info["fell_back"]) == fb, name
        if not fb:
            assert info["variant"] == k and info["selector"] == selector, name
        y = run(plan, info["variant"], x)
        y_ref, scale = spmv_exact(rp, ci, v, x)
        assert np.all(np.abs(y - y_ref) <= 1e-12 * scale), name
        plan.close()
    S.spmv_classifier_unload(which)
    # without a model the selector falls back to profiling
    rp, ci, v = CASES[0][1]()
    plan = make_plan(rp, ci, v, CASES[0][2])
    info = plan.select(selector)
    assert info["fell_back"] == 1 and info["selector"] == S.SEL_PROFILING
    plan.close()
