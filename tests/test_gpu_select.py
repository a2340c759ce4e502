"""Selectors on the device: profiling decision parity, fallback, exhaustive."""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.encode import delta16_ref
from oracle.features import features_ref
from oracle.select import decide_profile_ref, profile_scores
from oracle.spmv import spmv_exact, within_tolerance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import make_plan, run  # noqa: E402

MATS = [
    ("laplace64", lambda: synth.laplace2d(64), 4096),
    ("powerlaw", lambda: synth.powerlaw(50000, 109, 10000, seed=2), 50000),
    ("random", lambda: synth.uniform_random(50000, 200000, 8, seed=3), 200000),
    ("shortrows", lambda: synth.short_rows(100000, seed=4), 100000),
]


@pytest.mark.parametrize("name,build,m", MATS)
def test_profiling_decision_parity(name, build, m):
    rp, ci, v = build()
    plan = make_plan(rp, ci, v, m)
    info = plan.select(S.SEL_PROFILING)
    theta = S.spmv_get_thresholds()
    want = decide_profile_ref(info["meas"], info["features"], theta, info["feasible"])
    assert (info["variant"], info["klass"]) == want
    assert info["scores"] == profile_scores(info["meas"])
    assert all(t > 0 for t in info["meas"])
    assert plan.variant == info["variant"]
    x = synth.vector(m, 1)
    y = run(plan, info["variant"], x)
    yr, s = spmv_exact(rp, ci, v, x)
    assert within_tolerance(y, yr, s, 1e-12)[0]
    plan.close()


def test_mlp_without_model_falls_back():
    S.spmv_model_unload()
    rp, ci, v = synth.laplace2d(64)
    plan = make_plan(rp, ci, v, 4096)
    info = plan.select(S.SEL_MLP)
    assert info["fell_back"] == 1 and info["selector"] == S.SEL_PROFILING
    assert (info["variant"], info["klass"]) == decide_profile_ref(
        info["meas"], info["features"], S.spmv_get_thresholds(), info["feasible"])
    plan.close()


def test_exhaustive_picks_fastest_feasible():
    rp, ci, v = synth.banded(20000, 256, 64, seed=5)
    plan = make_plan(rp, ci, v, 20000)
    info = plan.select(S.SEL_EXHAUSTIVE)
    t = np.array(info["variant_times_s"])
    feas = info["feasible"]
    for k in range(6):
        assert (t[k] > 0) == bool((feas >> k) & 1)
    cand = [k for k in range(6) if (feas >> k) & 1]
    assert info["variant"] == min(cand, key=lambda k: (t[k], k))
    plan.close()


def test_partition_stamps_balance_score_high_on_long_row():
    rp, ci, v = synth.powerlaw(200000, 109, 100000, seed=6)
    plan = make_plan(rp, ci, v, 200000)
    meas = S.spmv_profile_measure(plan.handle, 3)
    assert meas[3] / meas[4] > 2.0
    plan.close()


def test_mlp_low_margin_falls_back_to_the_cascade(tmp_path):
    """A model whose margin threshold no prediction reaches: every SEL_MLP
    selection defers to the profiling cascade, which then decides exactly as
    the oracle's cascade on the measured times; a threshold of 0 keeps the
    MLP's own pick.  Same network both times, so only tau differs."""
    import os
    from paper_1511_02494_amd.model_io import read_model, write_model
    if not os.path.exists(S.DEFAULT_MODEL):
        pytest.skip("no trained model")
    params, mu, rho, _ = read_model(S.DEFAULT_MODEL)
    strict = str(tmp_path / "strict.bin")
    write_model(strict, params, mu, rho, 1e30)
    rp, ci, v = synth.powerlaw(50000, 109, 10000, seed=2)
    for path, expect_fb in ((strict, True), (S.DEFAULT_MODEL, None)):
        S.spmv_model_load(path)
        plan = make_plan(rp, ci, v, 50000)
        info = plan.select(S.SEL_MLP)
        pred = S.spmv_mlp_predict(info["features"], info["feasible"])
        if expect_fb:
            assert info["fell_back"] == 1 and info["selector"] == S.SEL_PROFILING
            assert (info["variant"], info["klass"]) == decide_profile_ref(
                info["meas"], info["features"], S.spmv_get_thresholds(), info["feasible"])
        else:
            assert bool(info["fell_back"]) == bool(pred["fallback"])
            if not pred["fallback"]:
                assert info["variant"] == pred["variant"] and info["selector"] == S.SEL_MLP
        plan.close()
    S.spmv_model_load(S.DEFAULT_MODEL)


def strided_rows(n, stride, seed):
    """Two nonzeros per row at columns stride * i and stride * i + 50: a
    block of 256 rows spans 255 stride + 50 columns, a block of 1024 rows
    four times as many."""
    rng = np.random.default_rng(seed)
    rp = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
    ci = np.empty(2 * n, np.int32)
    ci[0::2] = stride * np.arange(n)
    ci[1::2] = stride * np.arange(n) + 50
    return rp, ci, rng.uniform(-1, 1, 2 * n), stride * n


ONEPASS = MATS + [
    ("laplace256", lambda: synth.laplace2d(256), 65536),
    ("strided", lambda: strided_rows(20000, 200, 7)[:3], 4_000_000),
]


def _class_label_models():
    """A tree and naive Bayes on the training records' cascade classes (the
    paper's labelling), installed with class labels."""
    import json
    import os
    from oracle.select import classify, profile_scores
    path = os.path.join(os.path.dirname(S.__file__), "data", "labels_train.jsonl")
    with open(path) as f:
        recs = [json.loads(line) for line in f]
    X = np.array([r["features"] for r in recs])
    theta = S.spmv_get_thresholds()
    yc = np.array([classify(profile_scores(r["meas"]), theta) for r in recs])
    S.spmv_dtree_load(S.spmv_dtree_fit(X, yc, 4, 6, 5), S.SPMV_LABEL_CLASS)
    S.spmv_gnb_load(S.spmv_gnb_fit(X, yc, 4), S.SPMV_LABEL_CLASS)


@pytest.mark.parametrize("labels", ["variant", "class"])
@pytest.mark.parametrize("sel", [S.SEL_DTREE, S.SEL_GNB])
@pytest.mark.parametrize("name,build,m", ONEPASS[:2] + ONEPASS[4:])
def test_classifier_one_pass_matches_two_step(name, build, m, sel, labels):
    """SEL_DTREE / SEL_GNB on a fresh plan (one pass: the classifier runs on
    the device features) and on a plan whose features were already taken
    (step by step) pick the same variant from the same features and
    feasibility, with variant labels and with the cascade's class labels
    (mapped to a variant through Table 2 on the host)."""
    if labels == "variant":
        if "dtree" not in S.load_classifiers() or "gnb" not in S.load_classifiers():
            pytest.skip("no stored classifiers")
    else:
        _class_label_models()
    rp, ci, v = build()
    a = make_plan(rp, ci, v, m)
    b = make_plan(rp, ci, v, m)
    b.features()
    ia, ib = a.select(sel), b.select(sel)
    f_ref, _ = features_ref(rp, ci, m)
    assert list(ia["features"]) == f_ref == list(ib["features"])
    assert ia["feasible"] == ib["feasible"] == a.mask()
    assert ia["fell_back"] == ib["fell_back"]
    if not ia["fell_back"]:
        assert ia["variant"] == ib["variant"]
        assert (ia["feasible"] >> ia["variant"]) & 1
    assert (a.query(11), a.query(9)) == (b.query(11), b.query(9))
    a.close()
    b.close()
    if labels == "class":
        S.load_classifiers()  # the stored variant-label models back


@pytest.mark.parametrize("name,build,m", ONEPASS)
def test_mlp_one_pass_matches_two_step(name, build, m):
    """SEL_MLP on a fresh plan runs features, the delta16 span test, the
    device finalisation of the features and the network in one pass; on a
    plan whose features were already taken it runs them step by step.  Both
    give the same features (bit for bit the oracle's), feasibility, delta16
    block height and base columns, logits, margin and (unless the margin sent
    it to the timed cascade) variant."""
    import os
    if not os.path.exists(S.DEFAULT_MODEL):
        pytest.skip("no trained model")
    S.spmv_model_load(S.DEFAULT_MODEL)
    rp, ci, v = build()
    a = make_plan(rp, ci, v, m)
    b = make_plan(rp, ci, v, m)
    b.features()
    ia, ib = a.select(S.SEL_MLP), b.select(S.SEL_MLP)
    f_ref, _ = features_ref(rp, ci, m)
    assert list(ia["features"]) == f_ref == list(ib["features"])
    assert a.features() == b.features()
    assert ia["feasible"] == ib["feasible"] == a.mask()
    assert list(ia["logits"]) == list(ib["logits"]) and ia["margin"] == ib["margin"]
    assert ia["fell_back"] == ib["fell_back"]
    if not ia["fell_back"]:
        assert ia["variant"] == ib["variant"]
    H, ok = a.query(11), a.query(9)
    assert (H, ok) == (b.query(11), b.query(9))
    ok_ref, base, _ = delta16_ref(rp, ci, H)
    assert ok == int(ok_ref)
    if name == "strided":  # the 1024-row blocks are too wide: the 256-row base is kept
        assert (H, ok) == (256, 1) and not delta16_ref(rp, ci, 1024)[0]
    if ok:
        S.spmv_set_delta16_layout(a.handle, 0)
        assert np.array_equal(S.spmv_plan_copy_format(a.handle, 0, len(base)), base)
        x = synth.vector(m, 3)
        y = run(a, S.V_DELTA16, x)
        yr, sc = spmv_exact(rp, ci, v, x)
        assert within_tolerance(y, yr, sc, 1e-12)[0]
    a.close()
    b.close()
