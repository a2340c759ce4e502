"""Selectors on the device: profiling decision parity, fallback, exhaustive."""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
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
