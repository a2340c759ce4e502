"""Pins of the CART and Gaussian naive Bayes oracles (oracle/classic.py)
against brute force, closed forms and library routines."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import norm

from oracle.classic import (cart_fit_ref, cart_predict_ref, gnb_fit_ref, gnb_predict_ref,
                            gnb_scores_ref, split_threshold)
from oracle.mlp import raw_inputs


def gini_weighted(labels_l, labels_r, n_classes):
    """n_L * Gini_L + n_R * Gini_R as an exact fraction (textbook formula)."""
    out = Fraction(0)
    for part in (labels_l, labels_r):
        n = len(part)
        if n == 0:
            continue
        g = Fraction(1) - sum(Fraction(sum(1 for v in part if v == k), n) ** 2
                              for k in range(n_classes))
        out += n * g
    return out


def brute_root_split(X, y, n_classes, min_leaf):
    best = None
    for j in range(X.shape[1]):
        vals = sorted(set(X[:, j].tolist()))
        for a, b in zip(vals, vals[1:]):
            t = split_threshold(a, b)
            L = [y[i] for i in range(len(y)) if X[i, j] <= t]
            R = [y[i] for i in range(len(y)) if X[i, j] > t]
            if len(L) < min_leaf or len(R) < min_leaf:
                continue
            imp = gini_weighted(L, R, n_classes)
            if best is None or imp < best[0]:
                best = (imp, j, t)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_root_split_is_the_brute_force_gini_minimum(seed):
    rng = np.random.default_rng(seed)
    n, d, C = 14, 3, 3
    X = rng.integers(0, 6, size=(n, d)).astype(np.float64) * 0.5
    y = rng.integers(0, C, size=n)
    for min_leaf in (1, 3):
        tree = cart_fit_ref(X, y, C, max_depth=1, min_leaf=min_leaf)
        best = brute_root_split(X, y, C, min_leaf)
        parent = gini_weighted(list(y), [], C)
        if best is None or not best[0] < parent:
            assert tree["feature"][0] == -1
        else:
            assert (tree["feature"][0], tree["threshold"][0]) == (best[1], best[2])


def test_separable_data_fits_exactly_with_pure_leaves():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(200, 4))
    y = (X[:, 0] > 0.3).astype(int) + 2 * (X[:, 2] > -0.5).astype(int)
    tree = cart_fit_ref(X, y, 4, max_depth=20, min_leaf=1)
    for i in range(len(y)):
        k, leaf, fb = cart_predict_ref(tree, X[i], 0b1111)
        assert k == y[i] and not fb
        assert sum(1 for v in tree["counts"][leaf] if v) == 1


def test_xor_greedy_root_and_depth_two():
    X = np.array([[0, 0], [0, 1], [1, 0], [1, 1]] * 5, dtype=np.float64)
    y = np.array([0, 1, 1, 0] * 5)
    # balanced XOR: no single split lowers the Gini impurity, so greedy CART
    # keeps the root as a leaf at any depth
    assert cart_fit_ref(X, y, 2, max_depth=5, min_leaf=1)["feature"] == [-1]
    # one more (0, 0) sample breaks the tie; two levels then separate XOR
    X2 = np.vstack([X, [[0, 0]]])
    y2 = np.append(y, 0)
    deep = cart_fit_ref(X2, y2, 2, max_depth=2, min_leaf=1)
    assert all(cart_predict_ref(deep, X2[i], 3)[0] == y2[i] for i in range(len(y2)))
    assert cart_fit_ref(X2, y2, 2, max_depth=1, min_leaf=1)["feature"][0] == 0


def test_depth_leaf_size_and_counts_are_respected():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(150, 5))
    y = rng.integers(0, 6, size=150)
    tree = cart_fit_ref(X, y, 6, max_depth=4, min_leaf=7)

    def walk(node, depth):
        assert depth <= 4
        if tree["feature"][node] < 0:
            assert sum(tree["counts"][node]) >= 7
            return
        l, r = tree["left"][node], tree["right"][node]
        assert l == node + 1  # pre-order
        assert [a + b for a, b in zip(tree["counts"][l], tree["counts"][r])] == tree["counts"][node]
        walk(l, depth + 1)
        walk(r, depth + 1)
    walk(0, 0)
    assert tree["counts"][0] == np.bincount(y, minlength=6).tolist()


def test_monotone_feature_transform_keeps_the_partition():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 40, size=(120, 3)).astype(np.float64)
    y = rng.integers(0, 3, size=120)
    t1 = cart_fit_ref(X, y, 3, max_depth=6, min_leaf=2)
    t2 = cart_fit_ref(3 * X + 1, y, 3, max_depth=6, min_leaf=2)
    assert t1["feature"] == t2["feature"] and t1["counts"] == t2["counts"]
    assert [cart_predict_ref(t1, X[i], 7)[1] for i in range(120)] == \
        [cart_predict_ref(t2, 3 * X[i] + 1, 7)[1] for i in range(120)]


def test_predict_masks_infeasible_classes_and_falls_back():
    tree = dict(feature=[-1], threshold=[0.0], left=[-1], right=[-1], counts=[[0, 5, 5, 2]])
    assert cart_predict_ref(tree, [0.0], 0b1111) == (1, 0, False)   # tie -> lower index
    assert cart_predict_ref(tree, [0.0], 0b1101) == (2, 0, False)
    assert cart_predict_ref(tree, [0.0], 0b0001)[2] is True


def test_threshold_between_adjacent_values():
    a = 1.0
    b = np.nextafter(1.0, 2.0)
    t = split_threshold(a, b)
    assert a <= t < b
    assert split_threshold(2.0, 4.0) == 3.0


# ---------------------------------------------------------------- Gaussian NB
def _features_like(rng, n):
    f = np.zeros((n, 12))
    f[:, 0] = rng.integers(1e4, 4e6, n)
    f[:, 1] = f[:, 0] * rng.uniform(1, 64, n)
    f[:, 2:10] = rng.uniform(0, 50, (n, 8))
    f[:, 10] = rng.uniform(0, 1, n)
    f[:, 11] = rng.integers(0, 2, n)
    return f


def test_gnb_scores_equal_log_prior_plus_normal_log_densities():
    rng = np.random.default_rng(4)
    F = _features_like(rng, 300)
    y = rng.integers(0, 6, 300)
    G = np.array([raw_inputs(f) for f in F])
    model = gnb_fit_ref(G, y, 6)
    for i in range(0, 300, 37):
        s = gnb_scores_ref(model, G[i])
        for k in range(6):
            rows = G[y == k]
            eps = 1e-9 * np.var(G, axis=0).max()
            var = rows.var(axis=0) + eps
            ref = math.log(len(rows) / 300) + norm.logpdf(G[i], rows.mean(axis=0), np.sqrt(var)).sum()
            assert s[k] == pytest.approx(ref, rel=1e-10, abs=1e-9)


def test_gnb_separated_classes_and_priors():
    rng = np.random.default_rng(5)
    F = _features_like(rng, 400)
    y = (F[:, 2] > 25).astype(int) * 3          # classes 0 and 3 only
    G = np.array([raw_inputs(f) for f in F])
    model = gnb_fit_ref(G, y, 6)
    assert model["count"] == [int((y == k).sum()) for k in range(6)]
    acc = np.mean([gnb_predict_ref(model, F[i], 63)[0] == y[i] for i in range(400)])
    assert acc > 0.9
    # classes without samples are never chosen; no feasible class: fallback
    assert all(gnb_predict_ref(model, F[i], 0b111110)[0] == 3 for i in range(20))
    k, _, fb = gnb_predict_ref(model, F[0], 0b000110)
    assert fb and k == 0
    # identical class distributions: the larger prior wins
    G2 = np.vstack([G[:50], G[:50], G[:50]])
    y2 = np.array([1] * 100 + [2] * 50)
    m2 = gnb_fit_ref(G2, y2, 6)
    assert gnb_predict_ref(m2, F[3], 63)[0] == 1


def test_gnb_constant_feature_is_smoothed():
    rng = np.random.default_rng(6)
    F = _features_like(rng, 60)
    F[:, 11] = 1.0   # zero variance everywhere
    y = rng.integers(0, 2, 60)
    G = np.array([raw_inputs(f) for f in F])
    model = gnb_fit_ref(G, y, 2)
    assert all(math.isfinite(v) for row in model["w"] for v in row)
    assert all(math.isfinite(v) for v in gnb_scores_ref(model, G[0]))


def test_gnb_mean_and_variance_match_numpy():
    rng = np.random.default_rng(7)
    G = rng.normal(size=(90, 12)) * 3 + 1
    y = rng.integers(0, 3, 90)
    model = gnb_fit_ref(G, y, 3)
    eps = 1e-9 * G.var(axis=0).max()
    for k in range(3):
        rows = G[y == k]
        assert np.allclose(model["mu"][k], rows.mean(axis=0), rtol=1e-13, atol=0)
        assert np.allclose(0.5 / np.array(model["w"][k]), rows.var(axis=0) + eps, rtol=1e-12, atol=0)
        assert model["c"][k] == pytest.approx(
            math.log(len(rows) / 90) - 0.5 * np.log(2 * math.pi * (rows.var(axis=0) + eps)).sum(),
            rel=1e-12)


def test_cart_leave_one_out_brute_force_tiny():
    """LOOCV by its definition on a tiny set: every fold refits without one sample."""
    rng = np.random.default_rng(8)
    X = rng.integers(0, 5, size=(16, 2)).astype(np.float64)
    y = (X[:, 0] + X[:, 1] > 4).astype(int)
    hits = 0
    for i in range(16):
        keep = [j for j in range(16) if j != i]
        t = cart_fit_ref(X[keep], y[keep], 2, max_depth=3, min_leaf=1)
        hits += cart_predict_ref(t, X[i], 3)[0] == y[i]
    assert hits >= 12


@pytest.mark.parametrize("seed", range(4))
def test_cart_agrees_with_scikit_learn(seed):
    """scikit-learn's CART (Gini, best splits, mid-point thresholds) on data
    where every split strictly improves and no two candidates tie."""
    tree_mod = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(100 + seed)
    X = rng.normal(size=(400, 5))
    y = ((X[:, 0] + 0.5 * X[:, 1] ** 2 + 0.3 * rng.normal(size=400)) > 0.4).astype(int) \
        + (X[:, 3] > 0.8).astype(int)
    ours = cart_fit_ref(X, y, 3, max_depth=4, min_leaf=10)
    sk = tree_mod.DecisionTreeClassifier(max_depth=4, min_samples_leaf=10, random_state=0).fit(X, y)
    T = rng.normal(size=(300, 5))
    a = [cart_predict_ref(ours, T[i], 7)[0] for i in range(300)]
    assert a == sk.predict(T).tolist()
    assert sum(1 for f in ours["feature"] if f >= 0) == int((sk.tree_.feature >= 0).sum())


def test_gnb_agrees_with_scikit_learn():
    nb = pytest.importorskip("sklearn.naive_bayes")
    rng = np.random.default_rng(9)
    F = _features_like(rng, 500)
    y = np.digitize(F[:, 2] + 10 * F[:, 10], [15, 30, 45])   # 4 classes
    G = np.array([raw_inputs(f) for f in F])
    model = gnb_fit_ref(G, y, 4)
    sk = nb.GaussianNB().fit(G, y)
    T = _features_like(rng, 200)
    ours = [gnb_predict_ref(model, T[i], 15)[0] for i in range(200)]
    assert ours == sk.predict(np.array([raw_inputs(f) for f in T])).tolist()
    jl = sk.predict_joint_log_proba(np.array([raw_inputs(T[0])]))[0]
    assert np.allclose(gnb_scores_ref(model, raw_inputs(T[0])), jl, rtol=1e-10)
