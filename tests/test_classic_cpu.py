"""The library's CART and naive Bayes fitting (host code, no GPU) against the
oracle: identical trees and bit-equal naive Bayes parameters."""
import json
import os

import numpy as np
import pytest

import paper_1511_02494_amd as S
from oracle.classic import cart_fit_ref, gnb_fit_ref
from oracle.mlp import raw_inputs

DATA = os.path.join(os.path.dirname(S.__file__), "data")


def real_labels(name, limit):
    X, y = [], []
    with open(os.path.join(DATA, name)) as f:
        for line in f:
            r = json.loads(line)
            X.append(r["features"])
            y.append(r["label"])
            if len(y) == limit:
                break
    return np.array(X), np.array(y)


def random_set(seed, n=300, C=6):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 12)) * 10
    X[:, 3] = np.round(X[:, 3])        # many ties
    X[:, 7] = 1.0                      # constant feature
    y = np.digitize(X[:, 0] + 0.5 * X[:, 3] + rng.normal(size=n) * 5, [-15, -5, 0, 5, 15])
    return X, np.minimum(y, C - 1)


def same_tree(lib, ref):
    assert lib["feature"].tolist() == ref["feature"]
    assert lib["left"].tolist() == ref["left"]
    assert lib["right"].tolist() == ref["right"]
    assert lib["counts"].tolist() == ref["counts"]
    assert np.array_equal(lib["threshold"], np.array(ref["threshold"]))


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("depth,leaf", [(1, 1), (4, 1), (8, 5), (30, 1)])
def test_tree_fit_matches_oracle_on_random_data(seed, depth, leaf):
    X, y = random_set(seed)
    same_tree(S.spmv_dtree_fit(X, y, 6, depth, leaf), cart_fit_ref(X, y, 6, depth, leaf))


def test_tree_fit_matches_oracle_on_labels():
    X, y = real_labels("labels_train.jsonl", 400)
    same_tree(S.spmv_dtree_fit(X, y, 6, 10, 3), cart_fit_ref(X, y, 6, 10, 3))


@pytest.mark.parametrize("seed", range(3))
def test_gnb_fit_is_bit_equal_to_oracle(seed):
    X, y = random_set(seed)
    X = np.abs(X)
    lib = S.spmv_gnb_fit(X, y, 6)
    ref = gnb_fit_ref(np.array([raw_inputs(f) for f in X]), y, 6)
    assert lib["count"].tolist() == ref["count"]
    assert np.array_equal(lib["mu"], np.array(ref["mu"]))
    assert np.array_equal(lib["w"], np.array(ref["w"]))
    assert np.array_equal(lib["c"], np.array(ref["c"]))


def test_gnb_fit_on_labels_with_an_empty_class():
    X, y = real_labels("labels_test.jsonl", 300)
    y = np.where(y == 2, 0, y)           # class 2 has no sample
    lib = S.spmv_gnb_fit(X, y, 6)
    ref = gnb_fit_ref(np.array([raw_inputs(f) for f in X]), y, 6)
    assert lib["count"][2] == 0
    for k in ("mu", "w", "c"):
        assert np.array_equal(lib[k], np.array(ref[k]))


def test_fit_and_load_argument_errors():
    X, y = random_set(0, n=50)
    for args in [(X, np.full(50, 6), 6, 3, 1), (X, y, 6, 65, 1), (X, y, 6, 3, 0), (X, y, 9, 3, 1)]:
        with pytest.raises(S.SpmvError) as e:
            S.spmv_dtree_fit(*args)
        assert e.value.status == S.SPMV_ERR_ARG
    with pytest.raises(S.SpmvError):
        S.spmv_dtree_fit(X, y, 6, 30, 1, max_nodes=3)          # tree too big
    t = S.spmv_dtree_fit(X, y, 6, 3, 1)
    bad = {k: v.copy() for k, v in t.items()}
    if (bad["feature"] >= 0).any():
        i = int(np.nonzero(bad["feature"] >= 0)[0][0])
        bad["left"][i] = i                                       # a cycle
        with pytest.raises(S.SpmvError) as e:
            S.spmv_dtree_load(bad)
        assert e.value.status == S.SPMV_ERR_ARG
    with pytest.raises(S.SpmvError):
        S.spmv_dtree_load(t, S.SPMV_LABEL_CLASS)                 # 6 classes, class labels
    S.spmv_dtree_load(t)
    S.spmv_classifier_unload(S.SPMV_CLF_DTREE)
    with pytest.raises(S.SpmvError):
        S.spmv_gnb_fit(X, y, 0)
