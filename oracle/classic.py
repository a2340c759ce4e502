"""The paper's feature classifiers: a CART decision tree and Gaussian naive
Bayes (test infrastructure; written from the definitions, slow and plain).

Section 3.2.2 trains a decision tree and a Gaussian naive Bayes classifier
on the structural features (Table 1) and scores them by leave-one-out
cross-validation (Tables 4 and 5).  The paper gives no hyper-parameters or
tie rules; the readings fixed here are:

CART (Breiman, Friedman, Olshen, Stone 1984), Gini criterion.
* A node splits its samples on (feature j, threshold t): left x_j <= t,
  right x_j > t.  Candidate thresholds lie between consecutive distinct
  values a < b of feature j in the node: t = a/2 + b/2, or a if that
  rounding does not fall in [a, b).  Each child keeps at least ``min_leaf``
  samples.
* Minimising the weighted Gini impurity n_L G_L + n_R G_R equals maximising
  Q = sum_k cL_k^2 / n_L + sum_k cR_k^2 / n_R (class counts c); Q is
  compared exactly as a fraction of integers.  A split is taken only if Q
  exceeds the parent's sum_k c_k^2 / n (strictly lower impurity).  The best
  split is the largest Q; ties keep the first in scan order (features
  ascending, thresholds ascending).
* A node is a leaf at depth ``max_depth`` (root depth 0), when it is pure,
  when it has fewer than 2 min_leaf samples, or when no split qualifies.
* Nodes are numbered in pre-order (node, left subtree, right subtree);
  every node stores its class counts.
* Prediction walks from the root; at the leaf it returns the feasible class
  with the largest count (lowest index on ties) and reports ``fallback``
  when no feasible class has a positive count.

Gaussian naive Bayes, on g = the exact-op transform of the features used by
the MLP (plog2(1 + f_k) for k < 8, f_k otherwise).
* Per class k with n_k > 0 samples: mu_kj = (sum_i g_ij) / n_k and
  var_kj = (sum_i (g_ij - mu_kj)^2) / n_k, sums taken in sample order, plus
  eps = 1e-9 * max_j (population variance of feature j over all samples) to
  every var_kj (the smoothing scikit-learn applies by default; the paper used
  that library).  Prior pi_k = n_k / n.
* Stored per class: w_kj = 0.5 / var_kj and
  c_k = log(pi_k) - 0.5 * sum_j log(2 pi var_kj).
* Score s_k(g) = c_k - sum_j w_kj * ((g_j - mu_kj)^2), summed over j in
  order with every operation rounded separately; the decision is the
  feasible class with n_k > 0 and the largest score (lowest index on ties),
  with ``fallback`` when there is none.
"""
from __future__ import annotations

import math

import numpy as np

from .mlp import raw_inputs


# ---------------------------------------------------------------- CART
def _q_gt(a1: int, nl1: int, b1: int, nr1: int, a2: int, nl2: int, b2: int, nr2: int) -> bool:
    """a1/nl1 + b1/nr1 > a2/nl2 + b2/nr2, exactly (all positive integers)."""
    return (a1 * nr1 + b1 * nl1) * (nl2 * nr2) > (a2 * nr2 + b2 * nl2) * (nl1 * nr1)


def split_threshold(a: float, b: float) -> float:
    t = a / 2.0 + b / 2.0
    return t if a <= t < b else a


def cart_fit_ref(X, y, n_classes: int, max_depth: int, min_leaf: int):
    """Returns dict(feature, threshold, left, right, counts) as lists (pre-order)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    d = X.shape[1]
    feature, threshold, left, right, counts = [], [], [], [], []

    def build(idx, depth):
        node = len(feature)
        c = np.bincount(y[idx], minlength=n_classes)
        feature.append(-1)
        threshold.append(0.0)
        left.append(-1)
        right.append(-1)
        counts.append([int(v) for v in c])
        n = len(idx)
        if depth >= max_depth or n < 2 * min_leaf or np.count_nonzero(c) <= 1:
            return node
        sq = int(np.sum(c.astype(object) ** 2))
        best = None  # (A, nL, B, nR, j, t)
        for j in range(d):
            order = sorted(idx, key=lambda i: (X[i, j], i))
            vals = [X[i, j] for i in order]
            cl = [0] * n_classes
            cr = [int(v) for v in c]
            for p in range(n - 1):
                k = int(y[order[p]])
                cl[k] += 1
                cr[k] -= 1
                if vals[p] == vals[p + 1]:
                    continue
                nl, nr = p + 1, n - p - 1
                if nl < min_leaf or nr < min_leaf:
                    continue
                A = sum(v * v for v in cl)
                B = sum(v * v for v in cr)
                if best is None or _q_gt(A, nl, B, nr, best[0], best[1], best[2], best[3]):
                    best = (A, nl, B, nr, j, split_threshold(vals[p], vals[p + 1]))
        if best is None:
            return node
        A, nl, B, nr, j, t = best
        if not (A * nr + B * nl) * n > sq * nl * nr:  # impurity must drop
            return node
        li = [i for i in idx if X[i, j] <= t]
        ri = [i for i in idx if X[i, j] > t]
        feature[node] = j
        threshold[node] = t
        left[node] = build(li, depth + 1)
        right[node] = build(ri, depth + 1)
        return node

    build(list(range(len(y))), 0)
    return dict(feature=feature, threshold=threshold, left=left, right=right, counts=counts)


def cart_predict_ref(tree, x, feasible_bits: int):
    """(class, leaf, fallback) for one feature vector."""
    node = 0
    while tree["feature"][node] >= 0:
        j = tree["feature"][node]
        node = tree["left"][node] if float(x[j]) <= tree["threshold"][node] else tree["right"][node]
    best, bc = -1, 0
    for k, v in enumerate(tree["counts"][node]):
        if (feasible_bits >> k) & 1 and v > bc:
            best, bc = k, v
    if best < 0:
        return 0, node, True
    return best, node, False


# ---------------------------------------------------------------- Gaussian NB
def gnb_fit_ref(G, y, n_classes: int):
    """dict(mu[C][12], w[C][12], c[C], count[C]) from transformed inputs G."""
    G = [[float(v) for v in row] for row in np.asarray(G, dtype=np.float64)]
    y = [int(v) for v in y]
    n, d = len(G), len(G[0])
    # smoothing from the population variance of each feature over all samples
    vmax = 0.0
    for j in range(d):
        s = 0.0
        for i in range(n):
            s = s + G[i][j]
        m = s / n
        q = 0.0
        for i in range(n):
            t = G[i][j] - m
            q = q + t * t
        vmax = max(vmax, q / n)
    eps = 1e-9 * vmax
    mu = [[0.0] * d for _ in range(n_classes)]
    w = [[0.0] * d for _ in range(n_classes)]
    c = [0.0] * n_classes
    count = [0] * n_classes
    for k in range(n_classes):
        rows = [i for i in range(n) if y[i] == k]
        count[k] = len(rows)
        if not rows:
            continue
        logvar = 0.0
        for j in range(d):
            s = 0.0
            for i in rows:
                s = s + G[i][j]
            m = s / len(rows)
            q = 0.0
            for i in rows:
                t = G[i][j] - m
                q = q + t * t
            var = q / len(rows) + eps
            mu[k][j] = m
            w[k][j] = 0.5 / var
            logvar = logvar + math.log(2.0 * math.pi * var)
        c[k] = math.log(len(rows) / n) - 0.5 * logvar
    return dict(mu=mu, w=w, c=c, count=count)


def gnb_scores_ref(model, g):
    """s_k for every class (-inf for classes without samples)."""
    out = []
    for k in range(len(model["c"])):
        if model["count"][k] == 0:
            out.append(-math.inf)
            continue
        s = 0.0
        for j in range(len(g)):
            dlt = float(g[j]) - model["mu"][k][j]
            s = s + model["w"][k][j] * (dlt * dlt)
        out.append(model["c"][k] - s)
    return out


def gnb_predict_ref(model, features, feasible_bits: int):
    """(class, scores, fallback) from the twelve raw features."""
    s = gnb_scores_ref(model, raw_inputs(features))
    best = -1
    for k, v in enumerate(s):
        if (feasible_bits >> k) & 1 and model["count"][k] > 0 and (best < 0 or v > s[best]):
            best = k
    if best < 0:
        return 0, s, True
    return best, s, False
