"""Learned selector: a 12 -> 64 -> 64 -> 6 MLP (test infrastructure).

The paper's feature-based classifier is a decision tree or Gaussian naive
Bayes over the Table 1 features (Section 3.2.2); this build's learned
selector is a small MLP over the same kind of features that predicts the
fastest variant directly.  The oracle fixes:

* the input transform, made of exactly rounded operations only:
  g_k = plog2(1 + f_k) for k < 8 and g_k = f_k otherwise, where
  plog2(v) = (e - 1) + (2m - 1) with (m, e) = frexp(v) (a piecewise-linear
  log2); z_k = fl32(fl32(fl32(g_k) - mu_k) * rho_k);
* the FP32 forward pass with a fixed order: acc = 0; for k in order
  acc = fl32(acc + fl32(W[j,k] * in[k])); out = fl32(acc + b[j]);
  relu(v) = v if v > 0 else +0;
* the decision: infeasible logits are skipped, the first maximal logit
  wins, margin = fl32(top1 - top2) (+inf with a single feasible variant),
  and the selector falls back when margin < tau or any |z_k| > 8;
* FP64 mean softmax cross-entropy with its gradients, and one Adam step
  (Kingma and Ba 2015).

Parameters are one flat vector: W1[64,12], b1[64], W2[64,64], b2[64],
W3[6,64], b3[6] (row-major, output index first) — 5382 values.
"""
from __future__ import annotations

import math

import numpy as np

DIMS = (12, 64, 64, 6)
Z_LIMIT = 8.0


def layout():
    """[(name, shape, offset)] of the flat parameter vector."""
    out, off = [], 0
    for li in range(3):
        fi, fo = DIMS[li], DIMS[li + 1]
        out.append((f"W{li + 1}", (fo, fi), off))
        off += fo * fi
        out.append((f"b{li + 1}", (fo,), off))
        off += fo
    return out, off


LAYOUT, N_PARAMS = layout()


def unpack(p):
    return {name: np.asarray(p[off:off + int(np.prod(shape))]).reshape(shape)
            for name, shape, off in LAYOUT}


def plog2(v: float) -> float:
    m, e = math.frexp(v)
    return float(e - 1) + (2.0 * m - 1.0)


def transform(features, mu, rho) -> np.ndarray:
    """z (float32[12]) from the twelve FP64 features."""
    z = np.zeros(12, dtype=np.float32)
    for k in range(12):
        f = float(features[k])
        g = plog2(1.0 + f) if k < 8 else f
        t = np.float32(np.float32(g) - np.float32(mu[k]))
        z[k] = np.float32(t * np.float32(rho[k]))
    return z


def raw_inputs(features) -> np.ndarray:
    """g (float64[12]) before normalisation, for computing mu and rho."""
    return np.array([plog2(1.0 + float(features[k])) if k < 8 else float(features[k])
                     for k in range(12)], dtype=np.float64)


def _dense_f32(W, b, inp, relu):
    out = np.zeros(W.shape[0], dtype=np.float32)
    for j in range(W.shape[0]):
        acc = np.float32(0.0)
        for k in range(W.shape[1]):
            acc = np.float32(acc + np.float32(W[j, k] * inp[k]))
        v = np.float32(acc + b[j])
        out[j] = v if (not relu or v > 0) else np.float32(0.0)
    return out


def forward_f32(params, z) -> np.ndarray:
    """FP32 logits[6] with the fixed operation order."""
    P = unpack(np.asarray(params, dtype=np.float32))
    h1 = _dense_f32(P["W1"], P["b1"], np.asarray(z, dtype=np.float32), True)
    h2 = _dense_f32(P["W2"], P["b2"], h1, True)
    return _dense_f32(P["W3"], P["b3"], h2, False)


def decide(logits, z, feasible_bits: int, tau: float):
    """(variant, margin, fallback) with masked argmax and the fallback rule."""
    best, second = -1, -1
    for v in range(6):
        if not (feasible_bits >> v) & 1:
            continue
        if best < 0 or logits[v] > logits[best]:
            best, second = v, best
        elif second < 0 or logits[v] > logits[second]:
            second = v
    if best < 0:
        return -1, np.float32(0.0), True
    margin = (np.float32(logits[best] - logits[second]) if second >= 0
              else np.float32(np.inf))
    ood = bool(np.any(np.abs(np.asarray(z, dtype=np.float32)) > np.float32(Z_LIMIT)))
    fallback = bool(margin < np.float32(tau)) or ood
    return best, margin, fallback


# ---------------------------------------------------------------- training


def forward_backward64(params, Z, labels, mask=None, accept=None):
    """Mean softmax cross-entropy and its gradient, in FP64.

    ``Z`` [B,12], ``labels`` [B] ints, ``mask`` [B,6] booleans of feasible
    variants (None = all feasible).  Infeasible logits are removed from the
    softmax.  With ``accept`` [B,6] booleans (labels then unused), the
    target of sample b is the set A_b of its accepted feasible variants and
    its loss is -log(sum_{j in A_b} p_j): the probability that the network's
    distribution picks an acceptable variant; differentiating,
    dL/dlogit_j = p_j - [j in A_b] p_j / sum_{A_b} p.  Returns (loss, grad
    flat float64[5382]).
    """
    P = {k: v.astype(np.float64) for k, v in unpack(np.asarray(params, np.float64)).items()}
    Z = np.asarray(Z, dtype=np.float64)
    B = Z.shape[0]
    a1 = Z @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    lg = h2 @ P["W3"].T + P["b3"]
    if mask is not None:
        lg = np.where(mask, lg, -np.inf)
    mx = lg.max(axis=1, keepdims=True)
    ex = np.exp(lg - mx)
    sm = ex / ex.sum(axis=1, keepdims=True)
    if accept is None:
        lab = np.asarray(labels, dtype=np.int64)
        loss = float(np.mean(-np.log(sm[np.arange(B), lab])))
        d_lg = sm.copy()
        d_lg[np.arange(B), lab] -= 1.0
    else:
        A = np.asarray(accept, dtype=bool)
        if mask is not None:
            A = A & np.asarray(mask, dtype=bool)
        pa = np.where(A, sm, 0.0)
        sa = pa.sum(axis=1, keepdims=True)
        loss = float(np.mean(-np.log(sa[:, 0])))
        d_lg = sm - pa / sa
    d_lg /= B
    g = {}
    g["W3"] = d_lg.T @ h2
    g["b3"] = d_lg.sum(axis=0)
    d_h2 = d_lg @ P["W3"]
    d_a2 = d_h2 * (a2 > 0)
    g["W2"] = d_a2.T @ h1
    g["b2"] = d_a2.sum(axis=0)
    d_h1 = d_a2 @ P["W2"]
    d_a1 = d_h1 * (a1 > 0)
    g["W1"] = d_a1.T @ Z
    g["b1"] = d_a1.sum(axis=0)
    flat = np.zeros(N_PARAMS, dtype=np.float64)
    for name, shape, off in LAYOUT:
        flat[off:off + int(np.prod(shape))] = g[name].reshape(-1)
    return loss, flat


def loss64(params, Z, labels, mask=None, accept=None) -> float:
    return forward_backward64(params, Z, labels, mask, accept)[0]


def adam_step_ref(p, g, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (FP64); returns new (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
