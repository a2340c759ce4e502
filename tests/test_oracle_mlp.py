"""Pins of the MLP oracle: calculus identities, closed forms, exactness."""
import math

import numpy as np

import synth
from oracle import mlp


def batch(seed, B=16):
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(B, 12))
    lab = rng.integers(0, 6, size=B)
    mask = rng.random((B, 6)) < 0.8
    mask[np.arange(B), lab] = True
    return Z, lab, mask


def test_param_count():
    assert mlp.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 6 + 6 == 5382


def test_gradient_central_differences():
    p = synth.he_uniform_params(3).astype(np.float64)
    p += np.random.default_rng(0).normal(scale=0.05, size=p.shape)  # nonzero biases
    Z, lab, mask = batch(1)
    _, g = mlp.forward_backward64(p, Z, lab, mask)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, 300, replace=False)
    eps = 1e-6
    for i in idx:
        d = np.zeros_like(p)
        d[i] = eps
        num = (mlp.loss64(p + d, Z, lab, mask) - mlp.loss64(p - d, Z, lab, mask)) / (2 * eps)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (i, num, g[i])


def test_zero_hidden_weights_bias_only_softmax():
    """W = 0 everywhere: logits = b3, grads of b3 = mean(softmax - onehot)."""
    p = np.zeros(mlp.N_PARAMS)
    b3 = np.array([0.3, -0.1, 0.0, 0.7, -0.4, 0.2])
    off = dict((n, o) for n, _, o in mlp.LAYOUT)
    p[off["b3"]:off["b3"] + 6] = b3
    Z, lab, _ = batch(4)
    loss, g = mlp.forward_backward64(p, Z, lab)
    sm = np.exp(b3) / np.exp(b3).sum()
    onehot = np.zeros((len(lab), 6))
    onehot[np.arange(len(lab)), lab] = 1
    np.testing.assert_allclose(g[off["b3"]:off["b3"] + 6], (sm - onehot).mean(0), atol=1e-15)
    assert abs(loss - np.mean(-np.log(sm[lab]))) < 1e-14
    # every other gradient is zero (relu'(0) = 0 and h = 0)
    rest = np.delete(g, np.arange(off["b3"], off["b3"] + 6))
    assert np.all(rest == 0)


def test_adam_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2: update = lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    p1, m, v = mlp.adam_step_ref(p, g, np.zeros(4), np.zeros(4), 1)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_plog2_exact_at_powers_and_linear_between():
    for k in range(0, 40):
        assert mlp.plog2(2.0 ** k) == k
        assert mlp.plog2(1.5 * 2.0 ** k) == k + 0.5
    assert mlp.plog2(1.0) == 0.0
    v = np.linspace(1, 1e6, 1000)
    pl = [mlp.plog2(t) for t in v]
    assert all(b >= a for a, b in zip(pl, pl[1:]))
    assert all(abs(p - math.log2(t)) < 0.09 for p, t in zip(pl, v))


def test_forward_f32_close_to_fp64():
    p = synth.he_uniform_params(11)
    rng = np.random.default_rng(3)
    for _ in range(5):
        z = rng.normal(size=12).astype(np.float32)
        lf = mlp.forward_f32(p, z)
        P = mlp.unpack(p.astype(np.float64))
        h1 = np.maximum(P["W1"] @ z.astype(np.float64) + P["b1"], 0)
        h2 = np.maximum(P["W2"] @ h1 + P["b2"], 0)
        l64 = P["W3"] @ h2 + P["b3"]
        np.testing.assert_allclose(lf, l64, rtol=0, atol=1e-5 * (1 + np.abs(l64).max()))


def test_decide_masking_ties_fallback():
    lg = np.array([1.0, 3.0, 3.0, 0.5, 2.0, -1.0], dtype=np.float32)
    z = np.zeros(12, np.float32)
    v, m, fb = mlp.decide(lg, z, 0b111111, 0.1)
    assert v == 1 and m == 0 and fb                  # tie -> first, margin 0 < tau
    v, m, fb = mlp.decide(lg, z, 0b111101, 0.1)
    assert v == 2 and m == np.float32(1.0) and not fb
    z[3] = 9.0
    assert mlp.decide(lg, z, 0b111101, 0.1)[2]       # out of distribution
    v, m, fb = mlp.decide(lg, np.zeros(12, np.float32), 0b000001, 0.1)
    assert v == 0 and m == np.inf and not fb


def test_transform_order_of_operations():
    f = [4096.0, 20224.0, 4.9375, 0.25, 5.0, 3.0, 126.0, 11.0, 0.04, 0.01, 0.4, 1.0]
    mu = np.arange(12, dtype=np.float32) * 0.5
    rho = np.full(12, 0.25, dtype=np.float32)
    z = mlp.transform(f, mu, rho)
    for k in range(12):
        g = mlp.plog2(1.0 + f[k]) if k < 8 else f[k]
        assert z[k] == np.float32(np.float32(np.float32(g) - mu[k]) * rho[k])
    assert mlp.plog2(1.0 + 4096.0) == 12 + (2 * (4097 / 8192) - 1)


# ---------------------------------------------------------------- set targets
def accept_sets(seed, mask):
    rng = np.random.default_rng(seed)
    A = (rng.random(mask.shape) < 0.4) & mask
    first = np.argmax(mask, axis=1)
    A[np.arange(len(A)), first] = True           # at least one feasible mark
    return A


def test_set_loss_gradient_central_differences():
    p = synth.he_uniform_params(5).astype(np.float64)
    p += np.random.default_rng(6).normal(scale=0.05, size=p.shape)
    Z, lab, mask = batch(7)
    A = accept_sets(8, mask)
    _, g = mlp.forward_backward64(p, Z, lab, mask, A)
    idx = np.random.default_rng(9).choice(mlp.N_PARAMS, 300, replace=False)
    eps = 1e-6
    for i in idx:
        d = np.zeros_like(p)
        d[i] = eps
        num = (mlp.loss64(p + d, Z, lab, mask, A) - mlp.loss64(p - d, Z, lab, mask, A)) / (2 * eps)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (i, num, g[i])


def test_set_loss_special_cases():
    """Singleton sets are the cross-entropy bit for bit; a set holding every
    feasible variant costs nothing (its probability is 1: loss 0, gradient 0)."""
    p = synth.he_uniform_params(10).astype(np.float64)
    Z, lab, mask = batch(11)
    one = np.zeros_like(mask)
    one[np.arange(len(lab)), lab] = True
    l1, g1 = mlp.forward_backward64(p, Z, lab, mask)
    l2, g2 = mlp.forward_backward64(p, Z, None, mask, one)
    assert abs(l1 - l2) <= 1e-15 * max(1.0, abs(l1)) and np.allclose(g1, g2, rtol=0, atol=1e-17)
    l3, g3 = mlp.forward_backward64(p, Z, None, mask, mask.copy())
    assert abs(l3) < 1e-15 and np.max(np.abs(g3)) < 1e-15


def test_set_loss_bias_only_closed_form():
    """W = 0: logits = b3, so the loss is -log(sum_A softmax(b3)) for each
    sample and the b3 gradient is mean(p - p [A] / sum_A p)."""
    p = np.zeros(mlp.N_PARAMS)
    b3 = np.array([0.3, -0.1, 0.0, 0.7, -0.4, 0.2])
    off = dict((n, o) for n, _, o in mlp.LAYOUT)
    p[off["b3"]:off["b3"] + 6] = b3
    Z, lab, _ = batch(12)
    A = accept_sets(13, np.ones((len(lab), 6), bool))
    loss, g = mlp.forward_backward64(p, Z, None, None, A)
    sm = np.exp(b3) / np.exp(b3).sum()
    sa = (A * sm).sum(axis=1)
    assert abs(loss - np.mean(-np.log(sa))) < 1e-14
    want = (sm[None, :] - A * sm[None, :] / sa[:, None]).mean(axis=0)
    np.testing.assert_allclose(g[off["b3"]:off["b3"] + 6], want, atol=1e-15)
