"""MLP selector on the device against the oracle (GPU)."""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle import mlp
from paper_1511_02494_amd.model_io import write_model

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import dev  # noqa: E402


@pytest.fixture
def model(tmp_path):
    p = synth.he_uniform_params(5)
    p[768:832] = np.linspace(-0.1, 0.1, 64, dtype=np.float32)  # nonzero biases
    mu = np.linspace(0, 3, 12).astype(np.float32)
    rho = np.linspace(0.2, 1.1, 12).astype(np.float32)
    path = str(tmp_path / "m.bin")
    write_model(path, p, mu, rho, 0.05)
    S.spmv_model_load(path)
    yield p, mu, rho, np.float32(0.05)
    S.spmv_model_unload()


def feature_vectors():
    out = [[4096.0, 20224.0, 4.9375, 0.246, 5.0, 3.0, 126.03, 10.96, 0.039, 0.01, 0.398, 1.0],
           [1e6, 2.6e7, 26.46, 1.2, 27.0, 8.0, 20200.0, 300.0, 0.0013, 0.0002, 0.07, 0.0],
           [2e6, 1.6e7, 8.0, 0.0, 8.0, 8.0, 1.75e6, 1.4e5, 4.5e-6, 1e-6, 0.99, 0.0]]
    rng = np.random.default_rng(1)
    for _ in range(20):
        f = list(10 ** rng.uniform(0, 7, 8)) + list(rng.uniform(0, 1, 3)) + [float(rng.integers(0, 2))]
        out.append(f)
    return out


def test_predict_bit_exact(model):
    p, mu, rho, tau = model
    for i, f in enumerate(feature_vectors()):
        feas = [0x3F, 0x37, 0x27, 0x01, 0x20][i % 5]
        got = S.spmv_mlp_predict(f, feas)
        z = mlp.transform(f, mu, rho)
        lg = mlp.forward_f32(p, z)
        v, margin, fb = mlp.decide(lg, z, feas, tau)
        assert np.array_equal(got["z"].view(np.uint32), z.view(np.uint32))
        assert np.array_equal(got["logits"].view(np.uint32), lg.view(np.uint32))
        assert got["variant"] == v
        assert np.float32(got["margin"]).view(np.uint32) == np.float32(margin).view(np.uint32)
        assert got["fallback"] == fb


def test_predict_without_model():
    S.spmv_model_unload()
    with pytest.raises(S.SpmvError) as e:
        S.spmv_mlp_predict([1.0] * 12)
    assert e.value.status == S.SPMV_ERR_NO_MODEL


def rel_frob(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("B", [1, 7, 128])
def test_gradients_against_fp64_oracle(B):
    rng = np.random.default_rng(B)
    p = synth.he_uniform_params(9)
    p += rng.normal(scale=0.02, size=p.shape).astype(np.float32)
    Z = rng.normal(size=(B, 12)).astype(np.float32)
    lab = rng.integers(0, 6, B).astype(np.int32)
    mask = rng.random((B, 6)) < 0.8
    mask[np.arange(B), lab] = True
    loss64, g64 = mlp.forward_backward64(p.astype(np.float64), Z.astype(np.float64), lab, mask)
    dp, dZ, dl, dm = dev(p), dev(Z), dev(lab), dev(mask.astype(np.uint8))
    g = torch.empty(5382, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    S.spmv_mlp_forward_backward(dp, dZ, dl, dm, B, g, loss)
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    for name, shape, off in mlp.LAYOUT:
        k = int(np.prod(shape))
        assert rel_frob(gg[off:off + k], g64[off:off + k]) <= 1e-4, name
    assert abs(loss.item() - loss64) <= 1e-5 * max(1.0, abs(loss64))


@pytest.mark.parametrize("B", [1, 9, 256])
def test_set_gradients_against_fp64_oracle(B):
    """Set-valued targets (every acceptable variant marked): device FP32
    gradients within 1e-4 (Frobenius, per tensor) of the FP64 oracle."""
    rng = np.random.default_rng(100 + B)
    p = synth.he_uniform_params(11)
    p += rng.normal(scale=0.02, size=p.shape).astype(np.float32)
    Z = rng.normal(size=(B, 12)).astype(np.float32)
    mask = rng.random((B, 6)) < 0.8
    acc = (rng.random((B, 6)) < 0.4) & mask
    first = np.argmax(mask | (np.arange(6) == 0)[None, :], axis=1)
    mask[np.arange(B), first] = True
    acc[np.arange(B), first] = True
    loss64, g64 = mlp.forward_backward64(p.astype(np.float64), Z.astype(np.float64), None, mask, acc)
    g = torch.empty(5382, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    S.spmv_mlp_forward_backward_sets(dev(p), dev(Z), dev(acc.astype(np.uint8)), dev(mask.astype(np.uint8)),
                                     B, g, loss)
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    for name, shape, off in mlp.LAYOUT:
        k = int(np.prod(shape))
        assert rel_frob(gg[off:off + k], g64[off:off + k]) <= 1e-4, name
    assert abs(loss.item() - loss64) <= 1e-5 * max(1.0, abs(loss64))


def test_adam_step_against_oracle():
    rng = np.random.default_rng(3)
    n = 5382
    p = rng.normal(size=n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    m = rng.normal(scale=0.1, size=n).astype(np.float32)
    v = rng.uniform(0, 0.1, size=n).astype(np.float32)
    P, M, V = dev(p), dev(m), dev(v)
    S.spmv_mlp_adam_step(P, dev(g), M, V, n, 5, 1e-3, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    p1, m1, v1 = mlp.adam_step_ref(p, g, m, v, 5)
    got = P.cpu().numpy()
    # FP32 parameters: within two ulps of the FP64 update plus 1e-5 of the step
    ulp = np.spacing(np.abs(p1).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got - p1) <= 2 * ulp + 1e-5 * np.abs(p1 - p))
    assert rel_frob(M.cpu().numpy().astype(np.float64), m1) <= 1e-6
    assert rel_frob(V.cpu().numpy().astype(np.float64), v1) <= 1e-6


def test_loss_decreases_on_separable_toy():
    rng = np.random.default_rng(0)
    B = 128
    Z = rng.normal(size=(B, 12)).astype(np.float32)
    lab = (Z[:, 0] > 0).astype(np.int32) * 3
    mask = np.ones((B, 6), np.uint8)
    P = dev(synth.he_uniform_params(1))
    M = torch.zeros(5382, device="cuda:0")
    V = torch.zeros(5382, device="cuda:0")
    G = torch.empty(5382, device="cuda:0")
    L = torch.empty(1, device="cuda:0")
    dZ, dl, dm = dev(Z), dev(lab), dev(mask)
    losses = []
    for step in range(1, 201):
        S.spmv_mlp_forward_backward(P, dZ, dl, dm, B, G, L)
        S.spmv_mlp_adam_step(P, G, M, V, 5382, step, 1e-2)
        losses.append(L.item())
    assert losses[-1] < 0.1 * losses[0]
