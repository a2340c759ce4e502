"""Conjugate gradients with each variant (GPU, through the C ABI) against the
CG oracle: converged solutions, true residuals, iteration counts, determinism."""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S
from oracle.cg import cg_ref
from oracle.spmv import spmv_seq

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import dev, make_plan  # noqa: E402

SYSTEMS = {
    "laplace64": (lambda: synth.laplace2d(64), 4096),
    "stencil27_12": (lambda: synth.stencil3d_27(12, seed=3), 1728),
}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_cg_every_variant_matches_oracle(name):
    build, n = SYSTEMS[name]
    rp, ci, v = build()
    b = synth.vector(n, 5)
    x_ref, it_ref, _, _ = cg_ref(rp, ci, v, b, max_iters=2000, rtol=1e-10)
    plan = make_plan(rp, ci, v, n)
    mask = plan.mask()
    for var in range(6):
        if not (mask >> var) & 1:
            continue
        plan.set_variant(var)
        sols = []
        for _ in range(2):
            x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
            it, rel = S.spmv_cg(plan.handle, dev(b), x, 2000, 1e-10)
            sols.append(x.cpu().numpy())
        print(f"{name} {S.VARIANTS[var]}: {it} iterations (oracle {it_ref}), rel {rel:.2e}", flush=True)
        assert np.array_equal(sols[0], sols[1]), "not deterministic"
        assert abs(it - it_ref) <= 2 and rel <= 1e-10
        true = np.linalg.norm(b - spmv_seq(rp, ci, v, sols[0])) / np.linalg.norm(b)
        assert true <= 1e-9
        assert np.linalg.norm(sols[0] - x_ref) <= 1e-6 * np.linalg.norm(x_ref)
    plan.close()


def test_cg_edge_cases():
    rp, ci, v = synth.laplace2d(16)
    plan = make_plan(rp, ci, v, 256)
    x = torch.zeros(256, dtype=torch.float64, device="cuda:0")
    assert S.spmv_cg(plan.handle, dev(np.zeros(256)), x, 100, 1e-8) == (0, 0.0)
    b = synth.vector(256, 6)
    x0 = synth.vector(256, 7)
    x = dev(x0.copy())
    it, rel = S.spmv_cg(plan.handle, dev(b), x, 3, 1e-14)
    x_ref, it_ref, rel_ref, _ = cg_ref(rp, ci, v, b, x0=x0, max_iters=3, rtol=1e-14)
    assert it == it_ref == 3
    assert rel == pytest.approx(rel_ref, rel=1e-9)
    assert np.allclose(x.cpu().numpy(), x_ref, rtol=1e-11, atol=1e-13)
    plan.close()
    p32 = make_plan(rp, ci, v, 256, S.SPMV_F32)
    with pytest.raises(S.SpmvError) as e:
        S.spmv_cg(p32.handle, dev(b), x, 10, 1e-8)
    assert e.value.status == S.SPMV_ERR_ARG
    p32.close()
    rr, cc, vv = synth.uniform_random(100, 300, 4, seed=1)
    rect = make_plan(rr, cc, vv, 300)
    with pytest.raises(S.SpmvError):
        S.spmv_cg(rect.handle, dev(np.ones(100)), dev(np.zeros(300)), 10, 1e-8)
    rect.close()
