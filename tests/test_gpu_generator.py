"""The device generator produces the same bytes as the seeded CPU generator."""
import numpy as np
import pytest

import synth
import paper_1511_02494_amd as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPECS = [
    ("laplace2d", [40, 0], synth.laplace2d, dict(n=40, values="const")),
    ("laplace2d", [33, 1], synth.laplace2d, dict(n=33, values="random")),
    ("stencil2d_9", [30, 1], synth.stencil2d_9, dict(n=30)),
    ("stencil3d_7", [17, 1], synth.stencil3d_7, dict(n=17)),
    ("stencil3d_27", [15, 0], synth.stencil3d_27, dict(n=15, values="const")),
    ("stencil3d_27", [14, 1], synth.stencil3d_27, dict(n=14, values="random")),
    ("uniform_random", [5000, 70000, 8], synth.uniform_random, dict(n_rows=5000, n_cols=70000, per_row=8)),
    ("banded", [7000, 333, 50], synth.banded, dict(n=7000, d16=333, half_width=50)),
    ("banded", [3000, 2000, 10], synth.banded, dict(n=3000, d16=2000, half_width=10)),
    ("random_rows", [6000, 100], synth.random_rows, dict(n=6000, d16=100)),
    ("powerlaw", [20000, 109, 4000, 1], synth.powerlaw, dict(n=20000, p16=109, cap=4000)),
    ("powerlaw", [20000, 5, 4000, 0], synth.powerlaw, dict(n=20000, p16=5, cap=4000, force_long=False)),
    ("short_rows", [12345], synth.short_rows, dict(n=12345)),
]


def device_generate(fam, params, seed):
    fid = S.FAMILY[fam]
    if fid <= 1:
        n = params[0] ** 2
    elif fid <= 3:
        n = params[0] ** 3
    else:
        n = params[0]
    rp = torch.empty(n + 1, dtype=torch.int32, device="cuda:0")
    nnz = S.spmv_generate(fid, params, seed, rp)
    ci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda:0")
    v = torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda:0")
    S.spmv_generate(fid, params, seed, rp, ci, v)
    torch.cuda.synchronize()
    return rp.cpu().numpy(), ci.cpu().numpy()[:nnz], v.cpu().numpy()[:nnz]


@pytest.mark.parametrize("seed", [0, 7, 123456789])
@pytest.mark.parametrize("fam,params,fn,kw", SPECS)
def test_generator_bytes(fam, params, fn, kw, seed):
    grp, gci, gv = device_generate(fam, params, seed)
    rp, ci, v = fn(seed=seed, **kw)
    assert np.array_equal(grp, rp)
    assert np.array_equal(gci, ci)
    assert np.array_equal(gv.view(np.uint64), np.asarray(v, np.float64).view(np.uint64))


def test_vector_bytes():
    x = torch.empty(100003, dtype=torch.float64, device="cuda:0")
    S.spmv_generate_vector(100003, 42, x)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy().view(np.uint64), synth.vector(100003, 42).view(np.uint64))
