"""Long-row stress test of the FP32 path: one 200k-nonzero row of positive
values in [1, 2) with x = 1.  FP32 accumulation with Kahan compensation must
keep the error at a few units of rounding relative to sum |a||x|, whatever
the row length; the uncompensated sequential FP32 sum of the same row (on
the CPU) is shown beside it and is much worse."""
import math

import numpy as np
import pytest

import paper_1511_02494_amd as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import dev  # noqa: E402

N_COLS = 200_000


def test_kahan_keeps_a_200k_row_accurate():
    rng = np.random.default_rng(0)
    v = (1.0 + rng.random(N_COLS)).astype(np.float32)   # exact FP32 data
    rp = np.array([0, N_COLS], np.int32)
    ci = np.arange(N_COLS, dtype=np.int32)
    exact = math.fsum(float(a) for a in v)               # x = 1: s = the sum itself
    naive = abs(float(np.cumsum(v, dtype=np.float32)[-1]) - exact) / exact
    plan = S.Plan(dev(rp), dev(ci), dev(v), N_COLS, S.SPMV_F32, nnz=N_COLS)
    x = torch.ones(N_COLS, dtype=torch.float32, device="cuda:0")
    mask = plan.mask()
    errs = {}
    for var in range(6):
        if not (mask >> var) & 1:
            continue
        plan.set_variant(var)
        y = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda:0")
        plan.execute(x, y)
        torch.cuda.synchronize()
        errs[S.VARIANTS[var]] = abs(float(y.item()) - exact) / exact
    plan.close()
    print(f"\nuncompensated sequential FP32: {naive:.2e}; " +
          ", ".join(f"{k} {e:.2e}" for k, e in errs.items()), flush=True)
    u = 2.0 ** -24
    assert naive > 8 * u
    for k, e in errs.items():
        assert e <= 8 * u, (k, e)
