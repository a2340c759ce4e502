"""Long-row stress test of the FP32 path: one 200k-nonzero row of positive
values in [1, 2) with x = 1, run through the same kernels with Kahan
compensation on (the default for rows longer than 256) and off
(spmv_set_kahan_min_len(INT32_MAX)).

With compensation every variant stays within a few units of rounding of the
exact sum, whatever the row length.  Without it the one-thread-per-row
kernels (csr_scalar, short_row) reproduce the plain sequential FP32 sum bit
for bit, whose error grows with the row length, and the other kernels split
the row over many partial sums and land in between.
"""
import math

import numpy as np
import pytest

import paper_1511_02494_amd as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_util import dev  # noqa: E402

N_COLS = 200_000
INT32_MAX = 2 ** 31 - 1
SEQUENTIAL = {"csr_scalar", "short_row"}


def run_all(plan, x):
    out = {}
    mask = plan.mask()
    for var in range(6):
        if not (mask >> var) & 1:
            continue
        plan.set_variant(var)
        y = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda:0")
        plan.execute(x, y)
        torch.cuda.synchronize()
        out[S.VARIANTS[var]] = float(y.item())
    return out


def test_kahan_on_and_off_on_a_200k_row():
    rng = np.random.default_rng(0)
    v = (1.0 + rng.random(N_COLS)).astype(np.float32)   # exact FP32 data
    rp = np.array([0, N_COLS], np.int32)
    ci = np.arange(N_COLS, dtype=np.int32)
    exact = math.fsum(float(a) for a in v)               # x = 1: s = the sum itself
    naive = float(np.cumsum(v, dtype=np.float32)[-1])    # the plain sequential FP32 sum
    plan = S.Plan(dev(rp), dev(ci), dev(v), N_COLS, S.SPMV_F32, nnz=N_COLS)
    x = torch.ones(N_COLS, dtype=torch.float32, device="cuda:0")
    comp = run_all(plan, x)
    S.spmv_set_kahan_min_len(plan.handle, INT32_MAX)
    plain = run_all(plan, x)
    plan.close()
    rel = lambda y: abs(y - exact) / exact  # noqa: E731
    print(f"\nplain sequential FP32 (CPU): {rel(naive):.2e}")
    for k in comp:
        print(f"  {k:>10s}: Kahan {rel(comp[k]):.2e}   uncompensated {rel(plain[k]):.2e}", flush=True)
    u = 2.0 ** -24
    assert rel(naive) > 8 * u
    for k in comp:
        assert rel(comp[k]) <= 8 * u, (k, rel(comp[k]))
        if k in SEQUENTIAL:
            assert plain[k] == naive, (k, plain[k], naive)  # the same sequence of roundings
        assert rel(plain[k]) <= rel(naive) * 1.01 or k not in SEQUENTIAL
    # compensation is what keeps the sequential kernels accurate
    assert all(rel(plain[k]) > 8 * u for k in SEQUENTIAL if k in plain)
