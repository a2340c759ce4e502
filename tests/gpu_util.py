"""Helpers shared by the GPU tests: device copies and variant runs."""
import numpy as np
import torch

import paper_1511_02494_amd as S
from oracle.encode import to_bf16_bits_ref, to_f32_ref

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def upload_csr(rp, ci, val, dtype=S.SPMV_F64):
    """Device tensors for a CSR matrix; values quantised to ``dtype``."""
    r = dev(np.asarray(rp, np.int32))
    c = dev(np.asarray(ci, np.int32)) if len(ci) else torch.zeros(4, dtype=torch.int32, device=DEV)
    if dtype == S.SPMV_F64:
        v = np.asarray(val, np.float64)
        vt = dev(v) if len(v) else torch.zeros(2, dtype=torch.float64, device=DEV)
    elif dtype == S.SPMV_F32:
        v = to_f32_ref(val)
        vt = dev(v) if len(v) else torch.zeros(4, dtype=torch.float32, device=DEV)
    else:
        v = to_bf16_bits_ref(val).view(np.int16)
        vt = dev(v) if len(v) else torch.zeros(8, dtype=torch.int16, device=DEV)
    return r, c, vt


def x_tensor(x, dtype=S.SPMV_F64):
    x = np.asarray(x, np.float64)
    if dtype == S.SPMV_F64:
        return dev(x) if len(x) else torch.zeros(2, dtype=torch.float64, device=DEV)
    xf = x.astype(np.float32)
    return dev(xf) if len(xf) else torch.zeros(4, dtype=torch.float32, device=DEV)


def make_plan(rp, ci, val, n_cols, dtype=S.SPMV_F64, flags=0):
    r, c, v = upload_csr(rp, ci, val, dtype)
    return S.Plan(r, c, v, n_cols, dtype, flags=flags, nnz=len(ci))


def run(plan, variant, x, dtype=S.SPMV_F64, fill=np.nan):
    """y = A x with ``variant`` (y pre-filled with ``fill`` to catch unwritten rows)."""
    S.spmv_set_variant(plan.handle, variant)
    xt = x_tensor(x, dtype)
    tdt = torch.float64 if dtype == S.SPMV_F64 else torch.float32
    y = torch.full((max(plan.n, 1),), fill, dtype=tdt, device=DEV)
    plan.execute(xt, y)
    torch.cuda.synchronize()
    return y[:plan.n].cpu().numpy().astype(np.float64)
