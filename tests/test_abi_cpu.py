"""CPU checks of the C ABI: exported symbols, host-only entry points."""
import os
import re

import numpy as np
import pytest

import paper_1511_02494_amd as S
from paper_1511_02494_amd.model_io import read_model, write_model
from oracle.select import decide_profile_ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "spmvsel.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spmv_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(S.lib, n), n
        assert n in S._PROTOS, f"binding lacks {n}"


def test_profile_decide_matches_oracle():
    rng = np.random.default_rng(0)
    for _ in range(3000):
        meas = list(rng.choice([0.0, 0.5, 1.0, 1.5, 2.0, 3.0], 5) * rng.uniform(0.5, 2, 5))
        feats = [0.0] * 12
        feats[2] = float(rng.choice([1.0, 3.9, 4.0, 4.1, 27.0]))
        theta = list(rng.choice([1.0, 1.2, 1.5, 2.0], 3)) + [4.0]
        feas = int(rng.integers(0, 64)) | 0b100111
        assert S.spmv_profile_decide(meas, feats, theta, feas) == decide_profile_ref(meas, feats, theta, feas)


def test_thresholds_roundtrip():
    old = S.spmv_get_thresholds()
    S.spmv_set_thresholds([3.0, 1.1, 1.7, 2.0])
    assert S.spmv_get_thresholds() == [3.0, 1.1, 1.7, 2.0]
    S.spmv_set_thresholds(old)


def test_model_file_roundtrip_and_corruption(tmp_path):
    p = np.arange(5382, dtype=np.float32) / 5382
    path = str(tmp_path / "m.bin")
    write_model(path, p, np.ones(12), np.full(12, 0.5), 0.25)
    q, mu, rho, tau = read_model(path)
    assert np.array_equal(q, p) and tau == np.float32(0.25)
    S.spmv_model_load(path)
    S.spmv_model_unload()
    raw = bytearray(open(path, "rb").read())
    raw[200] ^= 1
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(S.SpmvError) as e:
        S.spmv_model_load(bad)
    assert e.value.status == S.SPMV_ERR_NO_MODEL
    with pytest.raises(S.SpmvError) as e:
        S.spmv_model_load(str(tmp_path / "missing.bin"))
    assert e.value.status == S.SPMV_ERR_NO_MODEL


def test_plan_create_argument_errors():
    for args in [(-1, 1, 0), (1, -1, 0), (1, 1, -1), (2 ** 31, 1, 0), (2 ** 31 - 1, 1, 0),
                 (1, 2 ** 31, 0), (1, 1, 2 ** 31 - 2 ** 16), (1, 1, 2 ** 31 - 1)]:
        with pytest.raises(S.SpmvError) as e:
            S.spmv_plan_create(*args, 16, 16, 16, S.SPMV_F64, 0)
        assert e.value.status == S.SPMV_ERR_ARG
    with pytest.raises(S.SpmvError):
        S.spmv_plan_create(4, 4, 4, 16, 16, 16, 7, 0)          # unknown dtype
    with pytest.raises(S.SpmvError):
        S.spmv_plan_create(4, 4, 4, None, 16, 16, S.SPMV_F64, 0)  # NULL rowptr
    with pytest.raises(S.SpmvError):
        S.spmv_plan_create(4, 4, 4, 16, 8, 16, S.SPMV_F64, 0)   # misaligned colind
    S.spmv_plan_destroy(None)


def test_null_plan_arguments():
    for fn, args in [(S.spmv_set_xblock_slices, (None, 4)), (S.spmv_set_variant, (None, 1))]:
        with pytest.raises(S.SpmvError) as e:
            fn(*args)
        assert e.value.status == S.SPMV_ERR_ARG


def test_noalloc_rejects_before_device_work():
    """Sizes beyond the static scratch array, bad sizes and dtypes are
    rejected on the host (no device call is made, so this runs without a GPU)."""
    limit = (((8 << 20) - 1024) // 20) * 2048
    for n, m, nnz, dt in [(-1, 4, 0, S.SPMV_F64), (4, 4, -1, S.SPMV_F64), (4, 4, 4, 9),
                          (limit, 4, 1, S.SPMV_F64), (2 ** 31, 4, 0, S.SPMV_F64)]:
        with pytest.raises(S.SpmvError) as e:
            S.spmv_merge_path_noalloc(n, m, nnz, 16, 16, 16, dt, 16, 16, 0)
        assert e.value.status == S.SPMV_ERR_ARG


def test_index_coding_rejects_unknown_values():
    """Checked before the plan is touched (no device call)."""
    for bad in (-2, 2, 16):
        with pytest.raises(S.SpmvError) as e:
            S.spmv_set_index_coding(16, bad)
        assert e.value.status == S.SPMV_ERR_ARG
    with pytest.raises(S.SpmvError) as e:
        S.spmv_set_index_coding(None, 1)
    assert e.value.status == S.SPMV_ERR_ARG
