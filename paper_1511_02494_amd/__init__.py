"""Python binding of libspmvsel (selected CSR SpMV on MI355X).

Argument marshalling only: every function below calls the entry point of
the same name in ``libspmvsel.so`` (declared in ``include/spmvsel.h``).
Device arrays are passed as ``torch`` tensors (or raw integer addresses);
streams default to torch's current HIP stream.  Every non-zero status
raises :class:`SpmvError` with the library's message.  Importing works
without a GPU; the library must have been built (``__graft_entry__.build()``)
or the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmvsel.so")
DEFAULT_MODEL = os.path.join(_HERE, "mlp_selector.bin")

# status codes
SPMV_OK, SPMV_ERR_ARG, SPMV_ERR_CSR_ROWPTR, SPMV_ERR_CSR_COL_RANGE, SPMV_ERR_CSR_UNSORTED, \
    SPMV_ERR_OOM, SPMV_ERR_HIP, SPMV_ERR_INFEASIBLE, SPMV_ERR_NO_MODEL = range(9)
SPMV_F64, SPMV_F32, SPMV_BF16 = range(3)
SPMV_IDX_AUTO, SPMV_IDX_I32, SPMV_IDX_CODED = -1, 0, 1
V_CSR_SCALAR, V_CSR_VECTOR, V_MERGE_PATH, V_DELTA16, V_XBLOCK_LDS, V_SHORT_ROW = range(6)
VARIANTS = ["csr_scalar", "csr_vector", "merge_path", "delta16", "xblock_lds", "short_row"]
CLASSES = ["CML", "MB", "IMB", "CMP"]
SEL_PROFILING, SEL_MLP, SEL_EXHAUSTIVE, SEL_DTREE, SEL_GNB = range(5)
SPMV_CLF_DTREE, SPMV_CLF_GNB = range(2)
SPMV_LABEL_VARIANT, SPMV_LABEL_CLASS = range(2)
SPMV_COPY_INPUTS, SPMV_SKIP_VALIDATE = 1, 2
FEATURE_NAMES = ["N", "NNZ", "nnz_avg", "nnz_sd", "nnz_max", "nnz_min", "bw_avg", "bw_sd",
                 "dispersion_avg", "dispersion_sd", "miss_per_nnz", "size"]
FAMILY = {"laplace2d": 0, "stencil2d_9": 1, "stencil3d_7": 2, "stencil3d_27": 3,
          "uniform_random": 4, "banded": 5, "random_rows": 6, "powerlaw": 7, "short_rows": 8}

# every entry point the header declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I32, _U32, _I64, _U64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64
_F32, _F64 = ctypes.c_float, ctypes.c_double
_PI32, _PU32, _PI64, _PU64 = (ctypes.POINTER(t) for t in (_I32, _U32, _I64, _U64))
_PF32, _PF64 = ctypes.POINTER(_F32), ctypes.POINTER(_F64)


class SelectInfo(ctypes.Structure):
    _fields_ = [("variant", _I32), ("klass", _I32), ("selector", _I32), ("fell_back", _I32),
                ("feasible", _U32), ("margin", _F32), ("logits", _F32 * 6),
                ("meas", _F64 * 5), ("scores", _F64 * 3), ("features", _F64 * 12),
                ("t_features_s", _F64), ("t_decide_s", _F64), ("t_profile_s", _F64),
                ("t_total_s", _F64), ("t_prepare_s", _F64), ("variant_times_s", _F64 * 6)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


_PROTOS = {
    "spmv_plan_create": (_I32, [ctypes.POINTER(_P), _I64, _I64, _I64, _P, _P, _P, _I32, _P, _U32]),
    "spmv_plan_destroy": (_I32, [_P]),
    "spmv_features": (_I32, [_P, _PF64, _PU64]),
    "spmv_select": (_I32, [_P, _I32, ctypes.POINTER(SelectInfo)]),
    "spmv_execute": (_I32, [_P, _P, _P, _P]),
    "spmv_set_variant": (_I32, [_P, _I32]),
    "spmv_get_variant": (_I32, [_P, _PI32]),
    "spmv_set_kahan_min_len": (_I32, [_P, _I32]),
    "spmv_set_index_coding": (_I32, [_P, _I32]),
    "spmv_variant_mask": (_I32, [_P, _PU32]),
    "spmv_set_xblock_slices": (_I32, [_P, _I32]),
    "spmv_set_delta16_layout": (_I32, [_P, _I32]),
    "spmv_set_delta16_sort": (_I32, [_P, _I32]),
    "spmv_set_delta16_offset_bits": (_I32, [_P, _I32]),
    "spmv_bytes": (_I32, [_P, _I32, _PI64]),
    "spmv_time_variant": (_I32, [_P, _I32, _I32, _I32, _PF64, _PF64]),
    "spmv_time_variant_batch": (_I32, [_P, _I32, _I32, _I32, _PF64, _PF64]),
    "spmv_plan_query": (_I32, [_P, _I32, _PI64]),
    "spmv_plan_copy_format": (_I32, [_P, _I32, _P, _I64]),
    "spmv_profile_measure": (_I32, [_P, _I32, _PF64]),
    "spmv_profile_decide": (_I32, [_PF64, _PF64, _PF64, _U32, _PI32, _PI32]),
    "spmv_set_thresholds": (_I32, [_PF64]),
    "spmv_get_thresholds": (_I32, [_PF64]),
    "spmv_model_load": (_I32, [ctypes.c_char_p]),
    "spmv_model_unload": (_I32, []),
    "spmv_mlp_predict": (_I32, [_PF64, _U32, _PI32, _PF32, _PI32, _PF32, _PF32]),
    "spmv_mlp_forward_backward": (_I32, [_P, _P, _P, _P, _I32, _P, _P, _P]),
    "spmv_mlp_forward_backward_sets": (_I32, [_P, _P, _P, _P, _I32, _P, _P, _P]),
    "spmv_mlp_adam_step": (_I32, [_P, _P, _P, _P, _I32, _I32, _F32, _F32, _F32, _F32, _P]),
    "spmv_quantize": (_I32, [_P, _P, _I64, _I32, _P]),
    "spmv_generate": (_I32, [_I32, _PI64, _I32, _U64, _P, _P, _P, _PI64, _P]),
    "spmv_generate_vector": (_I32, [_I64, _U64, _P, _P]),
    "spmv_dtree_fit": (_I32, [_P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _PI32]),
    "spmv_gnb_fit": (_I32, [_P, _P, _I64, _I32, _P, _P, _P, _P]),
    "spmv_dtree_load": (_I32, [_I32, _I32, _I32, _P, _P, _P, _P, _P]),
    "spmv_gnb_load": (_I32, [_I32, _I32, _P, _P, _P, _P]),
    "spmv_classifier_unload": (_I32, [_I32]),
    "spmv_classifier_predict": (_I32, [_I32, _PF64, _U32, _PI32, _PI32, _PI32, _PI32, _PF64]),
    "spmv_cg": (_I32, [_P, _P, _P, _I32, _F64, _P, _PI32, _PF64]),
    "spmv_release_cached_blocks": (_I32, []),
    "spmv_cache_flush": (_I32, [_P]),
    "spmv_hbm_probe": (_I32, [_I64, _PF64, _PF64]),
    "spmv_gather_probe": (_I32, [_I64, _I32, _I32, _I64, _PF64]),
    "spmv_gather_probe2": (_I32, [_I64, _I32, _I32, _I64, _I32, _PF64]),
    "spmv_merge_path_noalloc": (_I32, [_I64, _I64, _I64, _P, _P, _P, _I32, _P, _P, _P]),
    "spmv_last_error": (ctypes.c_char_p, []),
}


class SpmvError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} -> status {status}: {msg}")
        self.status = status


def _load():
    # torch ships its own HIP runtime with the same soname as /opt/rocm's.
    # Loading torch first makes this library bind to that same runtime, so
    # streams and device pointers from torch are valid here (two runtimes in
    # one process cannot share them).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()
SELECTOR_CONFIG = os.path.join(_HERE, "selector_config.json")


def spmv_last_error() -> str:
    return lib.spmv_last_error().decode(errors="replace")


def _check(fn: str, st: int):
    if st != SPMV_OK:
        raise SpmvError(fn, st, spmv_last_error())


def _addr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _darr(vals, ctype):
    return (ctype * len(vals))(*vals)


# ----------------------------------------------------------------------- plan


def spmv_plan_create(n_rows, n_cols, nnz, rowptr, colind, val, val_dtype=SPMV_F64,
                     stream=None, flags=0):
    h = _P()
    _check("spmv_plan_create",
           lib.spmv_plan_create(ctypes.byref(h), n_rows, n_cols, nnz, _addr(rowptr),
                                _addr(colind), _addr(val), val_dtype, _stream(stream), flags))
    return h


def spmv_plan_destroy(plan):
    _check("spmv_plan_destroy", lib.spmv_plan_destroy(plan))


def spmv_features(plan):
    f = (_F64 * 12)()
    a = (_U64 * 12)()
    _check("spmv_features", lib.spmv_features(plan, f, a))
    return list(f), [int(v) for v in a]


def spmv_select(plan, selector=SEL_MLP) -> dict:
    info = SelectInfo()
    _check("spmv_select", lib.spmv_select(plan, selector, ctypes.byref(info)))
    return info.as_dict()


def spmv_execute(plan, x, y, stream=None):
    _check("spmv_execute", lib.spmv_execute(plan, _addr(x), _addr(y), _stream(stream)))


def spmv_set_index_coding(plan, coding: int):
    _check("spmv_set_index_coding", lib.spmv_set_index_coding(plan, coding))


def spmv_set_kahan_min_len(plan, length: int):
    _check("spmv_set_kahan_min_len", lib.spmv_set_kahan_min_len(plan, length))


def spmv_set_variant(plan, variant: int):
    _check("spmv_set_variant", lib.spmv_set_variant(plan, variant))


def spmv_get_variant(plan) -> int:
    v = _I32()
    _check("spmv_get_variant", lib.spmv_get_variant(plan, ctypes.byref(v)))
    return v.value


def spmv_set_xblock_slices(plan, slices: int):
    _check("spmv_set_xblock_slices", lib.spmv_set_xblock_slices(plan, slices))


def spmv_set_delta16_layout(plan, layout: int):
    _check("spmv_set_delta16_layout", lib.spmv_set_delta16_layout(plan, layout))


def spmv_set_delta16_sort(plan, mode: int):
    _check("spmv_set_delta16_sort", lib.spmv_set_delta16_sort(plan, mode))


def spmv_set_delta16_offset_bits(plan, bits: int):
    _check("spmv_set_delta16_offset_bits", lib.spmv_set_delta16_offset_bits(plan, bits))


def spmv_variant_mask(plan) -> int:
    b = _U32()
    _check("spmv_variant_mask", lib.spmv_variant_mask(plan, ctypes.byref(b)))
    return b.value


def spmv_bytes(plan, variant: int) -> int:
    b = _I64()
    _check("spmv_bytes", lib.spmv_bytes(plan, variant, ctypes.byref(b)))
    return b.value


def spmv_time_variant(plan, variant: int, reps: int = 10, cold: bool = False):
    med, mn = _F64(), _F64()
    _check("spmv_time_variant", lib.spmv_time_variant(plan, variant, reps, int(cold),
                                                      ctypes.byref(med), ctypes.byref(mn)))
    return med.value, mn.value


def spmv_time_variant_batch(plan, variant: int, launches: int, reps: int = 5):
    """(median, min) seconds per SpMV over ``reps`` runs of ``launches`` back-to-back executions."""
    a, b = _F64(), _F64()
    _check("spmv_time_variant_batch",
           lib.spmv_time_variant_batch(plan, variant, launches, reps, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def spmv_plan_query(plan, key: int) -> int:
    v = _I64()
    _check("spmv_plan_query", lib.spmv_plan_query(plan, key, ctypes.byref(v)))
    return v.value


_FORMAT_DTYPES = {0: np.int32, 1: np.uint16, 2: np.int32, 3: np.int32, 4: np.int32,
                  5: np.int32, 6: np.int32, 7: np.int32, 8: np.int32, 9: np.int32, 10: np.int32,
                  11: np.uint16, 13: np.int32, 14: np.int32, 15: np.uint32, 16: np.int32,
                  17: np.int32, 18: np.int32, 19: np.uint16, 20: np.int32, 21: np.uint16,
                  22: np.int32}


def spmv_plan_copy_format(plan, which: int, count: int, dtype=None) -> np.ndarray:
    """Array ``which`` of the plan's formats; ``dtype`` is required for the
    sliced delta16 values (12), which have the plan's value type.  The sliced
    column codes (11) take the plan's code width (query key 17)."""
    if dtype is None and which == 11:
        dtype = np.uint8 if spmv_plan_query(plan, 17) == 8 else np.uint16
    out = np.empty(count, dtype=dtype or _FORMAT_DTYPES[which])
    _check("spmv_plan_copy_format",
           lib.spmv_plan_copy_format(plan, which, out.ctypes.data_as(_P), out.nbytes))
    return out


# ----------------------------------------------------------------- selectors


def spmv_profile_measure(plan, reps: int = 3):
    m = (_F64 * 5)()
    _check("spmv_profile_measure", lib.spmv_profile_measure(plan, reps, m))
    return list(m)


def spmv_profile_decide(meas, features, theta, feasible_bits: int):
    v, k = _I32(), _I32()
    _check("spmv_profile_decide",
           lib.spmv_profile_decide(_darr(meas, _F64), _darr(features, _F64),
                                   _darr(theta, _F64), feasible_bits, ctypes.byref(v),
                                   ctypes.byref(k)))
    return v.value, k.value


def spmv_set_thresholds(theta):
    _check("spmv_set_thresholds", lib.spmv_set_thresholds(_darr(theta, _F64)))


def spmv_get_thresholds():
    t = (_F64 * 4)()
    _check("spmv_get_thresholds", lib.spmv_get_thresholds(t))
    return list(t)


def spmv_model_load(path: str = DEFAULT_MODEL):
    _check("spmv_model_load", lib.spmv_model_load(path.encode()))


def spmv_model_unload():
    _check("spmv_model_unload", lib.spmv_model_unload())


def spmv_mlp_predict(features, feasible_bits: int = 0x3F) -> dict:
    v, fb = _I32(), _I32()
    mg = _F32()
    lg, z = (_F32 * 6)(), (_F32 * 12)()
    _check("spmv_mlp_predict",
           lib.spmv_mlp_predict(_darr(features, _F64), feasible_bits, ctypes.byref(v),
                                ctypes.byref(mg), ctypes.byref(fb), lg, z))
    return {"variant": v.value, "margin": mg.value, "fallback": bool(fb.value),
            "logits": np.array(lg, dtype=np.float32), "z": np.array(z, dtype=np.float32)}


def spmv_mlp_forward_backward(params, Z, labels, mask, B, grads, loss, stream=None):
    _check("spmv_mlp_forward_backward",
           lib.spmv_mlp_forward_backward(_addr(params), _addr(Z), _addr(labels), _addr(mask),
                                         B, _addr(grads), _addr(loss), _stream(stream)))


def spmv_mlp_forward_backward_sets(params, Z, accept, mask, B, grads, loss, stream=None):
    _check("spmv_mlp_forward_backward_sets",
           lib.spmv_mlp_forward_backward_sets(_addr(params), _addr(Z), _addr(accept), _addr(mask), B,
                                              _addr(grads), _addr(loss), _stream(stream)))


def spmv_mlp_adam_step(params, grads, m, v, n, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8,
                       stream=None):
    _check("spmv_mlp_adam_step",
           lib.spmv_mlp_adam_step(_addr(params), _addr(grads), _addr(m), _addr(v), n, step,
                                  lr, b1, b2, eps, _stream(stream)))


# ----------------------------------------------------------------- utilities


def spmv_quantize(src, dst, n, to_dtype, stream=None):
    _check("spmv_quantize", lib.spmv_quantize(_addr(src), _addr(dst), n, to_dtype,
                                              _stream(stream)))


def spmv_generate(family: int, params, seed: int, rowptr, colind=None, val=None,
                  stream=None) -> int:
    p = _darr([int(v) for v in params], _I64)
    nnz = _I64()
    _check("spmv_generate",
           lib.spmv_generate(family, p, len(params), seed, _addr(rowptr), _addr(colind),
                             _addr(val), ctypes.byref(nnz), _stream(stream)))
    return nnz.value


def spmv_generate_vector(n: int, seed: int, x, stream=None):
    _check("spmv_generate_vector", lib.spmv_generate_vector(n, seed, _addr(x), _stream(stream)))


# ------------------------------------------------- the paper's feature classifiers


def _np(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(_P)


def spmv_dtree_fit(X, y, n_classes: int, max_depth: int, min_leaf: int, max_nodes: int | None = None):
    """CART fit on X[n, 12]; returns dict(feature, threshold, left, right, counts) (numpy)."""
    X, px = _np(X, np.float64)
    y, py = _np(y, np.int32)
    n = len(y)
    cap = max_nodes or 2 * n + 1
    out = dict(feature=np.empty(cap, np.int32), threshold=np.empty(cap, np.float64),
               left=np.empty(cap, np.int32), right=np.empty(cap, np.int32),
               counts=np.empty((cap, n_classes), np.int32))
    nn = _I32()
    _check("spmv_dtree_fit", lib.spmv_dtree_fit(
        px, py, n, n_classes, max_depth, min_leaf, cap,
        *(out[k].ctypes.data_as(_P) for k in ("feature", "threshold", "left", "right", "counts")),
        ctypes.byref(nn)))
    return {k: v[:nn.value].copy() for k, v in out.items()}


def spmv_gnb_fit(F, y, n_classes: int):
    """Gaussian naive Bayes fit on raw features F[n, 12]; dict(mu, w, c, count)."""
    F, pf = _np(F, np.float64)
    y, py = _np(y, np.int32)
    out = dict(mu=np.empty((n_classes, 12)), w=np.empty((n_classes, 12)), c=np.empty(n_classes),
               count=np.empty(n_classes, np.int32))
    _check("spmv_gnb_fit", lib.spmv_gnb_fit(pf, py, len(y), n_classes,
                                            *(out[k].ctypes.data_as(_P) for k in ("mu", "w", "c", "count"))))
    return out


def spmv_dtree_load(tree, label_kind: int = SPMV_LABEL_VARIANT):
    arrs = [_np(tree["feature"], np.int32), _np(tree["threshold"], np.float64),
            _np(tree["left"], np.int32), _np(tree["right"], np.int32), _np(tree["counts"], np.int32)]
    counts = np.asarray(tree["counts"])
    _check("spmv_dtree_load", lib.spmv_dtree_load(len(tree["feature"]), counts.shape[1], label_kind,
                                                  *(p for _, p in arrs)))


def spmv_gnb_load(model, label_kind: int = SPMV_LABEL_VARIANT):
    arrs = [_np(model["mu"], np.float64), _np(model["w"], np.float64), _np(model["c"], np.float64),
            _np(model["count"], np.int32)]
    _check("spmv_gnb_load", lib.spmv_gnb_load(len(model["c"]), label_kind, *(p for _, p in arrs)))


def spmv_classifier_unload(which: int):
    _check("spmv_classifier_unload", lib.spmv_classifier_unload(which))


def spmv_classifier_predict(which: int, features, feasible: int = 63) -> dict:
    f = _darr([float(v) for v in features], _F64)
    v, lab, fb, leaf = _I32(), _I32(), _I32(), _I32()
    sc = (_F64 * 8)()
    _check("spmv_classifier_predict", lib.spmv_classifier_predict(
        which, f, feasible, ctypes.byref(v), ctypes.byref(lab), ctypes.byref(fb), ctypes.byref(leaf), sc))
    return dict(variant=v.value, label=lab.value, fallback=bool(fb.value), leaf=leaf.value,
                scores=list(sc))


def spmv_cg(plan, b, x, max_iters: int = 1000, rtol: float = 1e-8, stream=None):
    """Conjugate gradients in place on x; returns (iterations, ||r|| / ||b||)."""
    it, rel = _I32(), _F64()
    _check("spmv_cg", lib.spmv_cg(plan, _addr(b), _addr(x), max_iters, rtol, _stream(stream),
                                  ctypes.byref(it), ctypes.byref(rel)))
    return it.value, rel.value


DTREE_MODEL = os.path.join(_HERE, "dtree_selector.json")
GNB_MODEL = os.path.join(_HERE, "gnb_selector.json")


def load_classifiers(dtree: str = DTREE_MODEL, gnb: str = GNB_MODEL) -> list:
    """Install the stored CART and naive Bayes selectors (for SEL_DTREE / SEL_GNB);
    returns the names of those found."""
    import json
    got = []
    for path, loader, name in ((dtree, spmv_dtree_load, "dtree"), (gnb, spmv_gnb_load, "gnb")):
        if os.path.exists(path):
            with open(path) as f:
                m = json.load(f)
            kind = SPMV_LABEL_VARIANT if m.pop("label_kind") == "variant" else SPMV_LABEL_CLASS
            loader({k: np.asarray(v) for k, v in m.items()}, kind)
            got.append(name)
    return got


def spmv_merge_path_noalloc(n_rows: int, n_cols: int, nnz: int, rowptr, colind, val, val_dtype: int,
                            x, y, stream=None):
    _check("spmv_merge_path_noalloc",
           lib.spmv_merge_path_noalloc(n_rows, n_cols, nnz, _addr(rowptr), _addr(colind), _addr(val),
                                       val_dtype, _addr(x), _addr(y), _stream(stream)))


def spmv_release_cached_blocks():
    _check("spmv_release_cached_blocks", lib.spmv_release_cached_blocks())


def spmv_cache_flush(stream=None):
    _check("spmv_cache_flush", lib.spmv_cache_flush(_stream(stream)))


def spmv_hbm_probe(nbytes: int = 4 << 30):
    r, c = _F64(), _F64()
    _check("spmv_hbm_probe", lib.spmv_hbm_probe(nbytes, ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def spmv_gather_probe(window_elems: int, elem_bytes: int, windows: int, gathers: int) -> float:
    """Median time (s) of `gathers` random reads from per-XCD windows (see the header)."""
    t = _F64()
    _check("spmv_gather_probe", lib.spmv_gather_probe(window_elems, elem_bytes, windows, gathers,
                                                      ctypes.byref(t)))
    return t.value


def spmv_gather_probe2(window_elems: int, elem_bytes: int, windows: int, gathers: int,
                       indexed: bool) -> float:
    """Median time (s) of the gather ceiling, with the indices streamed when ``indexed``."""
    t = _F64()
    _check("spmv_gather_probe2", lib.spmv_gather_probe2(window_elems, elem_bytes, windows, gathers,
                                                        int(indexed), ctypes.byref(t)))
    return t.value


def load_selector_config(path: str = SELECTOR_CONFIG) -> bool:
    """Set the profiling thresholds calibrated for this GPU, if the file exists."""
    if not os.path.exists(path):
        return False
    import json
    with open(path) as f:
        spmv_set_thresholds(json.load(f)["theta"])
    return True


load_selector_config()


# ------------------------------------------------------------ convenience


class Plan:
    """Owns a plan handle and keeps the borrowed CSR tensors alive."""

    def __init__(self, rowptr, colind, val, n_cols, val_dtype=SPMV_F64, stream=None, flags=0,
                 nnz=None):
        self._keep = (rowptr, colind, val)
        self.n = int(rowptr.numel()) - 1
        self.m = int(n_cols)
        self.nnz = int(colind.numel()) if nnz is None else int(nnz)
        self.dtype = val_dtype
        self.handle = spmv_plan_create(self.n, self.m, self.nnz, rowptr, colind, val,
                                       val_dtype, stream, flags)

    def close(self):
        if self.handle:
            spmv_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def features(self):
        return spmv_features(self.handle)

    def select(self, selector=SEL_MLP):
        return spmv_select(self.handle, selector)

    def set_variant(self, v):
        spmv_set_variant(self.handle, v)

    def set_delta16_layout(self, layout):
        spmv_set_delta16_layout(self.handle, layout)

    def set_delta16_sort(self, mode):
        spmv_set_delta16_sort(self.handle, mode)

    def set_delta16_offset_bits(self, bits):
        spmv_set_delta16_offset_bits(self.handle, bits)

    @property
    def variant(self):
        return spmv_get_variant(self.handle)

    def mask(self):
        return spmv_variant_mask(self.handle)

    def _check_vector(self, t, length, what):
        """Reject a torch vector the plan would read or write out of bounds or
        misread: wrong dtype for the plan's value type, too short, not
        contiguous or not on a GPU.  Raw addresses (ints) are passed as given."""
        if isinstance(t, int) or t is None:
            return
        want = "torch.float64" if self.dtype == SPMV_F64 else "torch.float32"
        if str(t.dtype) != want:
            raise ValueError(f"{what} must be {want} for this plan, got {t.dtype}")
        if t.numel() < length:
            raise ValueError(f"{what} has {t.numel()} elements, the plan needs {length}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if t.device.type != "cuda":
            raise ValueError(f"{what} must be a device tensor, got {t.device}")

    def execute(self, x, y, stream=None):
        self._check_vector(x, self.m if self.nnz > 0 else 0, "x")
        self._check_vector(y, self.n, "y")
        spmv_execute(self.handle, x, y, stream)

    def bytes(self, v=None):
        return spmv_bytes(self.handle, self.variant if v is None else v)

    def time(self, v, reps=10, cold=False):
        return spmv_time_variant(self.handle, v, reps, cold)

    def query(self, key):
        return spmv_plan_query(self.handle, key)
