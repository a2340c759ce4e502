"""ctypes wrapper of ``csrc/spmv_ref.c`` (test infrastructure: host timing).

``build()`` compiles the C file into ``oracle/libspmv_ref.so`` with
``gcc -O2 -ffp-contract=off -fopenmp``.  Besides the timed loop it holds
the full-size accuracy reference (``dot2``: every row by Ogita, Rump and
Oishi's Dot2, with the row scales) and a row-parallel copy of the plain
sequential loop (``seq``), so whole vectors of the class matrices can be
checked in seconds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "spmv_ref.c")
LIB = os.path.join(HERE, "libspmv_ref.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.spmv_ref_f64.argtypes = [ctypes.c_int64, P, P, P, P, P]
        lib.spmv_ref_f64.restype = None
        lib.spmv_ref_f64_omp.argtypes = [ctypes.c_int64, P, P, P, P, P]
        lib.spmv_ref_f64_omp.restype = ctypes.c_int
        lib.spmv_ref_dot2.argtypes = [ctypes.c_int64, P, P, P, P, P, P]
        lib.spmv_ref_dot2.restype = None
        lib.spmv_ref_seq_par.argtypes = [ctypes.c_int64, P, P, P, P, P]
        lib.spmv_ref_seq_par.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def spmv(rowptr, colind, val, x, threads: bool = False):
    """y = A x with the plain C loop; returns (y, threads_used)."""
    lib = load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = len(rowptr) - 1
    y = np.empty(n, dtype=np.float64)
    if threads:
        used = lib.spmv_ref_f64_omp(n, _ptr(rowptr), _ptr(colind), _ptr(val), _ptr(x), _ptr(y))
    else:
        lib.spmv_ref_f64(n, _ptr(rowptr), _ptr(colind), _ptr(val), _ptr(x), _ptr(y))
        used = 1
    return y, used


def _csr(rowptr, colind, val, x):
    return (np.ascontiguousarray(rowptr, dtype=np.int32), np.ascontiguousarray(colind, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64), np.ascontiguousarray(x, dtype=np.float64))


def dot2(rowptr, colind, val, x):
    """(y_ref, scale): every row by Dot2 (error at most u|y_i| + gamma_L^2 scale_i)
    and scale_i = sum_j |a_ij| |x_j|."""
    lib = load()
    rowptr, colind, val, x = _csr(rowptr, colind, val, x)
    n = len(rowptr) - 1
    y = np.empty(n, dtype=np.float64)
    s = np.empty(n, dtype=np.float64)
    lib.spmv_ref_dot2(n, _ptr(rowptr), _ptr(colind), _ptr(val), _ptr(x), _ptr(y), _ptr(s))
    return y, s


def seq(rowptr, colind, val, x):
    """Algorithm 1's sequential sum for every row (rows in parallel)."""
    lib = load()
    rowptr, colind, val, x = _csr(rowptr, colind, val, x)
    n = len(rowptr) - 1
    y = np.empty(n, dtype=np.float64)
    lib.spmv_ref_seq_par(n, _ptr(rowptr), _ptr(colind), _ptr(val), _ptr(x), _ptr(y))
    return y
