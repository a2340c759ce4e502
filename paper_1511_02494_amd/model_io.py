"""Reader and writer of the MLP selector's parameter file.

Layout (little endian): b"SPMVMLP1", u32 version = 1, u32 n_params = 5382,
f32 mu[12], f32 rho[12], f32 tau, f32 params[5382], u32 CRC-32 (IEEE 802.3,
as zlib.crc32) of every preceding byte.  ``spmv_model_load`` reads the same
layout.
"""
from __future__ import annotations

import struct
import zlib

import numpy as np

MAGIC = b"SPMVMLP1"
N_PARAMS = 5382


def write_model(path: str, params, mu, rho, tau: float) -> None:
    params = np.asarray(params, dtype="<f4")
    assert params.shape == (N_PARAMS,)
    body = (MAGIC + struct.pack("<II", 1, N_PARAMS)
            + np.asarray(mu, dtype="<f4").tobytes() + np.asarray(rho, dtype="<f4").tobytes()
            + struct.pack("<f", float(tau)) + params.tobytes())
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def read_model(path: str):
    with open(path, "rb") as f:
        data = f.read()
    body, crc = data[:-4], struct.unpack("<I", data[-4:])[0]
    if data[:8] != MAGIC or zlib.crc32(body) & 0xFFFFFFFF != crc:
        raise ValueError(f"{path}: not a valid model file")
    mu = np.frombuffer(body, "<f4", 12, 16)
    rho = np.frombuffer(body, "<f4", 12, 64)
    tau = struct.unpack("<f", body[112:116])[0]
    params = np.frombuffer(body, "<f4", N_PARAMS, 116)
    return params.copy(), mu.copy(), rho.copy(), tau
