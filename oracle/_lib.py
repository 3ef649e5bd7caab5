"""Builds and loads the oracle's one C routine (oracle/laplacian_apply.c).

The library is compiled with gcc, -O2, no -march, -ffp-contract=off (no fused
multiply-add, so every product and sum is a separately rounded IEEE FP64
operation), and OpenMP.  It lives in oracle/_build/ and shares nothing with the
GPU library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "laplacian_apply.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_SO = os.path.join(_OUT_DIR, "liboracle_laplacian.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C code.  Returns the path of the shared library."""
    if not force and os.path.exists(_SO):
        return _SO
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-std=c11", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        L.oracle_apply_laplacian.argtypes = [i64, p, p, p, p, i64, i64, p, i64, i64, i64]
        L.oracle_apply_laplacian.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def apply_laplacian(csr, X: np.ndarray, out: np.ndarray | None = None) -> np.ndarray:
    """Y = A X for A = I - D^{-1/2} S D^{-1/2}; X is (n,) or (n, w) float64 in any
    memory order."""
    X = np.asarray(X)
    if X.dtype != np.float64:
        raise TypeError("oracle works in float64")
    vec = X.ndim == 1
    X2 = X.reshape(-1, 1) if vec else X
    n, w = X2.shape
    if n != csr.n:
        raise ValueError("row count mismatch")
    if out is None:
        out = np.empty((n, w), dtype=np.float64, order="F" if X2.flags.f_contiguous and not
                       X2.flags.c_contiguous else "C")
    Y2 = out.reshape(-1, 1) if out.ndim == 1 else out
    isz = 8
    rc = lib().oracle_apply_laplacian(
        n, csr.row_ptr.ctypes.data, csr.col.ctypes.data, csr.dinv.ctypes.data,
        X2.ctypes.data, X2.strides[0] // isz, X2.strides[1] // isz,
        Y2.ctypes.data, Y2.strides[0] // isz, Y2.strides[1] // isz, w)
    if rc != 0:
        raise MemoryError("oracle_apply_laplacian failed")
    return out.reshape(-1) if vec else out
