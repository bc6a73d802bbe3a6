"""Loader of the plain OpenMP CSR product in ``spmv.c`` (test
infrastructure: the benchmark's CPU baseline).  ``build()`` compiles it with
gcc next to the source."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmv.c")
LIB = os.path.join(HERE, "libspmv.so")


def build() -> str:
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"], check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _lib():
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    lib.oracle_csr_spmv.restype = ctypes.c_int
    lib.oracle_csr_spmv.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5
    return lib


def spmv(A, x, y=None):
    """y = A x for a SciPy CSR matrix with int64 indptr / int32 indices
    (converted if needed); returns (y, threads used)."""
    if A.indptr.dtype != np.int64:
        A.indptr = A.indptr.astype(np.int64)
    if A.indices.dtype != np.int32:
        A.indices = A.indices.astype(np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if y is None:
        y = np.empty(A.shape[0])
    used = _lib().oracle_csr_spmv(A.shape[0], A.indptr.ctypes.data, A.indices.ctypes.data,
                                  A.data.ctypes.data, x.ctypes.data, y.ctypes.data)
    return y, used
