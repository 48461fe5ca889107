"""Host-parallel CSR SpMV of the oracle's assembled tangent (oracle, test
infrastructure only): the matrix-based CPU baseline on all host cores, next to
SciPy's single-threaded product.  ``build()`` compiles oracle/spmv.c with gcc
into oracle/libspmv.so; ``spmv(K, x)`` equals ``K @ x`` up to summation order.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmv.c")
LIB = os.path.join(HERE, "libspmv.so")
_lib = None


def build():
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC], check=True)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.oracle_spmv.argtypes = [ctypes.c_int64, P, P, P, P, P]
        L.oracle_spmv.restype = None
        L.oracle_spmv_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def threads():
    return _load().oracle_spmv_threads()


def prepare(K):
    """CSR arrays of the scipy matrix in the C layout (int64 row pointers)."""
    K = K.tocsr()
    return (K.shape[0], np.ascontiguousarray(K.indptr, dtype=np.int64),
            np.ascontiguousarray(K.indices, dtype=np.int32), np.ascontiguousarray(K.data, dtype=np.float64))


def spmv(csr, x, y=None):
    n, rp, col, val = csr
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n) if y is None else y
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _load().oracle_spmv(n, p(rp), p(col), p(val), p(x), p(y))
    return y
