"""ctypes wrapper of oracle/spmv_c.c (test infrastructure: timing only)."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmv_c.c")
LIB = os.path.join(HERE, "libspmv_c.so")


def build(verbose=False):
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", SRC, "-o", LIB]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.csr_spmv_z.restype = None
        _lib.csr_spmv_z.argtypes = [C.c_int64] + [C.c_void_p] * 5
        _lib.csr_threads.restype = C.c_int
    return _lib


def threads():
    return _load().csr_threads()


def spmv(A, x, y=None):
    """y = A x for a scipy CSR matrix A (complex128), on all OpenMP threads."""
    lib = _load()
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int64)
    data = np.ascontiguousarray(A.data, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    if y is None:
        y = np.empty(A.shape[0], dtype=np.complex128)
    lib.csr_spmv_z(A.shape[0], indptr.ctypes.data, indices.ctypes.data, data.ctypes.data, x.ctypes.data,
                   y.ctypes.data)
    return y
