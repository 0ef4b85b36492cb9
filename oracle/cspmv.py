"""ctypes front of ``spmv.c``: the oracle's assembled operators multiplied on
all host cores (OpenMP), for the host timing beside scipy's single-threaded
product.  Test infrastructure; ``build()`` compiles the C file in place."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmv.c")
LIB = os.path.join(HERE, "libspmv.so")
_lib = None


def build():
    """gcc -O3 -fopenmp -shared spmv.c -> libspmv.so (next to the source)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: run oracle.cspmv.build()")
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.oracle_csr_spmv.argtypes = [ctypes.c_int32, P, P, P, P, P]
        lib.oracle_csr_spmv.restype = None
        lib.oracle_csr_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads():
    return _load().oracle_csr_threads()


def spmv(A, x, y=None):
    """y = A x for a scipy CSR matrix with 32-bit indices and FP64 values."""
    A = A.tocsr()
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int32)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.shape[0]) if y is None else y
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _load().oracle_csr_spmv(A.shape[0], ptr(indptr), ptr(indices), ptr(data), ptr(x), ptr(y))
    return y
