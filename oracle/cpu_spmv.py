"""ctypes wrapper of ``cpu_spmv.c``: the threaded FP64 CSR product y = A u
(the matrix-based comparison of Sec. 3.2) used as the CPU baseline.

TEST INFRASTRUCTURE ONLY (tests and the CPU-baseline leg of the benchmark).
The shared library ``libcpu_spmv.so`` is compiled next to the source by the
repository's build step (gcc -O3 -fopenmp); nothing here compiles it."""
import ctypes
import os

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpu_spmv.so")
SOURCE = os.path.join(_HERE, "cpu_spmv.c")
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (the repository build compiles {SOURCE})")
        L = ctypes.CDLL(LIB_PATH)
        L.spmv_create.restype = ctypes.c_void_p
        L.spmv_create.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 4
        L.spmv_destroy.argtypes = [ctypes.c_void_p]
        L.spmv_apply.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.spmv_time.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        L.spmv_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


class CsrSpmv:
    """A square scipy sparse matrix and an input vector copied into the C
    product's first-touch buffers."""

    def __init__(self, A, u):
        A = sp.csr_matrix(A)
        if A.shape[0] != A.shape[1]:
            raise ValueError("square matrix expected")
        self.n = A.shape[0]
        ptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        col = np.ascontiguousarray(A.indices, dtype=np.int32)
        val = np.ascontiguousarray(A.data, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.shape != (self.n,):
            raise ValueError("u has the wrong length")
        self.nnz = int(ptr[-1])
        self._h = _lib().spmv_create(self.n, ptr.ctypes.data, col.ctypes.data, val.ctypes.data, u.ctypes.data)
        if not self._h:
            raise MemoryError("spmv_create: allocation failed")

    def __del__(self):
        if getattr(self, "_h", None):
            _lib().spmv_destroy(self._h)
            self._h = None

    def apply(self):
        y = np.empty(self.n, dtype=np.float64)
        _lib().spmv_apply(self._h, y.ctypes.data)
        return y

    def time(self, warmup=3, runs=20):
        """Seconds of each of `runs` products after `warmup` untimed ones."""
        t = np.empty(runs, dtype=np.float64)
        _lib().spmv_time(self._h, int(warmup), int(runs), t.ctypes.data)
        return t

    @staticmethod
    def threads():
        return int(_lib().spmv_threads())
