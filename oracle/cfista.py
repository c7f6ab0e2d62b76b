"""FISTA of ``oracle.fista`` in plain C with OpenMP (``fista_omp.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The iteration of section 8.1 (FISTA, x_0 = 0, y_1 = x_0, t_1 = 1) over the
CSR of A and of A^T, FP64, the rows of each product split over host
threads.  Sums run in index order within a row and every row belongs to one
thread, so the iterates equal ``oracle.fista.fista`` on scipy's CSR products
bit for bit, at any thread count.  The library is compiled from source with
gcc on first use (or by ``__graft_entry__.build``).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fista_omp.c")
LIB = os.path.join(HERE, "_build", "liboracle_fista_omp.so")

_lib = None


def build():
    """Compile fista_omp.c (gcc, -O2 -fopenmp, no FMA contraction)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"],
                   check=True)
    os.replace(tmp, LIB)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = ctypes.CDLL(LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        _lib.oracle_fista_csr.argtypes = [i64, i64, p, p, p, p, p, p, p, ctypes.c_double, ctypes.c_double, i64, p,
                                          ctypes.c_int]
        _lib.oracle_fista_csr.restype = ctypes.c_int
        _lib.oracle_threads.restype = ctypes.c_int
    return _lib


def _csr_arrays(M):
    M = M.tocsr()
    M.sort_indices()
    return (np.ascontiguousarray(M.indptr, dtype=np.int64), np.ascontiguousarray(M.indices, dtype=np.int32),
            np.ascontiguousarray(M.data, dtype=np.float64))


class CsrPair:
    """A (m x n) and A^T as CSR arrays, prepared once for repeated solves."""

    def __init__(self, A):
        self.m, self.n = A.shape
        self.a = _csr_arrays(A)
        self.t = _csr_arrays(A.T)


def fista(pair, b, tau, L, iters, x0=None, threads=0):
    """x_iters of FISTA (section 8.1) from x0 (default 0); threads <= 0: the
    OpenMP default."""
    x = np.zeros(pair.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    b = np.ascontiguousarray(b, dtype=np.float64)
    (rp, ci, v), (tp, ti, tv) = pair.a, pair.t
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    st = lib().oracle_fista_csr(pair.m, pair.n, ptr(rp), ptr(ci), ptr(v), ptr(tp), ptr(ti), ptr(tv), ptr(b),
                                float(tau), float(L), int(iters), ptr(x), int(threads))
    if st != 0:
        raise MemoryError("oracle_fista_csr: out of host memory")
    return x


def max_threads():
    return int(lib().oracle_threads())
