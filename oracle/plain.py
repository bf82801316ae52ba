"""ctypes wrapper of the plain binary64 implementation of the paper's
algorithms (``eig3_plain.c``; see that file for the algorithm citations and
the readings taken).  TEST INFRASTRUCTURE: see ``oracle/__init__.py``.

All arrays are float64 NumPy arrays; matrices are (n, 9) row-major or
(n, 3, 3).  ``threads=0`` means the OpenMP default (all host cores)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

_D = ctypes.POINTER(ctypes.c_double)


def _mat(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 9))


def _p(x: np.ndarray):
    return x.ctypes.data_as(_D)


class PlainOracle:
    """The functions of one build of ``eig3_plain.c`` (``lib_path``)."""

    def __init__(self, lib_path: str):
        lib = ctypes.CDLL(lib_path)
        i64, i32 = ctypes.c_int64, ctypes.c_int
        lib.oracle_invariants.argtypes = [i64, _D, _D, _D, _D, _D, i32]
        lib.oracle_eigvals.argtypes = [i64, _D, _D, i32]
        lib.oracle_eigvals_from_invariants.argtypes = [i64, _D, _D, _D, _D, _D]
        lib.oracle_eigvals_backward.argtypes = [i64, _D, _D, _D, i32]
        lib.oracle_aux_vectors.argtypes = [_D, _D, _D]
        lib.oracle_naive.argtypes = [i64, _D, i32, _D, _D]
        lib.oracle_max_threads.restype = ctypes.c_int
        self.lib = lib
        self.path = lib_path

    def max_threads(self) -> int:
        return int(self.lib.oracle_max_threads())

    def invariants(self, a, threads: int = 0):
        """(I1, J2, J3, Delta), each shape (n,)."""
        a = _mat(a)
        n = a.shape[0]
        outs = [np.empty(n) for _ in range(4)]
        self.lib.oracle_invariants(n, _p(a), *map(_p, outs), threads)
        return tuple(outs)

    def eigvals(self, a, threads: int = 0) -> np.ndarray:
        """Ascending eigenvalues, shape (n, 3)."""
        a = _mat(a)
        lam = np.empty((a.shape[0], 3))
        self.lib.oracle_eigvals(a.shape[0], _p(a), _p(lam), threads)
        return lam

    def eigvals_from_invariants(self, i1, j2, j3, disc) -> np.ndarray:
        """Alg. alg:eigvals-stable alone, from given invariants."""
        arrs = [np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel()) for x in (i1, j2, j3, disc)]
        n = arrs[0].shape[0]
        lam = np.empty((n, 3))
        self.lib.oracle_eigvals_from_invariants(n, *map(_p, arrs), _p(lam))
        return lam

    def eigvals_backward(self, a, g, threads: int = 0) -> np.ndarray:
        """sum_k g_k d(lambda_k)/dA, shape (n, 9) row-major."""
        a = _mat(a)
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1, 3))
        if g.shape[0] != a.shape[0]:
            raise ValueError("g must have one row of 3 per matrix")
        grad = np.empty_like(a)
        self.lib.oracle_eigvals_backward(a.shape[0], _p(a), _p(g), _p(grad), threads)
        return grad

    def naive(self, a, variant: str):
        """The paper's comparators: variant "naive" (Alg. alg:J2-naive,
        alg:J3-naive) or "tensor" (Alg. alg:J2-tensor, alg:J3-tensor), with
        Delta = 4 J2^3 - 27 J3^2 and Alg. alg:eigvals-stable.  Returns
        (invariants (n, 4), eigenvalues (n, 3))."""
        a = _mat(a)
        n = a.shape[0]
        inv = np.empty((n, 4))
        lam = np.empty((n, 3))
        v = {"naive": 1, "tensor": 2}[variant]
        self.lib.oracle_naive(n, _p(a), v, _p(inv), _p(lam))
        return inv, lam

    def aux_vectors(self, a9):
        """u = dx(A), v = dx(A^T) of one matrix (Alg. alg:disc-stable)."""
        a = _mat(a9)[0].copy()
        u, v = np.empty(14), np.empty(14)
        self.lib.oracle_aux_vectors(_p(a), _p(u), _p(v))
        return u, v


_default: PlainOracle | None = None


def _load() -> PlainOracle:
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build()
        _default = PlainOracle(LIB)
    return _default


def max_threads() -> int:
    return _load().max_threads()


def invariants(a, threads: int = 0):
    return _load().invariants(a, threads)


def eigvals(a, threads: int = 0):
    return _load().eigvals(a, threads)


def eigvals_from_invariants(i1, j2, j3, disc):
    return _load().eigvals_from_invariants(i1, j2, j3, disc)


def eigvals_backward(a, g, threads: int = 0):
    return _load().eigvals_backward(a, g, threads)


def aux_vectors(a9):
    return _load().aux_vectors(a9)


def naive(a, variant: str):
    return _load().naive(a, variant)
