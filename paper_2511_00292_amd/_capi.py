"""ctypes binding of libeig3 (include/eig3.h): argument marshalling only.

Every computation happens in the HIP kernels of ``libeig3.so``.  There is no
fallback: if the library is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# EIG3_LIBRARY may name another build of the same sources (A/B timing of
# build-time knobs); by default the in-tree build next to this file is used
LIB_PATH = os.environ.get("EIG3_LIBRARY") or os.path.join(HERE, "libeig3.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "eig3.h")

# enums of include/eig3.h
EIG3_OK, EIG3_EINVAL, EIG3_EUNSUPPORTED, EIG3_ELAUNCH = 0, -1, -2, -3
EIG3_F64, EIG3_F32 = 0, 1
EIG3_GENERAL, EIG3_SYMMETRIC = 0, 1
EIG3_SOA, EIG3_AOS = 0, 1
EIG3_FMA, EIG3_COMPENSATED, EIG3_NAIVE, EIG3_NAIVE_TENSOR, EIG3_DOUBLE_WORD = 0, 1, 2, 3, 4


class Eig3Matrices(ctypes.Structure):
    """struct eig3_matrices"""
    _fields_ = [
        ("n", ctypes.c_int64),
        ("dtype", ctypes.c_int32),
        ("structure", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("accuracy", ctypes.c_int32),
        ("a", ctypes.c_void_p * 9),
    ]


class Eig3Error(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libeig3.so is not built ({LIB_PATH}); run `python -c 'import __graft_entry__ as g; g.build()'`"
                " or `python paper_2511_00292_amd/build.py`")
        l = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        pm = ctypes.POINTER(Eig3Matrices)
        l.eig3_invariants.argtypes = [pm, vp, vp, vp, vp, vp]
        l.eig3_invariants.restype = ctypes.c_int
        l.eig3_eigvals.argtypes = [pm, ctypes.c_int32, ctypes.POINTER(vp), vp]
        l.eig3_eigvals.restype = ctypes.c_int
        l.eig3_eigvals_backward.argtypes = [pm, ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        l.eig3_eigvals_backward.restype = ctypes.c_int
        l.eig3_mohr_coulomb.argtypes = [pm, ctypes.c_double, ctypes.c_double, vp, ctypes.POINTER(vp), vp]
        l.eig3_mohr_coulomb.restype = ctypes.c_int
        l.eig3_eigenprojectors.argtypes = [pm, ctypes.c_int32, ctypes.POINTER(vp), vp]
        l.eig3_eigenprojectors.restype = ctypes.c_int
        l.eig3_matrix_function.argtypes = [pm, ctypes.c_int32, ctypes.POINTER(vp), vp]
        l.eig3_matrix_function.restype = ctypes.c_int
        l.eig3_matrix_function_backward.argtypes = [pm, ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        l.eig3_matrix_function_backward.restype = ctypes.c_int
        l.eig3_status_string.argtypes = [ctypes.c_int]
        l.eig3_status_string.restype = ctypes.c_char_p
        l.eig3_version.argtypes = []
        l.eig3_version.restype = ctypes.c_char_p
        l.eig3_soa_stride.argtypes = [ctypes.c_int64, ctypes.c_int32]
        l.eig3_soa_stride.restype = ctypes.c_int64
        _lib = l
    return _lib


def status_string(status: int) -> str:
    return lib().eig3_status_string(int(status)).decode()


def version() -> str:
    return lib().eig3_version().decode()


def soa_stride(n: int, dtype: int) -> int:
    s = lib().eig3_soa_stride(int(n), int(dtype))
    if s < 0:
        raise Eig3Error(EIG3_EINVAL, "eig3_soa_stride")
    return s


def declared_functions() -> list[str]:
    """Names of the functions declared in include/eig3.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(eig3_\w+)\s*\(", text, re.M)))


def call_invariants(m: Eig3Matrices, outs, stream: int) -> None:
    st = lib().eig3_invariants(ctypes.byref(m), *[ctypes.c_void_p(p) for p in outs], ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_invariants")


def call_eigvals(m: Eig3Matrices, out_layout: int, outs, stream: int) -> None:
    arr = (ctypes.c_void_p * 3)(*outs)
    st = lib().eig3_eigvals(ctypes.byref(m), out_layout, arr, ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_eigvals")


def call_eigvals_backward(m: Eig3Matrices, g_layout: int, g, grads, stream: int) -> None:
    garr = (ctypes.c_void_p * 3)(*g)
    oarr = (ctypes.c_void_p * 9)(*grads)
    st = lib().eig3_eigvals_backward(ctypes.byref(m), g_layout, garr, oarr, ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_eigvals_backward")


def call_mohr_coulomb(m: Eig3Matrices, s_yc: float, mm: float, f: int, grads, stream: int) -> None:
    arr = (ctypes.c_void_p * 9)(*grads) if grads is not None else None
    st = lib().eig3_mohr_coulomb(ctypes.byref(m), float(s_yc), float(mm), ctypes.c_void_p(f), arr,
                                 ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_mohr_coulomb")


def call_matrix_function(m: Eig3Matrices, fn: int, outs, stream: int) -> None:
    arr = (ctypes.c_void_p * 9)(*outs)
    st = lib().eig3_matrix_function(ctypes.byref(m), fn, arr, ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_matrix_function")


def call_matrix_function_backward(m: Eig3Matrices, fn: int, g, outs, stream: int) -> None:
    garr = (ctypes.c_void_p * 9)(*g)
    arr = (ctypes.c_void_p * 9)(*outs)
    st = lib().eig3_matrix_function_backward(ctypes.byref(m), fn, garr, arr, ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_matrix_function_backward")


def call_eigenprojectors(m: Eig3Matrices, out_layout: int, outs, stream: int) -> None:
    arr = (ctypes.c_void_p * 27)(*outs)
    st = lib().eig3_eigenprojectors(ctypes.byref(m), out_layout, arr, ctypes.c_void_p(stream))
    if st != EIG3_OK:
        raise Eig3Error(st, "eig3_eigenprojectors")
