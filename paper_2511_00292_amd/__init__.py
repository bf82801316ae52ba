"""Batched closed-form eigenvalues of real, diagonalizable 3x3 matrices on
AMD Instinct MI355X (gfx950), after Habera & Zilian, "Numerically stable
evaluation of closed-form expressions for eigenvalues of 3x3 matrices"
(arXiv 2511.00292).

The three calls below mirror the C ABI of ``include/eig3.h`` one for one and
only marshal arguments: PyTorch provides device memory and the current
stream; all arithmetic runs in the HIP kernels of ``libeig3.so``.

Matrix batches are given either as a sequence of K device tensors of n
values each (structure of arrays, K = 9 general / 6 symmetric, in the entry
order of ``ENTRIES``) or as one device tensor with n*K values (array of
structures, e.g. a contiguous (n, 3, 3) tensor for general matrices or
(n, 6) for symmetric ones).
"""
from __future__ import annotations

from typing import Sequence, Union

import torch

from . import _capi
from ._capi import (EIG3_AOS, EIG3_COMPENSATED, EIG3_DOUBLE_WORD, EIG3_F32, EIG3_F64, EIG3_FMA, EIG3_GENERAL,
                    EIG3_NAIVE, EIG3_NAIVE_TENSOR, EIG3_SOA, EIG3_SYMMETRIC, Eig3Error)

__all__ = [
    "eig3_invariants", "eig3_eigvals", "eig3_eigvals_backward", "eig3_mohr_coulomb", "eig3_eigenprojectors",
    "eig3_matrix_function", "eig3_matrix_function_backward", "eigvals", "eigvals_symmetric", "matrix_function",
    "matrix_function_symmetric", "Eig3Eigvals", "Eig3EigvalsSymmetric", "Eig3MatrixFunction",
    "Eig3MatrixFunctionSymmetric",
    "ENTRIES", "Eig3Error", "version", "soa_stride", "empty_soa",
]

ENTRIES = {
    "general": ("A00", "A01", "A02", "A10", "A11", "A12", "A20", "A21", "A22"),
    "symmetric": ("A00", "A11", "A22", "A01", "A02", "A12"),
}

_STRUCT = {"general": EIG3_GENERAL, "symmetric": EIG3_SYMMETRIC}
_ACC = {"fma": EIG3_FMA, "compensated": EIG3_COMPENSATED, "naive": EIG3_NAIVE, "naive_tensor": EIG3_NAIVE_TENSOR,
        "double_word": EIG3_DOUBLE_WORD}
_DTYPE = {torch.float64: EIG3_F64, torch.float32: EIG3_F32}
_FN = {"exp": 0, "log": 1, "sqrt": 2}  # eig3_function

Batch = Union[torch.Tensor, Sequence[torch.Tensor]]


def version() -> str:
    return _capi.version()


def soa_stride(n: int, dtype=torch.float64) -> int:
    """eig3_soa_stride: the recommended distance, in elements, between
    consecutive arrays of a structure-of-arrays batch of n matrices held in
    one allocation (see include/eig3.h)."""
    if dtype not in _DTYPE:
        raise TypeError("dtype must be torch.float64 or torch.float32")
    return _capi.soa_stride(n, _DTYPE[dtype])


def empty_soa(n: int, count: int, dtype=torch.float64, device=None) -> list:
    """count uninitialised arrays of n values in one device allocation,
    array k at element k * soa_stride(n, dtype): the placement the library
    recommends for structure-of-arrays batches and their outputs.  The arrays
    are views of one buffer, which stays allocated while any of them is
    alive."""
    stride = soa_stride(n, dtype)
    buf = torch.empty(count * stride, dtype=dtype, device=device)
    return [buf[k * stride: k * stride + n] for k in range(count)]


def _check_device_tensor(t: torch.Tensor, what: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _check_out(t: torch.Tensor, numel: int, dtype, device, what: str) -> None:
    """Output tensors receive raw device writes of numel values: their size,
    dtype and device are checked here (the C ABI cannot see them)."""
    _check_device_tensor(t, what)
    if t.numel() != numel or t.dtype != dtype or t.device != device:
        raise ValueError(f"{what} needs {numel} values of {dtype} on {device}")


def _out_list(out, count: int, n: int, dtype, device, what: str) -> list:
    res = list(out) if out is not None else empty_soa(n, count, dtype, device)
    if len(res) != count:
        raise ValueError(f"{what} needs {count} tensors")
    for j, t in enumerate(res):
        _check_out(t, n, dtype, device, f"{what}[{j}]")
    return res


def _matrices(a: Batch, structure: str, accuracy: str):
    """Build the eig3_matrices descriptor; returns (descriptor, n, dtype,
    device, layout, keepalive)."""
    if structure not in _STRUCT:
        raise ValueError(f"structure must be one of {tuple(_STRUCT)}")
    if accuracy not in _ACC:
        raise ValueError(f"accuracy must be one of {tuple(_ACC)}")
    k = 9 if structure == "general" else 6
    m = _capi.Eig3Matrices()
    m.structure = _STRUCT[structure]
    m.accuracy = _ACC[accuracy]
    if isinstance(a, torch.Tensor):
        _check_device_tensor(a, "a")
        if a.numel() % k:
            raise ValueError(f"array-of-structures input needs a multiple of {k} values")
        n = a.numel() // k
        m.layout = EIG3_AOS
        m.a[0] = a.data_ptr() if n else 0
        ts = [a]
    else:
        ts = list(a)
        if len(ts) != k:
            raise ValueError(f"structure-of-arrays input needs {k} tensors for '{structure}'")
        for j, t in enumerate(ts):
            _check_device_tensor(t, f"a[{j}]")
        n = ts[0].numel()
        if any(t.numel() != n for t in ts) or any(t.dtype != ts[0].dtype for t in ts) or \
                any(t.device != ts[0].device for t in ts):
            raise ValueError("all entry tensors need the same length, dtype and device")
        m.layout = EIG3_SOA
        for j, t in enumerate(ts):
            m.a[j] = t.data_ptr() if n else 0
    dtype = ts[0].dtype
    if dtype not in _DTYPE:
        raise TypeError("matrices must be float64 or float32")
    m.dtype = _DTYPE[dtype]
    m.n = n
    return m, n, dtype, ts[0].device, m.layout, ts


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def eig3_invariants(a: Batch, structure: str = "general", accuracy: str = "double_word", out=None):
    """(I1, J2, J3, Delta), each a tensor of n values (Alg. alg:I1-stable,
    alg:J2-stable, alg:J3-stable, alg:disc-stable)."""
    m, n, dtype, dev, _, _keep = _matrices(a, structure, accuracy)
    outs = _out_list(out, 4, n, dtype, dev, "out")
    _capi.call_invariants(m, [t.data_ptr() if n else 0 for t in outs], _stream(dev))
    return tuple(outs)


def eig3_eigvals(a: Batch, structure: str = "general", accuracy: str = "double_word", out_layout: str = "aos", out=None):
    """Ascending eigenvalues (Alg. alg:eigvals-stable).  out_layout 'aos'
    returns an (n, 3) tensor, 'soa' a tuple of three n-vectors."""
    m, n, dtype, dev, _, _keep = _matrices(a, structure, accuracy)
    if out_layout == "aos":
        res = out if out is not None else torch.empty((n, 3), dtype=dtype, device=dev)
        _check_out(res, 3 * n, dtype, dev, "out")
        ptrs = [res.data_ptr() if n else 0, 0, 0]
        _capi.call_eigvals(m, EIG3_AOS, ptrs, _stream(dev))
        return res
    if out_layout == "soa":
        res = _out_list(out, 3, n, dtype, dev, "out")
        _capi.call_eigvals(m, EIG3_SOA, [t.data_ptr() if n else 0 for t in res], _stream(dev))
        return tuple(res)
    raise ValueError("out_layout must be 'aos' or 'soa'")


def eig3_eigvals_backward(a: Batch, g: Batch, structure: str = "general", accuracy: str = "double_word", out=None):
    """sum_k g_k d(lambda_k)/dA, in the structure and layout of ``a``.
    ``g``: an (n, 3) tensor (array of structures) or three n-vectors."""
    m, n, dtype, dev, layout, _keep = _matrices(a, structure, accuracy)
    k = 9 if structure == "general" else 6
    if isinstance(g, torch.Tensor):
        _check_out(g, 3 * n, dtype, dev, "g")
        g_layout, gp, gkeep = EIG3_AOS, [g.data_ptr() if n else 0, 0, 0], [g]
    else:
        gkeep = list(g)
        if len(gkeep) != 3:
            raise ValueError("g needs three tensors")
        for j, t in enumerate(gkeep):
            _check_out(t, n, dtype, dev, f"g[{j}]")
        g_layout, gp = EIG3_SOA, [t.data_ptr() if n else 0 for t in gkeep]
    if layout == EIG3_AOS:
        res = out if out is not None else torch.empty_like(a)
        _check_out(res, k * n, dtype, dev, "out")
        ptrs = [res.data_ptr() if n else 0] + [0] * 8
    else:
        res = _out_list(out, k, n, dtype, dev, "out")
        ptrs = [t.data_ptr() if n else 0 for t in res] + [0] * (9 - k)
    _capi.call_eigvals_backward(m, g_layout, gp, ptrs, _stream(dev))
    return res if layout == EIG3_AOS else tuple(res)


def eig3_mohr_coulomb(sigma: Batch, s_yc: float, m: float, structure: str = "symmetric", accuracy: str = "double_word",
                      grad: bool = True, out=None):
    """Mohr-Coulomb yield function f (n values) and, if ``grad``, df/dsigma
    in the structure and layout of ``sigma`` (symmetric: the 6 components of
    the tensor derivative).  Returns (f, dfds) with dfds None if not asked."""
    mdesc, n, dtype, dev, layout, _keep = _matrices(sigma, structure, accuracy)
    k = 9 if structure == "general" else 6
    f, dfds = (out if out is not None else (None, None))
    f = f if f is not None else torch.empty(n, dtype=dtype, device=dev)
    _check_out(f, n, dtype, dev, "f")
    ptrs = None
    if grad:
        if layout == EIG3_AOS:
            dfds = dfds if dfds is not None else torch.empty_like(sigma)
            _check_out(dfds, k * n, dtype, dev, "dfds")
            ptrs = [dfds.data_ptr() if n else 0] + [0] * 8
        else:
            dfds = _out_list(dfds, k, n, dtype, dev, "dfds")
            ptrs = [t.data_ptr() if n else 0 for t in dfds] + [0] * (9 - k)
            dfds = tuple(dfds)
    else:
        dfds = None
    _capi.call_mohr_coulomb(mdesc, s_yc, m, f.data_ptr() if n else 0, ptrs, _stream(dev))
    return f, dfds


def eig3_eigenprojectors(a: Batch, structure: str = "general", accuracy: str = "double_word", out_layout: str = "aos",
                         out=None):
    """Eigenprojectors E_1, E_2, E_3 of each matrix (ascending eigenvalues).
    out_layout 'aos': an (n, 3, K) tensor (K = 9 row-major entries, or the 6
    symmetric components); 'soa': a tuple of 3K n-vectors, slot K*k + e."""
    m, n, dtype, dev, _, _keep = _matrices(a, structure, accuracy)
    k = 9 if structure == "general" else 6
    if out_layout == "aos":
        res = out if out is not None else torch.empty((n, 3, k), dtype=dtype, device=dev)
        _check_out(res, 3 * k * n, dtype, dev, "out")
        _capi.call_eigenprojectors(m, EIG3_AOS, [res.data_ptr() if n else 0] + [0] * 26, _stream(dev))
        return res
    if out_layout == "soa":
        res = _out_list(out, 3 * k, n, dtype, dev, "out")
        _capi.call_eigenprojectors(m, EIG3_SOA, [t.data_ptr() if n else 0 for t in res] + [0] * (27 - 3 * k),
                                   _stream(dev))
        return tuple(res)
    raise ValueError("out_layout must be 'aos' or 'soa'")


def eig3_matrix_function(a: Batch, fn: str = "exp", structure: str = "general", accuracy: str = "double_word", out=None):
    """f(A) = sum_k f(lambda_k) E_k for fn in ('exp', 'log', 'sqrt'), in the
    structure and layout of ``a`` (symmetric: the 6 components)."""
    if fn not in _FN:
        raise ValueError(f"fn must be one of {tuple(_FN)}")
    m, n, dtype, dev, layout, _keep = _matrices(a, structure, accuracy)
    k = 9 if structure == "general" else 6
    if layout == EIG3_AOS:
        res = out if out is not None else torch.empty_like(a)
        _check_out(res, k * n, dtype, dev, "out")
        ptrs = [res.data_ptr() if n else 0] + [0] * 8
    else:
        res = _out_list(out, k, n, dtype, dev, "out")
        ptrs = [t.data_ptr() if n else 0 for t in res] + [0] * (9 - k)
    _capi.call_matrix_function(m, _FN[fn], ptrs, _stream(dev))
    return res if layout == EIG3_AOS else tuple(res)


def eig3_matrix_function_backward(a: Batch, g: Batch, fn: str = "exp", structure: str = "general",
                                  accuracy: str = "double_word", out=None):
    """d<G, f(A)>/dA in the structure and layout of ``a``; ``g`` in the
    layout of the forward's output (that of ``a``)."""
    if fn not in _FN:
        raise ValueError(f"fn must be one of {tuple(_FN)}")
    m, n, dtype, dev, layout, _keep = _matrices(a, structure, accuracy)
    k = 9 if structure == "general" else 6
    if layout == EIG3_AOS:
        if not isinstance(g, torch.Tensor):
            raise ValueError("g must have the layout of a (one tensor)")
        _check_out(g, k * n, dtype, dev, "g")
        gp, gkeep = [g.data_ptr() if n else 0] + [0] * 8, [g]
        res = out if out is not None else torch.empty_like(a)
        _check_out(res, k * n, dtype, dev, "out")
        ptrs = [res.data_ptr() if n else 0] + [0] * 8
    else:
        gkeep = list(g) if not isinstance(g, torch.Tensor) else None
        if gkeep is None or len(gkeep) != k:
            raise ValueError(f"g must have the layout of a ({k} tensors)")
        for j, t in enumerate(gkeep):
            _check_out(t, n, dtype, dev, f"g[{j}]")
        gp = [t.data_ptr() if n else 0 for t in gkeep] + [0] * (9 - k)
        res = _out_list(out, k, n, dtype, dev, "out")
        ptrs = [t.data_ptr() if n else 0 for t in res] + [0] * (9 - k)
    _capi.call_matrix_function_backward(m, _FN[fn], gp, ptrs, _stream(dev))
    return res if layout == EIG3_AOS else tuple(res)


class Eig3MatrixFunction(torch.autograd.Function):
    """F = f(A) for A of shape (..., 3, 3) (general; coalescing and repeated
    eigenvalues included), f in ('exp', 'log', 'sqrt'), with
    eig3_matrix_function_backward as its backward."""

    @staticmethod
    def forward(ctx, a: torch.Tensor, fn: str = "exp", accuracy: str = "double_word"):
        if a.shape[-2:] != (3, 3):
            raise ValueError("expected (..., 3, 3)")
        ac = a.contiguous()
        f = eig3_matrix_function(ac.reshape(-1, 9), fn, "general", accuracy)
        ctx.save_for_backward(ac)
        ctx.fn, ctx.accuracy = fn, accuracy
        return f.reshape(ac.shape)

    @staticmethod
    def backward(ctx, gf: torch.Tensor):
        (ac,) = ctx.saved_tensors
        grad = eig3_matrix_function_backward(ac.reshape(-1, 9), gf.contiguous().reshape(-1, 9), ctx.fn, "general",
                                             ctx.accuracy)
        return grad.reshape(ac.shape), None, None


def matrix_function(a: torch.Tensor, fn: str = "exp", accuracy: str = "double_word") -> torch.Tensor:
    """f(A) of a (..., 3, 3) device tensor, differentiable."""
    return Eig3MatrixFunction.apply(a, fn, accuracy)


class Eig3MatrixFunctionSymmetric(torch.autograd.Function):
    """F = f(S) for symmetric matrices stored as (..., 6) tensors (A00 A11 A22
    A01 A02 A12), F in the same six-component storage; the kernels read and
    write that storage as it is.  The backward is the symmetric
    eig3_matrix_function_backward: from dL/d(the six components of F) to
    dL/d(the six stored entries of S)."""

    @staticmethod
    def forward(ctx, s: torch.Tensor, fn: str = "exp", accuracy: str = "double_word"):
        if s.shape[-1] != 6:
            raise ValueError("expected (..., 6): A00 A11 A22 A01 A02 A12")
        sc = s.contiguous()
        f = eig3_matrix_function(sc.reshape(-1, 6), fn, "symmetric", accuracy)
        ctx.save_for_backward(sc)
        ctx.fn, ctx.accuracy = fn, accuracy
        return f.reshape(sc.shape)

    @staticmethod
    def backward(ctx, gf: torch.Tensor):
        (sc,) = ctx.saved_tensors
        grad = eig3_matrix_function_backward(sc.reshape(-1, 6), gf.contiguous().reshape(-1, 6), ctx.fn, "symmetric",
                                             ctx.accuracy)
        return grad.reshape(sc.shape), None, None


def matrix_function_symmetric(s: torch.Tensor, fn: str = "exp", accuracy: str = "double_word") -> torch.Tensor:
    """f(S) of symmetric matrices stored as a (..., 6) device tensor
    (A00 A11 A22 A01 A02 A12), in the same storage, differentiable."""
    return Eig3MatrixFunctionSymmetric.apply(s, fn, accuracy)


class Eig3Eigvals(torch.autograd.Function):
    """lambda = eigvals(A) for A of shape (..., 3, 3) (general) with the
    hand-written adjoint of ``eig3_eigvals_backward`` as its backward."""

    @staticmethod
    def forward(ctx, a: torch.Tensor, accuracy: str = "double_word"):
        shape = a.shape
        if shape[-2:] != (3, 3):
            raise ValueError("expected (..., 3, 3)")
        ac = a.contiguous()
        lam = eig3_eigvals(ac.reshape(-1, 9), "general", accuracy, "aos")
        ctx.save_for_backward(ac)
        ctx.accuracy = accuracy
        return lam.reshape(*shape[:-2], 3)

    @staticmethod
    def backward(ctx, glam: torch.Tensor):
        (ac,) = ctx.saved_tensors
        g = glam.contiguous().reshape(-1, 3)
        grad = eig3_eigvals_backward(ac.reshape(-1, 9), g, "general", ctx.accuracy)
        return grad.reshape(ac.shape), None


def eigvals(a: torch.Tensor, accuracy: str = "double_word") -> torch.Tensor:
    """Ascending eigenvalues of a (..., 3, 3) float64 device tensor, differentiable."""
    return Eig3Eigvals.apply(a, accuracy)


class Eig3EigvalsSymmetric(torch.autograd.Function):
    """lambda = eigvals(S) for symmetric matrices stored as (..., 6) tensors,
    entries (A00, A11, A22, A01, A02, A12), read by the kernels as they are;
    the backward is the symmetric ``eig3_eigvals_backward``: the gradient with
    respect to the six stored entries (an off-diagonal entry counts both of its
    positions)."""

    @staticmethod
    def forward(ctx, s: torch.Tensor, accuracy: str = "double_word"):
        shape = s.shape
        if shape[-1] != 6:
            raise ValueError("expected (..., 6): A00 A11 A22 A01 A02 A12")
        sc = s.contiguous()
        lam = eig3_eigvals(sc.reshape(-1, 6), "symmetric", accuracy, "aos")
        ctx.save_for_backward(sc)
        ctx.accuracy = accuracy
        return lam.reshape(*shape[:-1], 3)

    @staticmethod
    def backward(ctx, glam: torch.Tensor):
        (sc,) = ctx.saved_tensors
        g = glam.contiguous().reshape(-1, 3)
        grad = eig3_eigvals_backward(sc.reshape(-1, 6), g, "symmetric", ctx.accuracy)
        return grad.reshape(sc.shape), None


def eigvals_symmetric(s: torch.Tensor, accuracy: str = "double_word") -> torch.Tensor:
    """Ascending eigenvalues of symmetric matrices stored as a (..., 6) device
    tensor (A00 A11 A22 A01 A02 A12), float64 or float32, differentiable."""
    return Eig3EigvalsSymmetric.apply(s, accuracy)
