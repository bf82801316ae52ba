"""The C ABI library (no GPU needed): it loads, exports every function that
include/eig3.h declares, and rejects invalid arguments before launching
anything.  Every call here fails validation on the host, so no kernel ever
starts with the made-up pointers used below."""
import ctypes

import pytest

from paper_2511_00292_amd import _capi as capi

FAKE = 0x10000  # never dereferenced: every call below is rejected first


def _gpu_present() -> bool:
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:  # pragma: no cover
        return False


# belt and braces: the made-up pointers never reach a device
pytestmark = pytest.mark.skipif(_gpu_present(), reason="argument-validation tests run on hosts without a GPU")


@pytest.fixture(scope="module")
def lib():
    return capi.lib()


def _mat(n=16, dtype=0, structure=0, layout=0, accuracy=0, ptrs=None):
    m = capi.Eig3Matrices()
    m.n, m.dtype, m.structure, m.layout, m.accuracy = n, dtype, structure, layout, accuracy
    k = 9 if structure == 0 else 6
    ptrs = ptrs if ptrs is not None else [FAKE + 0x100000 * (j + 1) for j in range(k)]
    for j, p in enumerate(ptrs):
        m.a[j] = p
    return m


def test_exports_every_declared_symbol(lib):
    names = capi.declared_functions()
    assert set(names) >= {"eig3_invariants", "eig3_eigvals", "eig3_eigvals_backward", "eig3_status_string",
                          "eig3_version"}
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for st in (0, -1, -2, -3):
        assert capi.status_string(st).startswith("EIG3_")
    assert "unknown" in capi.status_string(42)
    assert capi.version().count(".") == 2


def _eigvals(lib, m, outs=(0x9000000, 0xA000000, 0xB000000), out_layout=0):
    arr = (ctypes.c_void_p * 3)(*outs)
    return lib.eig3_eigvals(ctypes.byref(m) if m is not None else None, out_layout, arr, None)


def test_null_and_bad_enums_rejected(lib):
    assert lib.eig3_eigvals(None, 0, (ctypes.c_void_p * 3)(1, 2, 3), None) == capi.EIG3_EINVAL
    assert _eigvals(lib, _mat(n=-1)) == capi.EIG3_EINVAL
    assert _eigvals(lib, _mat(n=(1 << 56) + 1)) == capi.EIG3_EINVAL     # beyond the largest batch
    assert _eigvals(lib, _mat(dtype=7)) == capi.EIG3_EINVAL
    assert _eigvals(lib, _mat(structure=3)) == capi.EIG3_EINVAL
    assert _eigvals(lib, _mat(layout=2)) == capi.EIG3_EINVAL
    assert _eigvals(lib, _mat(accuracy=9)) == capi.EIG3_EINVAL
    assert _eigvals(lib, _mat(), out_layout=5) == capi.EIG3_EINVAL
    ptrs = [FAKE] * 8 + [0]
    assert _eigvals(lib, _mat(ptrs=ptrs)) == capi.EIG3_EINVAL          # a null entry pointer
    assert _eigvals(lib, _mat(ptrs=[FAKE + 4] + [FAKE] * 8)) == capi.EIG3_EINVAL  # misaligned f64
    assert _eigvals(lib, _mat(), outs=(0x9000000, 0, 0xB000000)) == capi.EIG3_EINVAL


def test_empty_batch_is_noop(lib):
    assert _eigvals(lib, _mat(n=0, ptrs=[0] * 9)) == capi.EIG3_OK
    m = _mat(n=0, ptrs=[0] * 9)
    assert lib.eig3_invariants(ctypes.byref(m), None, None, None, None, None) == capi.EIG3_OK
    g = (ctypes.c_void_p * 3)(0, 0, 0)
    o = (ctypes.c_void_p * 9)(*([0] * 9))
    assert lib.eig3_eigvals_backward(ctypes.byref(m), 0, g, o, None) == capi.EIG3_OK


def test_aliasing_rejected(lib):
    n = 1024
    base = 0x20000000
    ins = [base + j * n * 8 for j in range(9)]
    m = _mat(n=n, ptrs=ins)
    # output overlapping an input
    assert _eigvals(lib, m, outs=(ins[4] + 8, 0x9000000, 0xA000000)) == capi.EIG3_EINVAL
    # outputs overlapping each other
    assert _eigvals(lib, m, outs=(0x9000000, 0x9000000 + 8, 0xA000000)) == capi.EIG3_EINVAL
    # AoS output of n*3 values overlapping an input
    ma = _mat(n=n, layout=1, ptrs=[base])
    assert _eigvals(lib, ma, outs=(base + n * 9 * 8 - 8, 0, 0), out_layout=1) == capi.EIG3_EINVAL
    # invariants: disc aliasing i1
    assert lib.eig3_invariants(ctypes.byref(m), ctypes.c_void_p(0x9000000), ctypes.c_void_p(0xA000000),
                               ctypes.c_void_p(0xB000000), ctypes.c_void_p(0x9000000), None) == capi.EIG3_EINVAL
    # backward: gradient aliasing g
    g = (ctypes.c_void_p * 3)(0x30000000, 0x31000000, 0x32000000)
    o = (ctypes.c_void_p * 9)(*([0x30000000 + 8] + [0x40000000 + j * 0x1000000 for j in range(8)]))
    assert lib.eig3_eigvals_backward(ctypes.byref(m), 0, g, o, None) == capi.EIG3_EINVAL


def test_python_binding_rejects_host_tensors():
    import torch

    import paper_2511_00292_amd as eig3
    with pytest.raises(ValueError):
        eig3.eig3_eigvals(torch.zeros(4, 9, dtype=torch.float64))
    with pytest.raises(ValueError):
        eig3.eig3_eigvals([torch.zeros(4, dtype=torch.float64)] * 3)


def test_eigenprojector_outputs_all_checked(lib):
    """27 structure-of-arrays outputs are each range-checked (regression: the
    host check once held room for 9); the last one aliases an input, so the
    call is rejected after every slot was examined."""
    n = 1024
    ins = [0x20000000 + j * n * 8 for j in range(9)]
    m = _mat(n=n, ptrs=ins)
    outs = [0x40000000 + j * 0x100000 for j in range(26)] + [ins[0]]
    arr = (ctypes.c_void_p * 27)(*outs)
    assert lib.eig3_eigenprojectors(ctypes.byref(m), 0, arr, None) == capi.EIG3_EINVAL
    # Mohr-Coulomb: the gradient arrays and f are checked against each other
    f = 0x50000000
    grads = (ctypes.c_void_p * 9)(*([f] + [0x60000000 + j * 0x100000 for j in range(8)]))
    assert lib.eig3_mohr_coulomb(ctypes.byref(m), ctypes.c_double(100.0), ctypes.c_double(10.0),
                                 ctypes.c_void_p(f), grads, None) == capi.EIG3_EINVAL
    assert lib.eig3_mohr_coulomb(ctypes.byref(m), ctypes.c_double(0.0), ctypes.c_double(10.0),
                                 ctypes.c_void_p(f), None, None) == capi.EIG3_EINVAL


def test_matrix_function_arguments(lib):
    n = 1024
    base = 0x20000000
    ins = [base + j * n * 8 for j in range(9)]
    m = _mat(n=n, ptrs=ins)
    outs = (ctypes.c_void_p * 9)(*[0x40000000 + j * 0x100000 for j in range(9)])
    assert lib.eig3_matrix_function(ctypes.byref(m), 3, outs, None) == capi.EIG3_EINVAL      # unknown function
    assert lib.eig3_matrix_function(ctypes.byref(m), -1, outs, None) == capi.EIG3_EINVAL
    alias = (ctypes.c_void_p * 9)(*([0x40000000 + j * 0x100000 for j in range(8)] + [ins[2]]))
    assert lib.eig3_matrix_function(ctypes.byref(m), 0, alias, None) == capi.EIG3_EINVAL     # output aliases input
    m0 = _mat(n=0, ptrs=[0] * 9)
    assert lib.eig3_matrix_function(ctypes.byref(m0), 0, (ctypes.c_void_p * 9)(*([0] * 9)), None) == capi.EIG3_OK


def test_matrix_function_backward_arguments(lib):
    n = 1024
    base = 0x20000000
    ins = [base + j * n * 8 for j in range(9)]
    m = _mat(n=n, ptrs=ins)
    g = (ctypes.c_void_p * 9)(*[0x30000000 + j * 0x100000 for j in range(9)])
    outs = (ctypes.c_void_p * 9)(*[0x40000000 + j * 0x100000 for j in range(9)])
    assert lib.eig3_matrix_function_backward(ctypes.byref(m), 5, g, outs, None) == capi.EIG3_EINVAL
    alias = (ctypes.c_void_p * 9)(*([0x40000000 + j * 0x100000 for j in range(8)] + [0x30000000 + 4 * 0x100000]))
    assert lib.eig3_matrix_function_backward(ctypes.byref(m), 0, g, alias, None) == capi.EIG3_EINVAL  # grad aliases g
    gnull = (ctypes.c_void_p * 9)(*([0x30000000] * 8 + [0]))
    assert lib.eig3_matrix_function_backward(ctypes.byref(m), 0, gnull, outs, None) == capi.EIG3_EINVAL


def test_soa_stride(lib):
    """eig3_soa_stride: n elements rounded up to a multiple of 64 KiB, plus
    42 KiB, counted in elements of the dtype; -1 for invalid arguments."""
    for n, dtype, size in ((0, 0, 8), (1, 0, 8), (1 << 24, 0, 8), (1 << 27, 1, 4), (10 ** 7, 0, 8), (12345, 1, 4),
                           (1 << 56, 0, 8)):
        stride = lib.eig3_soa_stride(n, dtype)
        pad = stride * size - 43008
        assert pad % 65536 == 0 and 0 <= pad - n * size < 65536, (n, dtype, stride)
    assert lib.eig3_soa_stride(-1, 0) == -1
    assert lib.eig3_soa_stride(16, 2) == -1
    assert lib.eig3_soa_stride((1 << 56) + 1, 0) == -1


def test_empty_soa_views():
    """The Python helper: count disjoint contiguous arrays of n values in one
    buffer, array k at element k * stride."""
    import torch

    import paper_2511_00292_amd as eig3
    for n, dtype in ((1000, torch.float64), (1 << 16, torch.float32), (0, torch.float64)):
        arrays = eig3.empty_soa(n, 5, dtype, device="cpu")
        stride = eig3.soa_stride(n, dtype)
        assert [t.numel() for t in arrays] == [n] * 5 and all(t.is_contiguous() and t.dtype == dtype for t in arrays)
        if n:
            base = arrays[0].data_ptr()
            assert [t.data_ptr() - base for t in arrays] == [k * stride * arrays[0].element_size() for k in range(5)]
    with pytest.raises(capi.Eig3Error):
        eig3.soa_stride(-5)
