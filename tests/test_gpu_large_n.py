"""Batches beyond 2^31 matrices: 64-bit span origins and the grid-stride loop
(the launch holds at most 2^20 workgroups).  n = 2^31 + 777 symmetric
matrices generated on the device, in binary32 (two matrices per lane) and in
binary64 (one per lane).  Matrices sampled around index 2^31, at both ends
and at random give bitwise the eigenvalues of a small batch made of the same
matrices, and a subset meets the bound against the exact oracle.  The
array-of-structures driver (LDS tile, barriers) is taken past its first
stride with n = 2^28 + 333 general matrices, eigenvalues and adjoint."""
import numpy as np
import pytest

from accuracy import EPS32, EPS64, Truth, check, lam_errors

pytestmark = pytest.mark.gpu

N = (1 << 31) + 777


def _indices(n, rng):
    edges = [np.arange(0, 300), np.arange((1 << 31) - 300, (1 << 31) + 300), np.arange(n - 300, n)]
    return np.unique(np.concatenate(edges + [rng.integers(0, n, 400)]))


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_symmetric_beyond_2p31(dtype_name):
    import torch

    import paper_2511_00292_amd as eig3
    dtype = getattr(torch, dtype_name)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2024)
    s = [torch.randn(N, dtype=dtype, device=dev, generator=g) for _ in range(6)]
    lam = eig3.eig3_eigvals(s, "symmetric", "double_word", "soa")
    torch.cuda.synchronize()
    idx = _indices(N, np.random.default_rng(31))
    it = torch.from_numpy(idx).to(dev)
    sub = [x.index_select(0, it).clone() for x in s]
    got = torch.stack([x.index_select(0, it) for x in lam], 1).cpu().numpy()
    del s, lam
    torch.cuda.empty_cache()
    ref = torch.stack(eig3.eig3_eigvals(sub, "symmetric", "double_word", "soa"), 1).cpu().numpy()
    assert np.array_equal(got, ref)
    host = np.stack([x.cpu().numpy().astype(np.float64) for x in sub], 1)
    a = np.stack([host[:, 0], host[:, 3], host[:, 4], host[:, 3], host[:, 1], host[:, 5],
                  host[:, 4], host[:, 5], host[:, 2]], 1)
    pick = np.arange(0, len(idx), max(1, len(idx) // 200))
    t = Truth(a[pick], np.ones(len(pick)))
    eps = EPS32 if dtype_name == "float32" else EPS64
    check(lam_errors(t, got[pick].astype(np.float64)), t.bound_lam(eps), what=f"n = 2^31 + 777 {dtype_name}")


N_AOS = (1 << 28) + 333


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_general_aos_beyond_grid(dtype_name):
    """Array-of-structures input beyond the launch's 2^20 workgroups of 256
    matrices: the LDS-staged driver's grid-stride loop (its tile reused
    across spans between barriers, the AoS outputs flushed through LDS).
    n = 2^28 + 333 general matrices (n, 3, 3), eigenvalues (n, 3) and their
    adjoint for g (n, 3); rows sampled around index 2^28, where the second
    stride begins, at both ends and at random equal bitwise the results of a
    small batch made of the same rows."""
    import torch

    import paper_2511_00292_amd as eig3
    dtype = getattr(torch, dtype_name)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2025)
    a = torch.randn((N_AOS, 3, 3), dtype=dtype, device=dev, generator=g)
    a = (a + a.transpose(1, 2)) * 0.5 + 0.25 * torch.randn((N_AOS, 3, 3), dtype=dtype, device=dev, generator=g)
    gl = torch.randn((N_AOS, 3), dtype=dtype, device=dev, generator=g)
    lam = eig3.eig3_eigvals(a, "general", "double_word", "aos")
    grad = eig3.eig3_eigvals_backward(a, gl, "general", "double_word")
    torch.cuda.synchronize()
    rng = np.random.default_rng(28)
    edges = [np.arange(0, 300), np.arange((1 << 28) - 300, (1 << 28) + 300), np.arange(N_AOS - 300, N_AOS)]
    idx = np.unique(np.concatenate(edges + [rng.integers(0, N_AOS, 400)]))
    it = torch.from_numpy(idx).to(dev)
    sub_a, sub_g = a.index_select(0, it).contiguous(), gl.index_select(0, it).contiguous()
    got_lam, got_grad = lam.index_select(0, it).cpu(), grad.index_select(0, it).cpu()
    del a, gl, lam, grad
    torch.cuda.empty_cache()
    ref_lam = eig3.eig3_eigvals(sub_a, "general", "double_word", "aos").cpu()
    ref_grad = eig3.eig3_eigvals_backward(sub_a, sub_g, "general", "double_word").cpu()
    assert got_lam.shape == (len(idx), 3) and got_grad.shape == (len(idx), 3, 3)
    # bit patterns: a perturbed matrix with a complex pair has a NaN gradient
    # on both sides
    bits = torch.int32 if dtype_name == "float32" else torch.int64
    assert torch.equal(got_lam.view(bits), ref_lam.view(bits))
    assert torch.equal(got_grad.view(bits), ref_grad.view(bits))
