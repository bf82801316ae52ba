"""Batches beyond 2^31 matrices: 64-bit span origins and the grid-stride loop
(the launch holds at most 2^20 workgroups).  n = 2^31 + 777 symmetric
matrices generated on the device, in binary32 (two matrices per lane) and in
binary64 (one per lane).  Matrices sampled around index 2^31, at both ends
and at random give bitwise the eigenvalues of a small batch made of the same
matrices, and a subset meets the bound against the exact oracle."""
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
    lam = eig3.eig3_eigvals(s, "symmetric", "fma", "soa")
    torch.cuda.synchronize()
    idx = _indices(N, np.random.default_rng(31))
    it = torch.from_numpy(idx).to(dev)
    sub = [x.index_select(0, it).clone() for x in s]
    got = torch.stack([x.index_select(0, it) for x in lam], 1).cpu().numpy()
    del s, lam
    torch.cuda.empty_cache()
    ref = torch.stack(eig3.eig3_eigvals(sub, "symmetric", "fma", "soa"), 1).cpu().numpy()
    assert np.array_equal(got, ref)
    host = np.stack([x.cpu().numpy().astype(np.float64) for x in sub], 1)
    a = np.stack([host[:, 0], host[:, 3], host[:, 4], host[:, 3], host[:, 1], host[:, 5],
                  host[:, 4], host[:, 5], host[:, 2]], 1)
    pick = np.arange(0, len(idx), max(1, len(idx) // 200))
    t = Truth(a[pick], np.ones(len(pick)))
    eps = EPS32 if dtype_name == "float32" else EPS64
    check(lam_errors(t, got[pick].astype(np.float64)), t.bound_lam(eps), what=f"n = 2^31 + 777 {dtype_name}")
