"""GPU parity of the hand-written adjoint (eig3_eigvals_backward) and of the
torch.autograd.Function built on it."""
import numpy as np
import pytest

import workloads as w
from gpu_util import download_lam, download_matrix, upload
from oracle import exact

pytestmark = pytest.mark.gpu

ACCS = ["fma", "compensated", "double_word"]


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


@pytest.fixture(scope="module")
def c5():
    return w.differentiation_batch(1 << 14, with_basis=True)


def _rel(err, ref):
    return np.abs(err).max(axis=1) / np.abs(ref).max(axis=1)


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("g_layout", ["soa", "aos"])
def test_backward_eigenvector_formula(eig3, c5, acc, layout, g_layout):
    """d(lambda_i) = y_i^T dA x_i / (y_i^T x_i), x_i = V[:, i], y_i^T = V^-1[i, :],
    for every matrix of the batch (sorted spectra, gap >= 1e-3, kappa <= 100)."""
    g = c5["g"]
    gd = upload(g, g_layout)
    grad = download_matrix(eig3.eig3_eigvals_backward(upload(c5["a"], layout), gd, "general", acc), 9)
    v = c5["v"].reshape(-1, 3, 3)
    vi = c5["vinv"].reshape(-1, 3, 3)
    ref = np.einsum("mk,mki,mjk->mij", g, vi, v).reshape(-1, 9)
    r = _rel(grad - ref, ref)
    assert r.max() <= 1e-7, r.max()


@pytest.mark.parametrize("acc", ACCS)
def test_backward_exact_gradient(eig3, c5, acc):
    """Against the exact eigenprojector gradient (80-digit) on a subset."""
    idx = np.arange(0, c5["a"].shape[0], 64)
    grad = download_matrix(eig3.eig3_eigvals_backward(upload(c5["a"][idx], "aos"), upload(c5["g"][idx], "aos"),
                                                      "general", acc), 9)
    ref = np.array([exact.eigvals_vjp(c5["a"][m], c5["g"][m]) for m in idx])
    r = _rel(grad - ref, ref)
    assert r.max() <= 1e-7, r.max()


def test_backward_against_plain_oracle(eig3, plain_oracle, c5):
    grad = download_matrix(eig3.eig3_eigvals_backward(upload(c5["a"], "aos"), upload(c5["g"], "aos")), 9)
    ref = plain_oracle.eigvals_backward(c5["a"], c5["g"])
    assert _rel(grad - ref, ref).max() <= 1e-7


def test_backward_identities(eig3, c5):
    """g = 1 -> I; g = lambda -> A^T."""
    a = c5["a"][:4096]
    n = a.shape[0]
    one = download_matrix(eig3.eig3_eigvals_backward(upload(a, "aos"), upload(np.ones((n, 3)), "aos")), 9)
    assert np.abs(one - np.eye(3).ravel()).max() < 1e-9
    lam = eig3.eig3_eigvals(upload(a, "aos"))
    at = download_matrix(eig3.eig3_eigvals_backward(upload(a, "aos"), lam), 9)
    ref = a.reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9)
    assert np.abs(at - ref).max() < 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("acc", ACCS)
def test_backward_central_differences(eig3, plain_oracle, c5, acc):
    """Central differences (h = 1e-6) of the plain binary64 oracle's
    eigenvalues (O1), g-weighted: within 2e-3 max|grad| (the truncation error
    of h = 1e-6 at gaps down to 1e-3 and kappa up to 100)."""
    a = c5["a"][:512]
    g = c5["g"][:512]
    grad = download_matrix(eig3.eig3_eigvals_backward(upload(a, "aos"), upload(g, "aos"), "general", acc), 9)
    h = 1e-6
    fd = np.zeros_like(grad)
    for e in range(9):
        ap = a.copy(); ap[:, e] += h
        am = a.copy(); am[:, e] -= h
        lp = plain_oracle.eigvals(ap)
        lm = plain_oracle.eigvals(am)
        fd[:, e] = ((lp - lm) * g).sum(1) / (ap[:, e] - am[:, e])
    assert _rel(fd - grad, grad).max() <= 2e-3


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_backward_symmetric(eig3, layout):
    """Symmetric storage: gradient with respect to the 6 stored entries equals
    the general gradient with the two off-diagonal positions summed."""
    s = w.stress_tensors(4096, seed=31)["s"]
    keep = np.ones(s.shape[0], dtype=bool)
    a = w.symmetric_to_general(s)
    rng = np.random.default_rng(5)
    g = rng.standard_normal((s.shape[0], 3))
    gg = download_matrix(eig3.eig3_eigvals_backward(upload(a, "aos"), upload(g, "aos")), 9)
    gs = download_matrix(eig3.eig3_eigvals_backward(upload(s, layout), upload(g, "soa"), "symmetric"), 6)
    ref = np.stack([gg[:, 0], gg[:, 4], gg[:, 8], gg[:, 1] + gg[:, 3], gg[:, 2] + gg[:, 6], gg[:, 5] + gg[:, 7]],
                   axis=1)
    # near-isotropic matrices have gaps down to ~1e-14 * 100; compare where
    # the spectrum is separated
    lam = download_lam(eig3.eig3_eigvals(upload(s, "aos"), "symmetric"))
    gap = np.minimum(lam[:, 1] - lam[:, 0], lam[:, 2] - lam[:, 1]) / np.maximum(np.abs(lam).max(1), 1e-300)
    keep &= gap > 1e-4
    assert keep.sum() > 1000
    assert np.abs(gs - ref)[keep].max() <= 1e-9 * np.abs(ref[keep]).max()


def test_autograd_function(eig3, c5):
    """eigvals(A).backward() runs the hand-written adjoint; cross-check with
    torch's own eigen-decomposition autograd on the CPU."""
    import torch
    a_np = c5["a"][:256]
    g_np = c5["g"][:256]
    a = torch.tensor(a_np, device="cuda:0").reshape(-1, 3, 3).requires_grad_(True)
    lam = eig3.eigvals(a)
    (lam * torch.tensor(g_np, device="cuda:0")).sum().backward()
    ac = torch.tensor(a_np).reshape(-1, 3, 3).requires_grad_(True)
    ev = torch.linalg.eigvals(ac).real
    evs, order = torch.sort(ev, dim=1)
    (evs * torch.tensor(g_np)).sum().backward()
    ref = ac.grad.numpy().reshape(-1, 9)
    got = a.grad.cpu().numpy().reshape(-1, 9)
    np.testing.assert_allclose(lam.detach().cpu().numpy(), evs.detach().numpy(), atol=1e-10)
    assert _rel(got - ref, ref).max() < 1e-6


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_autograd_symmetric_storage(eig3, dtype_name):
    """eig3.eigvals_symmetric on (..., 6) storage against eig3.eigvals on the
    full matrices built from the same six entries by differentiable torch
    ops (binary64), on separated spectra: same eigenvalues, and the gradient
    with respect to the six stored entries equals the full-matrix gradient
    pulled back through that construction (an off-diagonal entry gets the sum
    of its two positions)."""
    import torch
    dtype = getattr(torch, dtype_name)
    rng = np.random.default_rng(44)
    mats = []
    while len(mats) < 3000:  # Q diag(lambda) Q^T, Haar Q, gaps >= 0.05
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        lam = np.sort(rng.uniform(-1.0, 1.0, 3))
        if np.diff(lam).min() >= 0.05:
            m = q @ np.diag(lam) @ q.T
            mats.append([m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2]])
    s = torch.tensor(np.array(mats).reshape(2, 3, 500, 6), dtype=dtype, device="cuda:0")
    wgt = torch.tensor(np.random.default_rng(45).standard_normal((2, 3, 500, 3)), dtype=dtype, device="cuda:0")
    s1 = s.clone().requires_grad_(True)
    lam1 = eig3.eigvals_symmetric(s1)
    (lam1 * wgt).sum().backward()
    s2 = s.double().clone().requires_grad_(True)
    rows = [torch.stack([s2[..., 0], s2[..., 3], s2[..., 4]], -1),
            torch.stack([s2[..., 3], s2[..., 1], s2[..., 5]], -1),
            torch.stack([s2[..., 4], s2[..., 5], s2[..., 2]], -1)]
    a2 = torch.stack(rows, -2)
    lam2 = eig3.eigvals(a2)
    (lam2 * wgt.double()).sum().backward()
    assert lam1.shape == (2, 3, 500, 3) and s1.grad.shape == s.shape
    tol = 1e-12 if dtype_name == "float64" else 2e-5
    scale_l = lam2.detach().abs().amax(-1, keepdim=True)
    assert torch.all((lam1.double() - lam2).detach().abs() <= tol * scale_l)
    scale_g = s2.grad.abs().amax(-1, keepdim=True)
    assert torch.all((s1.grad.double() - s2.grad).abs() <= 10 * tol * scale_g)
