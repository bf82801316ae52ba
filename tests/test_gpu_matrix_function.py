"""Functions of matrices (eig3_matrix_function): f(A) = sum_k f(lambda_k) E_k,
evaluated as the interpolation polynomial in Newton form, against the exact
oracle (80-digit eigenprojectors and f), on general matrices with separated
spectra, on symmetric positive definite ones and on nearly isotropic ones;
repeated eigenvalues; identities and the domain rule.  The adjoint
(eig3_matrix_function_backward) likewise, including nearly and exactly
repeated eigenvalues and defective matrices."""
import numpy as np
import pytest

import workloads as w
from accuracy import EPS32
from gpu_util import download_matrix, upload
from oracle import exact

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


def _spd(n, seed, lo=0.3, hi=3.0, gap=1e-2):
    """Q diag(l) Q^T, Haar Q, l ~ U[lo, hi] sorted with gaps >= gap."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        lam = np.sort(rng.uniform(lo, hi, 3))
        if np.diff(lam).min() >= gap:
            out.append((q @ np.diag(lam) @ q.T).ravel())
    return np.array(out)


def _rel(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("acc", ["fma", "compensated", "double_word"])
def test_exp_general(eig3, layout, acc):
    """exp on the differentiation batch (kappa <= 100, gaps >= 1e-3)."""
    c = w.differentiation_batch(1000, seed=91)
    res = download_matrix(eig3.eig3_matrix_function(upload(c["a"], layout), "exp", "general", acc), 9)
    for m in range(0, 1000, 8):
        assert _rel(res[m], np.array(exact.matrix_function(c["a"][m], "exp"))) <= 1e-12, m


@pytest.mark.parametrize("fn", ["exp", "log", "sqrt"])
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_symmetric_positive_definite(eig3, fn, layout):
    """exp, log, sqrt of SPD matrices in symmetric storage (6 components)."""
    a = _spd(600, 92)
    s = np.stack([a[:, 0], a[:, 4], a[:, 8], a[:, 1], a[:, 2], a[:, 5]], axis=1)
    res = download_matrix(eig3.eig3_matrix_function(upload(s, layout), fn, "symmetric"), 6)
    for m in range(0, 600, 6):
        ref = np.array(exact.matrix_function(a[m], fn)).reshape(3, 3)
        ref6 = np.array([ref[0, 0], ref[1, 1], ref[2, 2], ref[0, 1], ref[0, 2], ref[1, 2]])
        assert _rel(res[m], ref6) <= 1e-13, (fn, m)


def test_identities_and_domain(eig3):
    """exp(log A) = A and sqrt(A)^2 = A for SPD A (2^16 matrices); the log of a
    matrix with a negative eigenvalue is NaN."""
    import torch
    a = _spd(1 << 16, 93)
    ad = upload(a, "aos")
    lg = eig3.eig3_matrix_function(ad, "log")
    back = eig3.eig3_matrix_function(lg, "exp").cpu().numpy()
    scale = np.abs(a).max(1)
    assert np.all(np.abs(back - a).max(1) <= 1e-13 * scale)
    r = eig3.eig3_matrix_function(ad, "sqrt").reshape(-1, 3, 3)
    sq = torch.matmul(r, r).reshape(-1, 9).cpu().numpy()
    assert np.all(np.abs(sq - a).max(1) <= 1e-13 * scale)
    neg = np.diag([-1.0, 1.0, 2.0]).ravel()[None, :].repeat(4, axis=0)
    out = eig3.eig3_matrix_function(upload(neg, "aos"), "log").cpu().numpy()
    assert np.isnan(out).any(axis=1).all()


@pytest.mark.parametrize("fn", ["exp", "log", "sqrt"])
@pytest.mark.parametrize("delta", [1e-3, 1e-7, 1e-12])
def test_nearly_isotropic(eig3, fn, delta):
    """p I + delta S (S symmetric Gaussian): eigenvalues that all but coalesce.
    The eigenprojectors themselves are ill-conditioned here, f(A) is not."""
    rng = np.random.default_rng(97)
    p = rng.uniform(0.5, 2.0, 300)
    s = rng.standard_normal((300, 3, 3))
    a = (p[:, None, None] * np.eye(3) + delta * (s + s.transpose(0, 2, 1)) / 2).reshape(-1, 9)
    res = download_matrix(eig3.eig3_matrix_function(upload(a, "soa"), fn), 9)
    for m in range(0, 300, 5):
        assert _rel(res[m], np.array(exact.matrix_function(a[m], fn))) <= 1e-13, (fn, delta, m)


def test_repeated_eigenvalues(eig3):
    """Exactly repeated eigenvalues: f(p I) = f(p) I and f of diagonal
    matrices with a double eigenvalue, in both layouts; log I = 0 exactly."""
    diag = np.array([[1.0, 1.0, 1.0], [2.5, 2.5, 2.5], [1.0, 1.0, 2.0], [3.0, 0.5, 3.0], [0.25, 4.0, 4.0]])
    a = np.zeros((len(diag), 9))
    a[:, [0, 4, 8]] = diag
    for fn, f in (("exp", np.exp), ("log", np.log), ("sqrt", np.sqrt)):
        for layout in ("soa", "aos"):
            res = download_matrix(eig3.eig3_matrix_function(upload(a, layout), fn), 9)
            ref = np.zeros_like(a)
            ref[:, [0, 4, 8]] = f(diag)
            assert np.abs(res - ref).max() <= 4e-15 * np.abs(ref).max(), (fn, layout)
    lg = download_matrix(eig3.eig3_matrix_function(upload(a[:1], "soa"), "log"), 9)
    assert np.all(lg == 0.0)


_DERIVATIVES = {  # f, f', f''/2 in closed form
    "exp": (np.exp, np.exp, lambda x: np.exp(x) / 2),
    "log": (np.log, lambda x: 1 / x, lambda x: -0.5 / x**2),
    "sqrt": (np.sqrt, lambda x: 0.5 / np.sqrt(x), lambda x: -0.125 / x**1.5),
}


@pytest.mark.parametrize("fn", ["exp", "log", "sqrt"])
def test_defective_jordan_blocks(eig3, fn):
    """p I + N with N strictly upper or lower triangular (a single Jordan
    block when N01 N12 != 0): f(A) = f(p) I + f'(p) N + f''(p)/2 N^2, the
    confluent (Hermite) limit of the interpolation polynomial."""
    rng = np.random.default_rng(98)
    p = rng.uniform(0.5, 3.0, 64)
    n = np.zeros((64, 3, 3))
    n[:, 0, 1], n[:, 0, 2], n[:, 1, 2] = rng.uniform(-4, 4, (3, 64))
    n[32:] = n[32:].transpose(0, 2, 1)
    f0, f1, f2 = _DERIVATIVES[fn]
    eye = np.eye(3)
    a = (p[:, None, None] * eye + n).reshape(-1, 9)
    ref = (f0(p)[:, None, None] * eye + f1(p)[:, None, None] * n
           + f2(p)[:, None, None] * np.matmul(n, n)).reshape(-1, 9)
    res = download_matrix(eig3.eig3_matrix_function(upload(a, "soa"), fn), 9)
    err = np.abs(res - ref).max(1) / np.abs(ref).max(1)
    assert err.max() <= 1e-14, (fn, int(err.argmax()), err.max())


def test_binary32_storage(eig3):
    """binary32 storage: binary64 arithmetic on the widened entries, rounded
    once; against the exact f of the binary32 input."""
    c = w.differentiation_batch(512, seed=94)
    a32 = c["a"].astype(np.float32)
    res = download_matrix(eig3.eig3_matrix_function(upload(a32, "aos"), "exp"), 9)
    for m in range(0, 512, 8):
        ref = np.array(exact.matrix_function(a32[m].astype(np.float64), "exp"))
        assert _rel(res[m], ref) <= 4 * EPS32, m


def test_rejects(eig3):
    c = w.haar_general(16, seed=95)
    with pytest.raises(ValueError):
        eig3.eig3_matrix_function(upload(c["a"], "aos"), "sin")
    with pytest.raises(eig3.Eig3Error):
        eig3.eig3_matrix_function(upload(c["a"], "aos"), "exp", "general", "naive")


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("acc", ["fma", "compensated", "double_word"])
def test_backward_exp_general(eig3, layout, acc):
    """d<G, exp(A)>/dA against the exact Daleckii-Krein product (kappa <= 100,
    gaps >= 1e-3)."""
    c = w.differentiation_batch(600, seed=96)
    g = np.random.default_rng(97).standard_normal((600, 9))
    res = download_matrix(eig3.eig3_matrix_function_backward(upload(c["a"], layout), upload(g, layout), "exp",
                                                             "general", acc), 9)
    for m in range(0, 600, 6):
        ref = np.array(exact.matrix_function_vjp(c["a"][m], "exp", g[m]))
        assert _rel(res[m], ref) <= 1e-11, m


@pytest.mark.parametrize("fn", ["exp", "log", "sqrt"])
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_backward_symmetric_positive_definite(eig3, fn, layout):
    """Symmetric storage: g = dL/d(the 6 stored components of f(A)), the result
    dL/d(the 6 stored entries of A)."""
    a = _spd(300, 98)
    s = np.stack([a[:, 0], a[:, 4], a[:, 8], a[:, 1], a[:, 2], a[:, 5]], axis=1)
    g6 = np.random.default_rng(99).standard_normal((300, 6))
    res = download_matrix(eig3.eig3_matrix_function_backward(upload(s, layout), upload(g6, layout), fn,
                                                             "symmetric"), 6)
    for m in range(0, 300, 5):
        gf = np.array([[g6[m, 0], g6[m, 3] / 2, g6[m, 4] / 2], [g6[m, 3] / 2, g6[m, 1], g6[m, 5] / 2],
                       [g6[m, 4] / 2, g6[m, 5] / 2, g6[m, 2]]]).ravel()
        full = np.array(exact.matrix_function_vjp(a[m], fn, gf)).reshape(3, 3)
        ref = np.array([full[0, 0], full[1, 1], full[2, 2], full[0, 1] + full[1, 0], full[0, 2] + full[2, 0],
                        full[1, 2] + full[2, 1]])
        assert _rel(res[m], ref) <= 1e-13, (fn, m)


def test_autograd_against_torch_matrix_exp(eig3):
    """eig3.matrix_function(A, 'exp') and its backward against
    torch.linalg.matrix_exp and torch's autograd of it (an independent
    algorithm) on 4096 matrices of the differentiation batch."""
    import torch
    c = w.differentiation_batch(4096, seed=100)
    a0 = torch.tensor(c["a"].reshape(-1, 3, 3), dtype=torch.float64, device="cuda:0")
    wgt = torch.tensor(np.random.default_rng(101).standard_normal((4096, 3, 3)), dtype=torch.float64,
                       device="cuda:0")
    a1 = a0.clone().requires_grad_(True)
    f1 = eig3.matrix_function(a1, "exp")
    (f1 * wgt).sum().backward()
    a2 = a0.clone().requires_grad_(True)
    f2 = torch.linalg.matrix_exp(a2)
    (f2 * wgt).sum().backward()
    scale_f = f2.detach().abs().amax(dim=(1, 2))
    assert torch.all((f1 - f2).detach().abs().amax(dim=(1, 2)) <= 1e-11 * scale_f)
    scale_g = a2.grad.abs().amax(dim=(1, 2))
    assert torch.all((a1.grad - a2.grad).abs().amax(dim=(1, 2)) <= 1e-10 * scale_g)


@pytest.mark.parametrize("fn", ["exp", "log", "sqrt"])
def test_backward_coalescing_eigenvalues(eig3, fn):
    """The adjoint as eigenvalues coalesce, against the exact Daleckii-Krein
    product at 80 digits: nearly isotropic p I + delta S, a nearly double root
    at either end of the spectrum (symmetric), and nearly double roots of
    nonsymmetric matrices (kappa(V) = 10)."""
    rng = np.random.default_rng(102)

    def rot():
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        return q * np.sign(np.diag(r))

    mats = []
    for delta in (1e-4, 1e-9, 1e-13):
        for _ in range(20):
            p = rng.uniform(0.5, 2.0)
            sm = rng.standard_normal((3, 3))
            mats.append((p * np.eye(3) + delta * (sm + sm.T) / 2).ravel())
    for eps in (1e-7, 1e-13):
        for _ in range(20):
            q, b = rot(), rng.uniform(0.5, 1.5)
            c = b + rng.uniform(0.5, 2.0)
            mats.append((q @ np.diag([b, b * (1 + eps), c]) @ q.T).ravel())
            mats.append((q @ np.diag([b, c, c * (1 + eps)]) @ q.T).ravel())
            v = rot() @ np.diag([1.0, 10 ** -0.5, 0.1]) @ rot().T
            mats.append((v @ np.diag([b, b * (1 + eps), b + 1.0]) @ np.linalg.inv(v)).ravel())
    a = np.array(mats)
    g = rng.standard_normal(a.shape)
    res = download_matrix(eig3.eig3_matrix_function_backward(upload(a, "soa"), upload(g, "soa"), fn), 9)
    for m in range(len(a)):
        ref = np.array(exact.matrix_function_vjp(a[m], fn, g[m]))
        assert _rel(res[m], ref) <= 1e-13, (fn, m)


def test_backward_repeated_and_defective(eig3):
    """Exactly repeated eigenvalues of diagonal matrices, where the adjoint is
    f[d_i, d_j] G_ij (f' on equal entries), for exp, log and sqrt; and
    d<G, exp(A)>/dA for single Jordan blocks p I + N against torch's autograd
    of torch.linalg.matrix_exp (binary64 on the CPU)."""
    import torch
    rng = np.random.default_rng(103)
    diag = np.array([[1.0, 1.0, 1.0], [2.5, 2.5, 2.5], [1.0, 1.0, 2.0], [3.0, 0.5, 3.0], [0.25, 4.0, 4.0]])
    a = np.zeros((len(diag), 9))
    a[:, [0, 4, 8]] = diag
    g = rng.standard_normal(a.shape)
    funcs = {"exp": (np.exp, np.exp), "log": (np.log, lambda x: 1 / x), "sqrt": (np.sqrt, lambda x: 0.5 / np.sqrt(x))}
    for fn, (f, df) in funcs.items():
        res = download_matrix(eig3.eig3_matrix_function_backward(upload(a, "soa"), upload(g, "soa"), fn), 9)
        ref = np.zeros_like(a)
        for m, d in enumerate(diag):
            for i in range(3):
                for j in range(3):
                    x, y = d[i], d[j]
                    ref[m, 3 * i + j] = g[m, 3 * i + j] * (df(x) if x == y else (f(x) - f(y)) / (x - y))
        assert np.abs(res - ref).max() <= 1e-15 * np.abs(ref).max() * 8, fn
    p = rng.uniform(0.5, 2.0, 64)
    nil = np.zeros((64, 3, 3))
    nil[:, 0, 1], nil[:, 0, 2], nil[:, 1, 2] = rng.uniform(-3, 3, (3, 64))
    nil[32:] = nil[32:].transpose(0, 2, 1)
    a = (p[:, None, None] * np.eye(3) + nil).reshape(-1, 9)
    g = rng.standard_normal(a.shape)
    res = download_matrix(eig3.eig3_matrix_function_backward(upload(a, "soa"), upload(g, "soa"), "exp"), 9)
    at = torch.tensor(a.reshape(-1, 3, 3), requires_grad=True)
    torch.linalg.matrix_exp(at).backward(torch.tensor(g.reshape(-1, 3, 3)))
    ref = at.grad.numpy().reshape(-1, 9)
    err = np.abs(res - ref).max(1) / np.abs(ref).max(1)
    assert err.max() <= 1e-13, (int(err.argmax()), err.max())


def test_autograd_isotropic_log(eig3):
    """Hencky-type use: log of (nearly) isotropic stretch tensors through the
    autograd Function stays finite and matches the exact product; at A = p I
    the gradient of <G, log A> is G / p."""
    import torch
    a = torch.eye(3, dtype=torch.float64, device="cuda:0").repeat(8, 1, 1) * 1.5
    noise = np.random.default_rng(104).standard_normal((4, 3, 3))
    a[4:] += 1e-10 * torch.tensor(noise + noise.transpose(0, 2, 1), device="cuda:0")  # real spectrum
    a = a.requires_grad_(True)
    wgt = torch.tensor(np.random.default_rng(105).standard_normal((8, 3, 3)), dtype=torch.float64, device="cuda:0")
    (eig3.matrix_function(a, "log") * wgt).sum().backward()
    grad = a.grad.cpu().numpy()
    assert np.isfinite(grad).all()
    ref = wgt[:4].cpu().numpy() / 1.5
    assert np.abs(grad[:4] - ref).max() <= 4 * 2.0**-52 * np.abs(ref).max()
    ad = a.detach().cpu().numpy().reshape(-1, 9)
    for m in range(4, 8):
        ref = np.array(exact.matrix_function_vjp(ad[m], "log", wgt[m].cpu().numpy().ravel()))
        assert _rel(grad[m].ravel(), ref) <= 1e-13, m


@pytest.mark.parametrize("fn", ["exp", "log", "sqrt"])
def test_autograd_symmetric_storage(eig3, fn):
    """eig3.matrix_function_symmetric on (..., 6) storage against
    eig3.matrix_function on the full matrices built from the same six entries
    by differentiable torch ops, with the loss taken on the six components of
    F: same values, and the same gradient with respect to the stored entries."""
    import torch
    a = _spd(400, 106)
    s = np.stack([a[:, 0], a[:, 4], a[:, 8], a[:, 1], a[:, 2], a[:, 5]], axis=1).reshape(4, 100, 6)
    wgt = torch.tensor(np.random.default_rng(107).standard_normal((4, 100, 6)), device="cuda:0")
    s1 = torch.tensor(s, device="cuda:0").requires_grad_(True)
    f1 = eig3.matrix_function_symmetric(s1, fn)
    (f1 * wgt).sum().backward()
    s2 = torch.tensor(s, device="cuda:0").requires_grad_(True)
    rows = [torch.stack([s2[..., 0], s2[..., 3], s2[..., 4]], -1),
            torch.stack([s2[..., 3], s2[..., 1], s2[..., 5]], -1),
            torch.stack([s2[..., 4], s2[..., 5], s2[..., 2]], -1)]
    full = eig3.matrix_function(torch.stack(rows, -2), fn)
    f2 = torch.stack([full[..., 0, 0], full[..., 1, 1], full[..., 2, 2], full[..., 0, 1], full[..., 0, 2],
                      full[..., 1, 2]], -1)
    (f2 * wgt).sum().backward()
    assert f1.shape == s1.shape and s1.grad.shape == s1.shape
    assert torch.all((f1 - f2).detach().abs() <= 1e-13 * f2.detach().abs().amax(-1, keepdim=True))
    assert torch.all((s1.grad - s2.grad).abs() <= 1e-12 * s2.grad.abs().amax(-1, keepdim=True))
