"""Mohr-Coulomb yield function and its gradient (eig3_mohr_coulomb) on the
GPU against the exact oracle, and the paper's pi-plane experiment: the naive
evaluation errs by up to ~1e-8 near the Lode angles k * 60 degrees while the
stable path stays near machine precision."""
import os

import numpy as np
import pytest

import workloads as w
from accuracy import EPS64
from gpu_util import download_matrix, upload
from oracle import exact

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_mohr_coulomb.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


def _pi_plane(n, j2):
    """sigma = U_symm diag(s_k) U_symm^T, s_k = (2/3) sqrt(3 J2) cos(theta + 2 pi k/3)."""
    th = np.linspace(0.0, 2 * np.pi, n, endpoint=False)
    u = w.paper_basis("symm")
    r = 2.0 / 3.0 * np.sqrt(3.0 * j2)
    a = np.empty((n, 9))
    for i, t in enumerate(th):
        s = r * np.cos(t + 2 * np.pi * np.arange(1, 4) / 3)
        a[i] = (u @ np.diag(s) @ u.T).ravel()
    return th, a


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_stress_states(eig3, layout, dtype):
    g = _golden()
    syc, m = g["S_yc"], g["S_yc"] / g["S_yt"]
    s = w.stress_tensors(600, seed=71)["s"]
    s = s[np.abs(s).max(1) < 1e3]  # the generic half and the near-isotropic half
    eps = EPS64
    if dtype == "f32":
        s = s.astype(np.float32)
        eps = 2.0 ** -24
    a = w.symmetric_to_general(s.astype(np.float64))
    f, dfds = eig3.eig3_mohr_coulomb(upload(s, layout), syc, m, "symmetric")
    f = f.double().cpu().numpy()
    dfds = download_matrix(dfds, 6)
    for i in range(0, len(a), 3):
        fe, ge = exact.mohr_coulomb(a[i], syc, m)
        nrm = np.linalg.norm(a[i])
        assert abs(f[i] - fe) <= 8 * (m + 1) / syc * nrm * eps + 8 * eps, (i, f[i], fe)
        lam = np.sort(np.real(exact.eigvals_float(a[i])))
        gap = min(lam[1] - lam[0], lam[2] - lam[1]) / max(nrm, 1e-300)
        if gap > 1e-6:
            gs = np.array(ge).reshape(3, 3)
            gs = 0.5 * (gs + gs.T)
            ref = np.array([gs[0, 0], gs[1, 1], gs[2, 2], gs[0, 1], gs[0, 2], gs[1, 2]])
            tol = (1e-9 if dtype == "f64" else 1e-5) * np.abs(ref).max() / min(gap * 1e3, 1.0)
            assert np.abs(dfds[i] - ref).max() <= tol, (i, dfds[i], ref)


def test_general_structure_and_no_gradient(eig3):
    g = _golden()
    syc, m = g["S_yc"], g["S_yc"] / g["S_yt"]
    c = w.haar_general(300, seed=72)
    f_only, none = eig3.eig3_mohr_coulomb(upload(c["a"], "aos"), syc, m, "general", grad=False)
    assert none is None
    f, grad = eig3.eig3_mohr_coulomb(upload(c["a"], "aos"), syc, m, "general")
    assert np.array_equal(f_only.cpu().numpy(), f.cpu().numpy())
    grad = grad.cpu().numpy().reshape(-1, 9)
    for i in range(0, 300, 10):
        fe, ge = exact.mohr_coulomb(c["a"][i], syc, m)
        assert abs(f.cpu().numpy()[i] - fe) <= 8 * (m + 1) / syc * np.linalg.norm(c["a"][i]) * EPS64 + 1e-15
        np.testing.assert_allclose(grad[i], ge, rtol=0, atol=1e-9 * np.abs(ge).max())


def test_pi_plane_naive_vs_stable(eig3):
    """The paper's pi-plane experiment (tests/golden/paper_mohr_coulomb.txt)."""
    g = _golden()
    syc, m = g["S_yc"], g["S_yc"] / g["S_yt"]
    th, a = _pi_plane(720, g["J2"])
    fe = np.array([exact.mohr_coulomb(x, syc, m)[0] for x in a])
    stable, _ = eig3.eig3_mohr_coulomb(upload(a, "soa"), syc, m, "general", "fma", grad=False)
    naive, _ = eig3.eig3_mohr_coulomb(upload(a, "soa"), syc, m, "general", "naive", grad=False)
    es = np.abs(stable.cpu().numpy() - fe)
    en = np.abs(naive.cpu().numpy() - fe)
    assert es.max() <= 30 * g["present_error_about"], es.max()
    assert g["naive_max_error_about"] / 30 <= en.max() <= g["naive_max_error_about"] * 30, en.max()
    # the naive errors peak next to the Lode angles k * 60 degrees
    worst = th[np.argsort(en)[-10:]]
    dist = np.abs(((np.degrees(worst) + 30) % 60) - 30)
    assert np.median(dist) < 5.0, np.degrees(worst)


def test_invalid_parameters(eig3):
    s = upload(w.stress_tensors(8, seed=1)["s"], "aos")
    for syc, m in ((0.0, 10.0), (100.0, -1.0), (float("nan"), 2.0)):
        with pytest.raises(eig3.Eig3Error):
            eig3.eig3_mohr_coulomb(s, syc, m, "symmetric")


@pytest.mark.parametrize("acc", ["fma", "compensated", "double_word"])
def test_binary64_scale_invariance(eig3, acc):
    """Binary64 stresses are evaluated on sigma scaled by a power of two:
    with sigma and S_yc both scaled by 2^k, f is bitwise unchanged and
    df/dsigma scales by exactly 2^-k, from 2^-900 to 2^900 (where the
    unscaled discriminant would over- or underflow; S_yc itself is limited
    to 1e300)."""
    import math

    import torch
    g = _golden()
    syc, m = g["S_yc"], g["S_yc"] / g["S_yt"]
    rng = np.random.default_rng(81)
    s = rng.standard_normal((500, 6)) * 50.0
    st = torch.tensor(s, device="cuda:0")
    f0, d0 = eig3.eig3_mohr_coulomb(st, syc, m, "symmetric", acc)
    for k in (-900, -300, 300, 900):
        fac = math.ldexp(1.0, k)  # exact power of two
        f, d = eig3.eig3_mohr_coulomb(st * fac, syc * fac, m, "symmetric", acc)
        assert torch.equal(f, f0), k
        assert torch.equal(d, d0 * math.ldexp(1.0, -k)), k
