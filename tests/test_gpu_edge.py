"""Degenerate and out-of-contract inputs on the GPU."""
import math

import numpy as np
import pytest

import workloads as w
from accuracy import Truth, check, inv_errors, lam_errors
from gpu_util import download_inv, download_lam, upload

pytestmark = pytest.mark.gpu

ACCS = ["fma", "compensated", "double_word"]


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


@pytest.mark.parametrize("acc", ACCS)
def test_scaled_identity_exact(eig3, acc):
    """fl(J2(alpha I)) = 0 exactly (the remark on Algorithm alg:J2-stable's
    exactness); J3 and Delta vanish, and lambda = I1/3 three times."""
    alphas = np.array([0.1, -3.7, 1e-300, 1e300, 12345.678, 0.0])
    a = np.zeros((alphas.size, 9))
    a[:, 0] = a[:, 4] = a[:, 8] = alphas
    inv = download_inv(eig3.eig3_invariants(upload(a, "soa"), "general", acc))
    assert np.all(inv[:, 1:] == 0.0)
    lam = download_lam(eig3.eig3_eigvals(upload(a, "aos"), "general", acc))
    assert np.all(lam == lam[:, :1])
    assert np.allclose(lam[:, 0], alphas, rtol=4 * 2.0 ** -53, atol=0)
    s = np.stack([alphas, alphas, alphas, 0 * alphas, 0 * alphas, 0 * alphas], axis=1)
    invs = download_inv(eig3.eig3_invariants(upload(s, "soa"), "symmetric", acc))
    assert np.all(invs[:, 1:] == 0.0)


@pytest.mark.parametrize("acc", ACCS)
def test_triangular_bitwise_equals_diagonal(eig3, acc):
    rng = np.random.default_rng(41)
    n = 5000
    d = rng.standard_normal((n, 3))
    off = rng.standard_normal((n, 3))
    up = np.zeros((n, 9)); lo = np.zeros((n, 9)); dg = np.zeros((n, 9))
    for m in (up, lo, dg):
        m[:, 0], m[:, 4], m[:, 8] = d[:, 0], d[:, 1], d[:, 2]
    up[:, 1], up[:, 2], up[:, 5] = off[:, 0], off[:, 1], off[:, 2]
    lo[:, 3], lo[:, 6], lo[:, 7] = off[:, 0], off[:, 1], off[:, 2]
    ref = download_inv(eig3.eig3_invariants(upload(dg, "soa"), "general", acc))
    for t in (up, lo):
        got = download_inv(eig3.eig3_invariants(upload(t, "soa"), "general", acc))
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("acc", ACCS)
def test_exact_repeated_roots(eig3, acc):
    cases = [[1, 1, 2], [2, 2, 2], [-1, 3, 3], [0.5, 0.5, -7.25], [1, 2, 3]]
    a = np.zeros((len(cases), 9))
    for i, c in enumerate(cases):
        a[i, 0], a[i, 4], a[i, 8] = c
    inv = download_inv(eig3.eig3_invariants(upload(a, "soa"), "general", acc))
    assert np.all(inv[:4, 3] == 0.0)      # Delta = 0 exactly for the repeated roots
    assert inv[4, 2] == 0.0               # J3 = 0 exactly for diag(1, 2, 3)
    lam = download_lam(eig3.eig3_eigvals(upload(a, "aos"), "general", acc))
    ref = np.sort(np.array(cases, dtype=np.float64), axis=1)
    assert np.allclose(lam, ref, rtol=0, atol=8 * 2.0 ** -53 * np.abs(ref).max(1, keepdims=True) * 3)


def test_nan_propagates_per_matrix(eig3):
    c = w.haar_general(300, seed=5)
    a = c["a"].copy()
    a[17, 4] = np.nan
    a[200, 2] = np.inf
    lam = download_lam(eig3.eig3_eigvals(upload(a, "aos")))
    assert np.all(np.isnan(lam[17]))
    assert not np.isfinite(lam[200]).all()
    good = np.ones(300, dtype=bool)
    good[[17, 200]] = False
    assert np.isfinite(lam[good]).all()


@pytest.mark.parametrize("acc", ACCS)
def test_complex_spectrum_stays_finite(eig3, acc):
    """Outside the precondition (a complex pair): Delta < 0 is clamped to 0,
    the results are finite, ascending, and still sum to the trace."""
    th = np.linspace(0.1, 3.0, 50)
    a = np.zeros((50, 9))
    a[:, 0] = np.cos(th); a[:, 1] = -np.sin(th); a[:, 3] = np.sin(th); a[:, 4] = np.cos(th); a[:, 8] = 0.3
    lam = download_lam(eig3.eig3_eigvals(upload(a, "aos"), "general", acc))
    assert np.isfinite(lam).all()
    assert np.all(np.diff(lam, axis=1) >= 0)
    assert np.allclose(lam.sum(1), 2 * np.cos(th) + 0.3, atol=1e-14)


def test_nan_off_diagonal_propagates(eig3):
    """A NaN off-diagonal entry (the trace stays finite) still gives NaN."""
    c = w.haar_general(64, seed=5)
    a = c["a"].copy()
    a[10, 1] = np.nan
    a[20, 7] = np.nan
    for acc in ACCS:
        lam = download_lam(eig3.eig3_eigvals(upload(a, "aos"), "general", acc))
        assert np.all(np.isnan(lam[[10, 20]]))
        assert np.isfinite(np.delete(lam, [10, 20], axis=0)).all()


def test_zero_matrix_and_empty_batch(eig3):
    import torch
    z = np.zeros((3, 9))
    assert np.all(download_lam(eig3.eig3_eigvals(upload(z, "aos"))) == 0.0)
    e = torch.empty((0, 9), dtype=torch.float64, device="cuda:0")
    out = eig3.eig3_eigvals(e)
    assert out.shape == (0, 3)
    inv = eig3.eig3_invariants(e)
    assert all(x.numel() == 0 for x in inv)


@pytest.mark.parametrize("scale", [1e-40, 1e-10, 1e10, 1e40])
def test_scaling_range(eig3, scale):
    """Delta is a sixth-degree form: entries up to ~1e50 keep it in range."""
    c = w.haar_general(500, seed=6)
    a = c["a"] * scale
    t = Truth(a, c["kappa"])
    lam = download_lam(eig3.eig3_eigvals(upload(a, "aos")))
    check(lam_errors(t, lam), t.bound_lam(), what=f"scale {scale}")
    inv = download_inv(eig3.eig3_invariants(upload(a, "soa")))
    check(inv_errors(t, inv), t.bound_inv(), what=f"invariants scale {scale}")
    assert math.isfinite(float(np.abs(inv).max()))


def test_output_tensors_validated(eig3):
    """Caller-supplied outputs of the wrong size, dtype or count are rejected
    by the binding before anything is launched."""
    import torch
    d = torch.device("cuda:0")
    f64 = torch.float64
    a = torch.zeros((100, 9), dtype=f64, device=d)
    s = torch.zeros((100, 6), dtype=f64, device=d)
    g = torch.zeros((100, 3), dtype=f64, device=d)
    bad = [
        lambda: eig3.eig3_eigvals(a, out=torch.empty((99, 3), dtype=f64, device=d)),
        lambda: eig3.eig3_eigvals(a, out=torch.empty((100, 3), dtype=torch.float32, device=d)),
        lambda: eig3.eig3_eigvals(a, out_layout="soa", out=[torch.empty(100, dtype=f64, device=d)] * 2),
        lambda: eig3.eig3_invariants(a, out=[torch.empty(100, dtype=f64, device=d) for _ in range(3)]),
        lambda: eig3.eig3_invariants(a, out=[torch.empty(n, dtype=f64, device=d) for n in (100, 100, 100, 50)]),
        lambda: eig3.eig3_eigvals_backward(a, g, out=torch.empty((100, 8), dtype=f64, device=d)),
        lambda: eig3.eig3_eigvals_backward(a, g[:50]),
        lambda: eig3.eig3_eigenprojectors(a, out=torch.empty((100, 3, 6), dtype=f64, device=d)),
        lambda: eig3.eig3_mohr_coulomb(s, 100.0, 10.0, out=(torch.empty(99, dtype=f64, device=d), None)),
        lambda: eig3.eig3_mohr_coulomb(s, 100.0, 10.0, out=(None, torch.empty((100, 9), dtype=f64, device=d))),
    ]
    for j, call in enumerate(bad):
        with pytest.raises(ValueError):
            call()
    # well-formed outputs still work
    lam = eig3.eig3_eigvals(a, out=torch.empty((100, 3), dtype=f64, device=d))
    assert torch.all(lam == 0)


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("structure", ["general", "symmetric"])
def test_binary64_full_range(eig3, acc, structure):
    """Binary64 batches are evaluated on A scaled by a power of two, so
    eigenvalues of 2^k A are exactly 2^k times those of A, and the adjoint and
    the eigenprojectors of 2^k A are those of A, over the whole binary64
    range (k = -900 .. 1000; without the scaling Delta ~ |A|^6 over- or
    underflows beyond about 2^+-160); sampled matrices at 2^-900 meet the
    bound against the exact oracle (at 2^1000 the oracle's own bound scales
    exceed binary64; there the exact relation to the scale-1 results is the
    check)."""
    import torch
    rng = np.random.default_rng(77)
    mats = []
    for _ in range(300):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        lam = np.sort(rng.uniform(-1.0, 1.0, 3))
        m = q @ np.diag(lam) @ q.T
        mats.append(m.ravel() if structure == "general" else
                    [m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2]])
    a = np.array(mats)
    g = rng.standard_normal((len(a), 3))
    dev = torch.device("cuda:0")
    at = torch.tensor(a, device=dev)
    gt = torch.tensor(g, device=dev)
    lam0 = eig3.eig3_eigvals(at, structure, acc, "aos")
    grad0 = eig3.eig3_eigvals_backward(at, gt, structure, acc)
    proj0 = eig3.eig3_eigenprojectors(at, structure, acc, "aos")
    for k in (-900, -300, 300, 1000):
        f = math.ldexp(1.0, k)  # exact power of two (a device pow need not be)
        ak = at * f
        lam = eig3.eig3_eigvals(ak, structure, acc, "aos")
        assert torch.equal(lam, lam0 * f), k
        assert torch.equal(eig3.eig3_eigvals_backward(ak, gt, structure, acc), grad0), k
        assert torch.equal(eig3.eig3_eigenprojectors(ak, structure, acc, "aos"), proj0), k
        if k == -900:
            full = w.symmetric_to_general(ak.cpu().numpy()) if structure == "symmetric" else ak.cpu().numpy()
            t = Truth(full[::10], np.ones(len(full[::10])))
            check(lam_errors(t, lam.cpu().numpy()[::10]), t.bound_lam(), what=f"2^{k} {structure} {acc}")


@pytest.mark.parametrize("acc", ACCS)
def test_matrix_function_wide_range(eig3, acc):
    """Functions of matrices take their eigenvalues from the invariants of
    the prescaled matrix (Delta ~ |A|^6 would over- or underflow beyond about
    2^+-170) and keep A's own entries otherwise: for symmetric positive
    definite A and s = 2^k, log(s A) = k log(2) I + log(A) and
    sqrt(s A) = 2^(k/2) sqrt(A) for k = -400 .. 400, and the adjoints scale as
    1/s and 2^(-k/2) for k = -150 .. 150 (their divided differences reach the
    fifth order, ~lambda^-5 for log, which leaves binary64 near 2^+-200)."""
    import torch
    rng = np.random.default_rng(78)
    mats = []
    for _ in range(200):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        m = q @ np.diag(np.sort(rng.uniform(0.5, 2.0, 3))) @ q.T
        mats.append(m.ravel())
    dev = torch.device("cuda:0")
    at = torch.tensor(np.array(mats), device=dev)
    gt = torch.tensor(rng.standard_normal((200, 9)), device=dev)
    eye = torch.eye(3, dtype=torch.float64, device=dev).reshape(1, 9)
    log0 = eig3.eig3_matrix_function(at, "log", "general", acc)
    sq0 = eig3.eig3_matrix_function(at, "sqrt", "general", acc)
    glog0 = eig3.eig3_matrix_function_backward(at, gt, "log", "general", acc)
    gsq0 = eig3.eig3_matrix_function_backward(at, gt, "sqrt", "general", acc)
    for k in (-400, -150, 150, 400):
        s = math.ldexp(1.0, k)
        h = math.ldexp(1.0, k // 2)
        ak = at * s
        lg = eig3.eig3_matrix_function(ak, "log", "general", acc)
        ref = log0 + k * math.log(2.0) * eye
        assert torch.all((lg - ref).abs() <= 1e-12 * (abs(k) + ref.abs().amax(1, keepdim=True))), k
        sq = eig3.eig3_matrix_function(ak, "sqrt", "general", acc)
        assert torch.all((sq - h * sq0).abs() <= 1e-13 * h * sq0.abs().amax(1, keepdim=True)), k
        if abs(k) > 150:
            continue
        gl = eig3.eig3_matrix_function_backward(ak, gt, "log", "general", acc)
        assert torch.all((gl * s - glog0).abs() <= 1e-12 * glog0.abs().amax(1, keepdim=True)), k
        gs = eig3.eig3_matrix_function_backward(ak, gt, "sqrt", "general", acc)
        assert torch.all((gs * h - gsq0).abs() <= 1e-12 * gsq0.abs().amax(1, keepdim=True)), k
