"""Pins of the plain binary64 implementation of the paper's algorithms
(oracle/eig3_plain.c) to the exact oracle, to exact-arithmetic special
cases and to the paper's printed examples."""
import os

import numpy as np
import pytest

import workloads as w
from oracle import exact

EPS = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append([float(v) for v in vals])
    return rows


def _ratios(plain, a, kappa):
    """max over the batch of |plain - exact| / (bound scale * eps) per output."""
    inv = plain.invariants(a)
    lam = plain.eigvals(a)
    worst = np.zeros(5)
    for m in range(a.shape[0]):
        ex = exact.invariants(a[m])
        b = exact.bound_scales(a[m])
        el = exact.eigvals_float(a[m])
        for k, key in enumerate(("I1", "J2", "J3", "Delta")):
            err = abs(inv[k][m] - float(ex[k]))
            worst[k] = max(worst[k], err / (b[key] * EPS) if b[key] > 0 else (0.0 if err == 0 else np.inf))
        err = max(abs(lam[m, k] - el[k]) for k in range(3))
        worst[4] = max(worst[4], err / (kappa[m] * b["lam"] * EPS))
    return worst


def _weights():
    from oracle import gen_formulas
    return np.array([w for w, _, _ in gen_formulas.factor_classes()], dtype=np.float64)


def test_integer_matrices_aux_vectors_exact(plain_oracle):
    """Small-integer matrices: every product and sum of Alg. alg:disc-stable is
    exact in binary64, so sum_i w_i u_i v_i must equal the exact Delta.  This
    pins each derived factor of dx (and the weights: the class sizes of the
    Cauchy-Binet minors, 9, 6, 6, 6, 8, 8, 8, 2 x 6 and 1, summing to 64)."""
    rng = np.random.default_rng(21)
    wts = _weights()
    assert sorted(wts.tolist()) == sorted([9, 6, 6, 6, 8, 8, 8, 2, 2, 2, 2, 2, 2, 1])
    for _ in range(300):
        a = rng.integers(-9, 10, 9).astype(np.float64)
        u, v = plain_oracle.aux_vectors(a)
        assert float(np.dot(wts * u, v)) == float(exact.invariants(a)[3])
        _, _, _, disc = plain_oracle.invariants(a)
        assert disc[0] == float(exact.invariants(a)[3])


def test_printed_r10_sign_breaks_identity(plain_oracle):
    """Documents the reading of r10: in the derived factor with the terms
    M01 d1 d2, -M01^2 M10 and M01 M02 M20 (the paper's r10), flipping its
    + M02 M21 d2 term to the printed - makes the sum of products differ from
    Delta."""
    from oracle import gen_formulas as g
    cls = g.factor_classes()
    # the class whose terms are M01 d1 d2, M02 M21 d2, M01^2 M10, M01 M02 M20
    want = {("M01", "d1", "d2"), ("M02", "M21", "d2"), ("M01", "M01", "M10"), ("M01", "M02", "M20")}
    idx = [i for i, (_, _, terms) in enumerate(cls)
           if {tuple(g.OFF_NAMES[j] for j in range(6) for _ in range(off[j])) +
               tuple(f"d{j}" for j in range(3) for _ in range(e[j])) for _, off, e in terms} == want]
    assert len(idx) == 1
    k = idx[0]
    assert [t[0] for t in cls[k][2] if t[2] == (0, 0, 1)] == [1]  # + M02 M21 d2
    rng = np.random.default_rng(22)
    wts = _weights()
    differs = 0
    for _ in range(50):
        a = rng.integers(-9, 10, 9).astype(np.float64)
        u, v = plain_oracle.aux_vectors(a)
        d2 = a[4] - a[8]
        up, vp = u.copy(), v.copy()
        up[k] -= 2 * a[2] * a[7] * d2          # M = A:   M02 = A02, M21 = A21
        vp[k] -= 2 * a[6] * a[5] * d2          # M = A^T: M02 = A20, M21 = A12
        differs += float(np.dot(wts * up, vp)) != float(exact.invariants(a)[3])
    assert differs >= 45


@pytest.mark.parametrize("which", ["Haar-similar batch", "stress tensors", "differentiation batch"])
def test_within_stability_bounds_well_conditioned(plain_oracle, which):
    """The paper reports its algorithms within the (C = 1) stability bounds for
    well-conditioned eigenbases; on kappa <= 10 the plain implementation stays
    within 8x of them, and a dropped term or a wrong sign would not."""
    if which == "Haar-similar batch":
        c = w.haar_general(300)
        a, kappa = c["a"], c["kappa"]
    elif which == "stress tensors":
        c = w.stress_tensors(300)
        a, kappa = w.symmetric_to_general(c["s"]), np.ones(300)
    else:
        c = w.differentiation_batch(600)
        sel = c["kappa"] <= 10
        a, kappa = c["a"][sel], c["kappa"][sel]
    worst = _ratios(plain_oracle, a, kappa)
    assert np.all(worst <= 8.0), worst


@pytest.mark.parametrize("kappa,factor", [(1.0, 8.0), (10.0, 32.0)])
def test_perturbation_sweep_buckets(plain_oracle, kappa, factor):
    """Perturbation-sweep buckets (all three spectra, delta down to 1e-16).
    With an orthogonal eigenbasis the algorithms stay within 8x of the C = 1
    bounds, as the paper reports for U_symm and U_1.  Its constant grows with
    the eigenbasis condition (Delta reaches about 10x at kappa = 10, and the
    paper reports bound violations for the ill-conditioned U_2), so kappa = 10
    is held to 32x here; kappa = 100 is left to the G2 rule of the GPU tests."""
    c = w.perturbation_sweep(9 * 60)
    sel = c["kappa"] == kappa
    worst = _ratios(plain_oracle, c["a"][sel], c["kappa"][sel])
    assert np.all(worst <= factor), worst


def test_paper_performance_example(plain_oracle):
    """The worked example of Sec. "Performance benchmarks": absolute error of
    about 1e-16 (tests/golden/paper_perf_example.txt)."""
    g = _read_golden("paper_perf_example.txt")
    a = np.array(g["A"]).ravel()
    lam = plain_oracle.eigvals(a)[0]
    ex = [float(x) for x in exact.eigvals(a)]
    # fl(A) has the prescribed spectrum up to the rounding of its entries
    assert np.allclose(ex, g["lambda"][0], atol=1e-15, rtol=0)
    err = np.abs(lam - ex).max()
    assert err <= 8 * g["abs_error_about"][0][0]
    # and within 8x of the eigenvalue bound with kappa_2(U1) = 2
    assert err <= 8 * g["kappa2_U1"][0][0] * np.linalg.norm(a) * EPS


def test_paper_j2_example(plain_oracle):
    """D1 path, U_symm, delta = 1e-16: J2 about 1e-32 with abs. error of order
    1e-48 (tests/golden/paper_j2_example.txt)."""
    g = _read_golden("paper_j2_example.txt")
    c = w.paper_path("D1", "symm", [g["delta"][0][0]])
    _, j2, _, _ = plain_oracle.invariants(c["a"])
    ex = float(exact.invariants(c["a"][0])[1])
    assert 0.1 * g["J2_about"][0][0] < ex < 10 * g["J2_about"][0][0]
    assert abs(j2[0] - ex) < 10 * g["J2_abs_error_order"][0][0]


def test_scaled_identity_exact_zero(plain_oracle):
    """fl(J2(alpha I)) = 0 (remark after Cor. cor:J2-rel-bwd-stability); J3 and
    Delta vanish too, and all three eigenvalues equal I1/3."""
    for alpha in (0.1, -3.7, 1e-300, 1e300, 12345.678):
        a = np.eye(3).ravel() * alpha
        i1, j2, j3, disc = plain_oracle.invariants(a)
        assert (j2[0], j3[0], disc[0]) == (0.0, 0.0, 0.0)
        lam = plain_oracle.eigvals(a)[0]
        assert np.all(lam == i1[0] / 3)
        assert np.allclose(lam, alpha, rtol=4 * EPS, atol=0)


def test_j3_singular_deviator_example(plain_oracle):
    """diag(1, 2, 3): exactly representable differences give J3 = 0 exactly
    (tests/golden/paper_j3_example.txt)."""
    g = _read_golden("paper_j3_example.txt")
    a = np.array(g["A"]).ravel()
    assert plain_oracle.invariants(a)[2][0] == g["J3"][0][0]
    assert np.allclose(plain_oracle.eigvals(a)[0], [1.0, 2.0, 3.0], rtol=0, atol=8 * np.linalg.norm(a) * EPS)


def test_triangular_bitwise_equals_diagonal(plain_oracle):
    """Off-diagonal products vanish exactly for triangular input, so the
    computed invariants equal those of the diagonal matrix bit for bit."""
    rng = np.random.default_rng(23)
    for _ in range(200):
        d = rng.standard_normal(3)
        off = rng.standard_normal(3)
        up = np.array([d[0], off[0], off[1], 0, d[1], off[2], 0, 0, d[2]])
        lo = np.array([d[0], 0, 0, off[0], d[1], 0, off[1], off[2], d[2]])
        dg = np.array([d[0], 0, 0, 0, d[1], 0, 0, 0, d[2]])
        ref = plain_oracle.invariants(dg)
        for t in (up, lo):
            got = plain_oracle.invariants(t)
            for x, y in zip(got, ref):
                assert x[0] == y[0]


def test_symmetric_discriminant_nonnegative(plain_oracle):
    """For symmetric input u = v bit for bit, so the computed Delta is a sum
    of nonnegative terms."""
    c = w.stress_tensors(20000)
    a = w.symmetric_to_general(c["s"])
    _, _, _, disc = plain_oracle.invariants(a)
    assert np.all(disc >= 0)


def test_ordering_and_spectral_sums(plain_oracle):
    """Ascending order; sum of eigenvalues equals I1 within the bound."""
    c = w.haar_general(20000)
    lam = plain_oracle.eigvals(c["a"])
    assert np.all(np.diff(lam, axis=1) >= 0)
    tr = c["a"][:, 0] + c["a"][:, 4] + c["a"][:, 8]
    nrm = np.linalg.norm(c["a"], axis=1)
    assert np.all(np.abs(lam.sum(1) - tr) <= 16 * nrm * EPS)


def test_backward_against_exact_and_eigenvectors(plain_oracle):
    """Eigenprojector backward vs the exact gradient and the eigenvector
    formula y_i x_i^T / (y_i^T x_i) from the generator's basis."""
    c = w.differentiation_batch(200, with_basis=True)
    grad = plain_oracle.eigvals_backward(c["a"], c["g"])
    for m in range(0, 200, 10):
        ref = exact.eigvals_vjp(c["a"][m], c["g"][m])
        scale = np.abs(ref).max()
        assert np.abs(grad[m] - ref).max() <= 1e-7 * scale
    v = c["v"].reshape(-1, 3, 3)
    vi = c["vinv"].reshape(-1, 3, 3)
    ev = np.einsum("mk,mki,mjk->mij", c["g"], vi, v).reshape(-1, 9)
    scale = np.abs(ev).max(axis=1)
    assert np.all(np.abs(grad - ev).max(axis=1) <= 1e-7 * scale)


def test_backward_identities(plain_oracle):
    """g = 1 -> I and g = lambda -> A^T."""
    c = w.differentiation_batch(500)
    one = plain_oracle.eigvals_backward(c["a"], np.ones((500, 3)))
    assert np.abs(one - np.eye(3).ravel()).max() < 1e-9
    lam = plain_oracle.eigvals(c["a"])
    at = plain_oracle.eigvals_backward(c["a"], lam)
    ref = c["a"].reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9)
    assert np.abs(at - ref).max() < 1e-8 * np.abs(ref).max()


def test_backward_central_differences(plain_oracle):
    """Central differences (h = 1e-6) of the plain eigenvalues."""
    c = w.differentiation_batch(50)
    grad = plain_oracle.eigvals_backward(c["a"], c["g"])
    h = 1e-6
    fd = np.zeros_like(grad)
    for e in range(9):
        ap = c["a"].copy(); ap[:, e] += h
        am = c["a"].copy(); am[:, e] -= h
        fd[:, e] = ((plain_oracle.eigvals(ap) - plain_oracle.eigvals(am)) * c["g"]).sum(1) / (ap[:, e] - am[:, e])
    scale = np.abs(grad).max(axis=1)
    assert np.all(np.abs(fd - grad).max(axis=1) <= 2e-3 * scale)


def test_threads_do_not_change_results(plain_oracle):
    c = w.haar_general(5000)
    assert np.array_equal(plain_oracle.eigvals(c["a"], threads=1), plain_oracle.eigvals(c["a"], threads=4))
