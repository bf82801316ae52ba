"""binary32 storage (EIG3_F32): eigenvalues against the exact oracle at the
binary32 input widened to binary64, with the binary32 unit roundoff in the
bounds.  Every evaluation is checked: "fma" (the paper's algorithms in
binary64 on the widened entries), "double_word" (K2, K3 and Delta from
them in binary64 on the widened entries) and "compensated" (K2, K3 with
binary32 error-free products and sums, binary64 Delta accumulation)."""
import numpy as np
import pytest

import workloads as w
from accuracy import EPS32, Truth, check, inv_errors, lam_errors
from oracle import exact
from gpu_util import download_inv, download_lam, upload

pytestmark = pytest.mark.gpu

ACCS = ["fma", "compensated", "double_word"]
F32_TINY = np.finfo(np.float32).tiny


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


@pytest.fixture(scope="module")
def c4():
    c = w.stress_tensors_f32(1500)
    s = c["s"]  # float32
    a = w.symmetric_to_general(s.astype(np.float64))
    return s, Truth(a, np.ones(a.shape[0]))


@pytest.fixture(scope="module")
def c1f():
    c = w.haar_general(1500)
    a32 = c["a"].astype(np.float32)
    return a32, Truth(a32.astype(np.float64), c["kappa"])


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_stress_tensors_f32_symmetric_f32(eig3, c4, acc, layout):
    s, t = c4
    lam = download_lam(eig3.eig3_eigvals(upload(s, layout), "symmetric", acc, "soa"))
    check(lam_errors(t, lam), t.bound_lam(EPS32), what=f"binary32 stress tensors f32 eigvals {acc} {layout}")
    assert np.all(np.diff(lam, axis=1) >= 0)


@pytest.mark.parametrize("acc", ACCS)
def test_stress_tensors_f32_invariants_f32(eig3, c4, acc):
    """I1 and J2 everywhere; J3 and Delta where the result is a binary32
    normal number (below, the subnormal spacing exceeds the bound)."""
    s, t = c4
    inv = download_inv(eig3.eig3_invariants(upload(s, "soa"), "symmetric", acc))
    err = inv_errors(t, inv)
    b = t.bound_inv(EPS32)
    normal = np.abs(t.inv) >= F32_TINY
    normal[:, :2] = True
    check(np.where(normal, err, 0.0), b, what=f"binary32 stress tensors f32 invariants {acc}")


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_general_f32(eig3, c1f, acc, layout):
    a32, t = c1f
    lam = download_lam(eig3.eig3_eigvals(upload(a32, layout), "general", acc, "aos"))
    check(lam_errors(t, lam), t.bound_lam(EPS32), what=f"general f32 eigvals {acc} {layout}")


@pytest.mark.parametrize("n", [1, 63, 257, 1000])
def test_f32_ragged(eig3, n):
    c = w.stress_tensors_f32(n, seed=91)
    s = c["s"]
    t = Truth(w.symmetric_to_general(s.astype(np.float64)), np.ones(n))
    for acc in ACCS:
        for layout in ("soa", "aos"):
            lam = download_lam(eig3.eig3_eigvals(upload(s, layout), "symmetric", acc, "aos"))
            check(lam_errors(t, lam), t.bound_lam(EPS32), what=f"f32 ragged n={n} {acc} {layout}")


@pytest.mark.parametrize("structure", ["symmetric", "general"])
@pytest.mark.parametrize("acc", ACCS)
def test_f32_two_per_lane(eig3, structure, acc):
    """binary32 structure-of-arrays eigenvalues with every array 8-byte aligned
    take two adjacent matrices per lane in spans of 512, with a one-per-lane
    ragged last span; arrays that are only 4-byte aligned take the
    one-per-lane kernel.  The arithmetic per matrix is the same, so both give
    bitwise equal eigenvalues, and both meet the bound."""
    import torch
    for n in (1, 2, 511, 512, 513, 1024 + 37, 5 * 512):
        if structure == "symmetric":
            a32 = w.stress_tensors_f32(n, seed=95)["s"]
            t = Truth(w.symmetric_to_general(a32.astype(np.float64)), np.ones(n))
        else:
            c = w.haar_general(n, seed=95)
            a32 = c["a"].astype(np.float32)
            t = Truth(a32.astype(np.float64), c["kappa"])
        aligned = [x.clone() for x in upload(a32, "soa")]  # own allocations
        shifted = []
        for x in aligned:  # the same values one element into a larger buffer
            buf = torch.empty(n + 1, dtype=torch.float32, device=x.device)
            buf[1:] = x
            shifted.append(buf[1:])
        assert all(x.data_ptr() % 8 == 0 for x in aligned) and shifted[0].data_ptr() % 8 == 4
        pair = download_lam(eig3.eig3_eigvals(aligned, structure, acc, "soa"))
        one = download_lam(eig3.eig3_eigvals(shifted, structure, acc, "soa"))
        assert np.array_equal(pair, one, equal_nan=True), (structure, acc, n)
        check(lam_errors(t, pair), t.bound_lam(EPS32), what=f"f32 two per lane {structure} {acc} n={n}")


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_f32_backward(eig3, layout):
    """binary32 adjoint: binary64 arithmetic on the widened entries, rounded
    once; against the exact gradient at the binary32 input."""
    c = w.differentiation_batch(2048, seed=33)
    a32 = c["a"].astype(np.float32)
    g32 = c["g"].astype(np.float32)
    from gpu_util import download_matrix
    grad = download_matrix(eig3.eig3_eigvals_backward(upload(a32, layout), upload(g32, "aos"), "general"), 9)
    idx = np.arange(0, 2048, 16)
    ref = np.array([exact.eigvals_vjp(a32[m].astype(np.float64), g32[m].astype(np.float64)) for m in idx])
    rel = np.abs(grad[idx] - ref).max(1) / np.abs(ref).max(1)
    assert rel.max() <= 4 * EPS32, rel.max()
    s = w.stress_tensors(1024, seed=34)["s"].astype(np.float32)
    gs = np.random.default_rng(3).standard_normal((1024, 3)).astype(np.float32)
    gsym = download_matrix(eig3.eig3_eigvals_backward(upload(s, layout), upload(gs, "soa"), "symmetric"), 6)
    assert np.isfinite(gsym[np.abs(gsym).max(1) < 1e30]).all()


def _scaled_symmetric(k: int, n: int = 400, seed: int = 93) -> np.ndarray:
    """Symmetric binary32 matrices scaled by 2^k (exact in binary32: every
    entry stays a normal number): half random, half near a repeated root."""
    rng = np.random.default_rng([seed, k + 1000])
    s = 100.0 * rng.standard_normal((n, 6))
    half = n // 2
    s[half:, :3] = 100.0 * rng.standard_normal((n - half, 1))
    s[half:] += 1e-2 * rng.standard_normal((n - half, 6))
    s32 = (s * 2.0 ** k).astype(np.float32)
    assert np.all(np.abs(s32) >= F32_TINY) and np.isfinite(s32).all()
    return s32


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("k", [-100, -60, 0, 60, 100])
def test_f32_power_of_two_scales(eig3, acc, k):
    """J2 and Delta span about 2^(2k) and 2^(6k) (far outside binary32 for
    |k| >= 60); the square roots and the arctangent quotient run on values
    brought back by exact powers of two, so the relative accuracy is the same
    at every scale."""
    s = _scaled_symmetric(k)
    t = Truth(w.symmetric_to_general(s.astype(np.float64)), np.ones(s.shape[0]))
    for layout in ("soa", "aos"):
        lam = download_lam(eig3.eig3_eigvals(upload(s, layout), "symmetric", acc, "soa"))
        check(lam_errors(t, lam), t.bound_lam(EPS32), what=f"f32 scale 2^{k} {acc} {layout}")
        assert np.all(np.diff(lam, axis=1) >= 0)


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_f32_compensated_scaling_window(eig3, c4, layout):
    """The binary32-compensated evaluation scales the deviatoric data by a
    power of two unless every matrix of the wave has its largest magnitude in
    [2^-10, 2^36).  The stress tensors lie inside that window; the same
    tensors are evaluated once alone (every wave skips the scaling) and once
    with every 64th tensor replaced by a copy times 2^100 (every wave that
    holds one scales all its matrices): both runs are within the bounds of
    the exact eigenvalues, and the replaced tensors within theirs."""
    s, t = c4
    lam_skip = download_lam(eig3.eig3_eigvals(upload(s, layout, "symmetric"), "symmetric", "compensated", "soa"))
    mixed = s.copy()
    far = np.arange(0, s.shape[0], 64)
    mixed[far] = (s[far].astype(np.float64) * 2.0 ** 100).astype(np.float32)
    lam_mix = download_lam(eig3.eig3_eigvals(upload(mixed, layout, "symmetric"), "symmetric", "compensated", "soa"))
    keep = np.setdiff1d(np.arange(s.shape[0]), far)
    b = t.bound_lam(EPS32)
    err_skip, err_mix = lam_errors(t, lam_skip), lam_errors(t, lam_mix)
    check(err_skip, b, what=f"f32 compensated, no scaling ({layout})")
    check(err_mix[keep], b[keep], what=f"f32 compensated, scaled waves ({layout})")
    tf = Truth(w.symmetric_to_general(mixed[far].astype(np.float64)), np.ones(far.size))
    check(lam_errors(tf, lam_mix[far]), tf.bound_lam(EPS32), what=f"f32 compensated, 2^100 tensors ({layout})")


@pytest.mark.parametrize("acc", ACCS)
def test_f32_special_matrices(eig3, acc):
    """Zero, scaled identity (J2 = 0), exact double roots (Delta = 0), J3 = 0
    at tiny and huge scales (Delta alone sets the angle), a scaled identity
    with off-diagonal entries near 2^-51 (J3 near the binary32 subnormal
    range, Delta = 0), and NaN in a diagonal or an off-diagonal entry (NaN in
    that matrix only)."""
    diag = [(0, 0, 0), (3, 3, 3), (1, 1, 2), (-2, 1, 1), (1, 2, 3), (-5e30, -5e30, 7e30),
            (2.0 ** -100, 2.0 ** -99, 3 * 2.0 ** -100), (2.0 ** 100, 2.0 ** 101, 3 * 2.0 ** 100),
            (97.2, 97.2, 97.2), (1, 2, 3), (4, 5, 6)]
    g = np.zeros((len(diag), 9), dtype=np.float32)
    for i, d in enumerate(diag):
        g[i, 0], g[i, 4], g[i, 8] = d
    off = np.float32(2.0 ** -51) * np.array([1.03, -1.88, 1.01], dtype=np.float32)
    g[8, [1, 3]], g[8, [2, 6]], g[8, [5, 7]] = off[0], off[1], off[2]
    g[9, 4] = np.nan
    g[10, 5] = g[10, 7] = np.nan
    lam = download_lam(eig3.eig3_eigvals(upload(g, "soa"), "general", acc, "soa"))
    assert np.all(lam[0] == 0.0) and np.all(lam[1] == 3.0)
    t = Truth(g[:9].astype(np.float64), np.ones(9))
    check(lam_errors(t, lam[:9]), t.bound_lam(EPS32), what=f"f32 special matrices {acc}")
    assert np.isnan(lam[9:]).all()
    # the same matrices tiled over full 512-matrix spans of the two-per-lane
    # kernel (and its ragged tail): the same values at every copy
    reps = 100
    tiled = download_lam(eig3.eig3_eigvals(upload(np.tile(g, (reps, 1)), "soa"), "general", acc, "soa"))
    assert np.array_equal(tiled, np.tile(lam, (reps, 1)), equal_nan=True)


@pytest.mark.parametrize("acc", ACCS)
def test_general_invariants_f32(eig3, c1f, acc):
    """General binary32 invariants (nonsymmetric storage path) against the
    exact invariants of the binary32 input; J3 and Delta where binary32
    normal, as for the symmetric batch."""
    a32, t = c1f
    inv = download_inv(eig3.eig3_invariants(upload(a32, "soa"), "general", acc))
    err = inv_errors(t, inv)
    normal = np.abs(t.inv) >= F32_TINY
    normal[:, :2] = True
    check(np.where(normal, err, 0.0), t.bound_inv(EPS32), what=f"general f32 invariants {acc}")


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_eigenprojectors_f32(eig3, layout):
    """binary32 eigenprojectors: binary64 arithmetic on the widened entries,
    rounded once; against the exact Frobenius covariants of the binary32
    input (well-separated spectra, kappa <= 100)."""
    c = w.differentiation_batch(256, seed=85)
    a32 = c["a"].astype(np.float32)
    e = eig3.eig3_eigenprojectors(upload(a32, layout), "general", "fma", "aos").double().cpu().numpy()
    e = e.reshape(-1, 27)
    for m in range(0, 256, 4):
        ref = np.array(exact.eigenprojectors(a32[m].astype(np.float64)))
        assert np.abs(e[m] - ref).max() <= 4 * EPS32 * np.abs(ref).max(), m
