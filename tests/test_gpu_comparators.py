"""The paper's naive comparators on the GPU (accuracy="naive" and
"naive_tensor"): operation-for-operation parity with the plain oracle, and
the error levels the paper reports for them next to the stable path."""
import os

import numpy as np
import pytest

import workloads as w
from accuracy import EPS64, Truth, check, lam_errors
from gpu_util import download_inv, download_lam, upload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_naive_claims.txt")


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


@pytest.mark.parametrize("mode,variant", [("naive", "naive"), ("naive_tensor", "tensor")])
@pytest.mark.parametrize("structure", ["general", "symmetric"])
def test_bitwise_invariants(eig3, plain_oracle, mode, variant, structure):
    """Plain binary64 in the printed order on both sides: identical bits."""
    if structure == "general":
        a = np.concatenate([w.perturbation_sweep(3000, seed=61)["a"], w.haar_general(1000, seed=62)["a"]])
        dev = upload(a, "aos")
    else:
        s = w.stress_tensors(4000, seed=63)["s"]
        a = w.symmetric_to_general(s)
        dev = upload(s, "soa")
    inv = download_inv(eig3.eig3_invariants(dev, structure, mode))
    ref, lam_ref = plain_oracle.naive(a, variant)
    assert np.array_equal(inv, ref), np.argwhere(inv != ref)[:5]
    lam = download_lam(eig3.eig3_eigvals(dev, structure, mode, "aos"))
    # same invariants; the eigenvalue step differs only in its sqrt/atan/cos
    scale = np.abs(ref[:, :1]) + 2 * np.sqrt(np.maximum(3 * ref[:, 1:2], 0))
    assert np.all(np.abs(lam - lam_ref) <= 16 * EPS64 * scale + 1e-300)


def test_paper_error_levels(eig3):
    """Naive errors ~eps^(1/3) near a triple root and ~eps^(1/2) near a double
    root (tests/golden/paper_naive_claims.txt); the stable path within 8x its
    bound on the same matrices (orthogonal U_symm and U_1)."""
    g = _golden()
    deltas = 10.0 ** np.linspace(-16, -1, 121)
    for path, key in (("D1", "triple_root_error_about"), ("D2", "double_root_error_about")):
        for basis in ("symm", "U1"):
            c = w.paper_path(path, basis, deltas)
            t = Truth(c["a"], c["kappa"])
            stable = download_lam(eig3.eig3_eigvals(upload(c["a"], "soa"), "general", "fma", "soa"))
            check(lam_errors(t, stable), t.bound_lam(), what=f"stable {path}/{basis}")
            naive = download_lam(eig3.eig3_eigvals(upload(c["a"], "soa"), "general", "naive", "soa"))
            worst = lam_errors(t, naive).max()
            assert g[key] / 30 <= worst <= g[key] * 30, (path, basis, worst)


def test_naive_j3_example(eig3):
    """D1 path, U_1, delta ~ 1e-16: the naive J3 keeps an error of order 1e-16
    while the stable J3 stays within its bound."""
    g = _golden()
    c = w.paper_path("D1", "U1", [1e-16, 2e-16, 5e-16])
    t = Truth(c["a"], c["kappa"])
    naive = download_inv(eig3.eig3_invariants(upload(c["a"], "soa"), "general", "naive"))
    err = np.abs(naive[:, 2] - t.inv[:, 2]).max()
    assert g["naive_j3_error_order_at_delta_1e-16"] / 30 <= err <= g["naive_j3_error_order_at_delta_1e-16"] * 30
    stable = download_inv(eig3.eig3_invariants(upload(c["a"], "soa"), "general", "fma"))
    assert np.all(np.abs(stable[:, 2] - t.inv[:, 2]) <= 8 * t.bound_inv()[:, 2])


def test_comparators_reject_other_calls(eig3):
    import torch
    a = upload(w.haar_general(8, seed=1)["a"], "aos")
    g = torch.zeros((8, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(eig3.Eig3Error):
        eig3.eig3_eigvals_backward(a, g, "general", "naive")
    with pytest.raises(eig3.Eig3Error):
        eig3.eig3_eigvals(a.float(), "general", "naive_tensor")
