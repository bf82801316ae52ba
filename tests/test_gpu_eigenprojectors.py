"""Eigenprojectors (eig3_eigenprojectors) against the exact Frobenius
covariants, their algebraic identities over a large batch, and the paper's
motivating use: a closed-form function of a matrix (the exponential)."""
import numpy as np
import pytest

import workloads as w
from gpu_util import upload
from oracle import exact

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("out_layout", ["soa", "aos"])
@pytest.mark.parametrize("acc", ["fma", "compensated", "double_word"])
def test_against_exact(eig3, layout, out_layout, acc):
    c = w.differentiation_batch(512, seed=81)
    res = eig3.eig3_eigenprojectors(upload(c["a"], layout), "general", acc, out_layout)
    if out_layout == "aos":
        e = res.cpu().numpy().reshape(-1, 27)
    else:
        e = np.stack([t.cpu().numpy() for t in res], axis=1)
    for m in range(0, 512, 8):
        ref = np.array(exact.eigenprojectors(c["a"][m]))
        assert np.abs(e[m] - ref).max() <= 1e-8 * np.abs(ref).max(), m


def test_identities_large_batch(eig3):
    """sum E_k = I and sum lambda_k E_k = A on 2^20 matrices."""
    c = w.differentiation_batch(1 << 20, seed=82)
    a = upload(c["a"], "aos")
    e = eig3.eig3_eigenprojectors(a).cpu().numpy().reshape(-1, 3, 3, 3)
    lam = eig3.eig3_eigvals(a).cpu().numpy()
    scale = np.abs(e).reshape(-1, 27).max(1)
    assert np.all(np.abs(e.sum(1) - np.eye(3)).reshape(-1, 9).max(1) <= 1e-10 * scale)
    rec = np.einsum("mk,mkij->mij", lam, e)
    err = np.abs(rec - c["a"].reshape(-1, 3, 3)).reshape(-1, 9).max(1)
    assert np.all(err <= 1e-10 * scale * np.abs(c["a"]).max(1))


def test_symmetric_components(eig3):
    s = w.stress_tensors(2048, seed=83)["s"]
    s = s[np.abs(s[:, 3:]).max(1) > 1.0]  # the generic half: well-separated spectra
    eg = eig3.eig3_eigenprojectors(upload(w.symmetric_to_general(s), "aos")).cpu().numpy()
    es = eig3.eig3_eigenprojectors(upload(s, "aos"), "symmetric").cpu().numpy()
    ref = np.stack([eg[..., 0], eg[..., 4], eg[..., 8], eg[..., 1], eg[..., 2], eg[..., 5]], axis=-1)
    assert np.abs(es - ref).max() <= 1e-9


def test_matrix_exponential(eig3):
    """exp(A) = sum_k exp(lambda_k) E_k against scipy.linalg.expm."""
    import scipy.linalg
    c = w.differentiation_batch(256, seed=84)
    a = upload(c["a"], "aos")
    e = eig3.eig3_eigenprojectors(a).cpu().numpy().reshape(-1, 3, 3, 3)
    lam = eig3.eig3_eigvals(a).cpu().numpy()
    ex = np.einsum("mk,mkij->mij", np.exp(lam), e)
    for m in range(0, 256, 4):
        ref = scipy.linalg.expm(c["a"][m].reshape(3, 3))
        assert np.abs(ex[m] - ref).max() <= 1e-8 * np.abs(ref).max()
