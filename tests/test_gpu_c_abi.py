"""The C ABI from a plain C program (tests/c_abi/c_caller.c): hipMalloc'd
structure-of-arrays buffers, a stream of its own, eig3_invariants,
eig3_eigvals and eig3_eigvals_backward, a rejected call, no Python in the
caller.  Its results equal the Python binding's bit for bit (same kernels,
same inputs) and meet the exact oracle's gates."""
import os
import subprocess

import numpy as np
import pytest

import workloads as w
from accuracy import Truth, check, check_g12, lam_errors
from gpu_util import download_inv, download_lam, download_matrix, upload
from oracle import exact

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "c_caller")


def test_c_caller_matches_binding_and_oracle(tmp_path, plain_oracle):
    import paper_2511_00292_amd as eig3
    n = 3000  # a ragged tail after 11 full workgroup spans
    c = w.differentiation_batch(n, seed=61)
    f = {k: str(tmp_path / f"{k}.bin") for k in ("a", "g", "lam", "inv", "grad")}
    np.ascontiguousarray(c["a"], dtype=np.float64).tofile(f["a"])
    np.ascontiguousarray(c["g"], dtype=np.float64).tofile(f["g"])
    print("c_caller", n, flush=True)
    r = subprocess.run([EXE, str(n), f["a"], f["g"], f["lam"], f["inv"], f["grad"]],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lam_c = np.fromfile(f["lam"]).reshape(n, 3)
    inv_c = np.fromfile(f["inv"]).reshape(n, 4)
    grad_c = np.fromfile(f["grad"]).reshape(n, 9)

    a_dev = upload(c["a"], "soa")
    lam_p = download_lam(eig3.eig3_eigvals(a_dev, "general", "double_word", "soa"))
    inv_p = download_inv(eig3.eig3_invariants(a_dev, "general", "double_word"))
    grad_p = download_matrix(eig3.eig3_eigvals_backward(a_dev, upload(c["g"], "soa"), "general", "double_word"), 9)
    assert np.array_equal(lam_c, lam_p)
    assert np.array_equal(inv_c, inv_p)
    assert np.array_equal(grad_c, grad_p)

    idx = np.arange(0, n, 5)
    t = Truth(c["a"][idx], c["kappa"][idx])
    check(lam_errors(t, lam_c[idx]), t.bound_lam(), what="C caller eigvals (T8)")
    check_g12(lam_c[idx], plain_oracle.eigvals(c["a"][idx]), t.lam.real, t.bound_lam(), what="C caller eigvals (G1/G2)")
    for m in idx[::10]:
        ref = np.array(exact.eigvals_vjp(c["a"][m], c["g"][m]))
        assert np.abs(grad_c[m] - ref).max() <= 1e-7 * np.abs(ref).max(), m
