"""Truth subsets of 4096 matrices for every (spectrum, kappa) bucket of the
perturbation sweep: its three spectra (1, 1+d, 1+2d; 1, 1, 1+d; I + d S)
times kappa(V) in {1, 10, 100}, d = 10^U(-16, -1), 9 x 4096 = 36 864
matrices against the plain binary64 oracle (O1) and the exact invariants and
80-digit eigenvalues of the stored matrices (O2).  Gates (tests/accuracy.py),
elementwise on every matrix and output:

  double_word, compensated: G1/G2 and T8 (within 8x the bound of the exact
      result) for eigenvalues, I1, J2, J3 and Delta at every kappa;
  fma: G1/G2 for every output at kappa <= 10, T8 for the eigenvalues at
      kappa <= 10 and for every output at kappa = 1.  At kappa = 100 fma is
      not claimed (it fails G1 and G2 on some J3, Delta and eigenvalue
      elements; counted in the accuracy report)."""
import numpy as np
import pytest

import workloads as w
from accuracy import Truth, check, check_g12
from gpu_util import download_inv, download_lam, upload

pytestmark = pytest.mark.gpu

PER_BUCKET = 4096
SPECTRA = ("diag(1, 1+d, 1+2d)", "diag(1, 1, 1+d)", "I + d S")


@pytest.fixture(scope="module")
def sweep(plain_oracle):
    c = w.perturbation_sweep(9 * PER_BUCKET)
    t = Truth(c["a"], c["kappa"])
    o1_lam = plain_oracle.eigvals(c["a"])
    o1_inv = np.stack(plain_oracle.invariants(c["a"]), axis=1)
    return c, t, o1_lam, o1_inv


@pytest.mark.parametrize("acc", ["fma", "compensated", "double_word"])
def test_buckets_of_4096(sweep, acc):
    import paper_2511_00292_amd as eig3
    c, t, o1_lam, o1_inv = sweep
    a_dev = upload(c["a"], "soa")
    lam = download_lam(eig3.eig3_eigvals(a_dev, "general", acc, "soa"))
    inv = download_inv(eig3.eig3_invariants(a_dev, "general", acc))
    bl_all, bi_all = t.bound_lam(), t.bound_inv()
    for v, name in enumerate(SPECTRA):
        for kappa in (1.0, 10.0, 100.0):
            sel = (c["variant"] == v) & (c["kappa"] == kappa)
            assert sel.sum() == PER_BUCKET, (name, kappa, int(sel.sum()))
            what = f"{name} kappa={kappa:g} {acc}"
            if acc == "fma" and kappa > 10.0:
                assert np.all(np.diff(lam[sel], axis=1) >= 0)
                continue
            bl, bi = bl_all[sel], bi_all[sel]
            check_g12(lam[sel], o1_lam[sel], t.lam.real[sel], bl, what=f"{what} eigvals (G1/G2)")
            check_g12(inv[sel], o1_inv[sel], t.inv[sel], bi, what=f"{what} invariants (G1/G2)")
            check(np.abs(lam[sel] - t.lam.real[sel]), bl, what=f"{what} eigvals (T8)")
            if acc != "fma" or kappa == 1.0:
                check(np.abs(inv[sel] - t.inv[sel]), bi, what=f"{what} invariants (T8)")
