"""Truth subsets of 4096 matrices for every (spectrum, kappa) bucket of the
perturbation sweep: its three spectra (1, 1+d, 1+2d;
1, 1, 1+d; I + d S) times kappa(V) in {1, 10, 100}, d = 10^U(-16, -1),
9 x 4096 = 36 864 matrices against the exact invariants and 80-digit
eigenvalues of the stored matrices.  Gates per bucket: `compensated`
within 8x the bounds (G1) for eigenvalues, J2, J3 and Delta at every kappa;
`fma` G1 for the eigenvalues at kappa <= 10 and for the invariants at
kappa = 1, else no worse than 8 + 2x the worst ratio of the paper's own
algorithm (the plain binary64 oracle) on the same bucket (G2)."""
import numpy as np
import pytest

import workloads as w
from accuracy import Truth, check, check_g2, inv_errors, lam_errors
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
    return c, t, lam_errors(t, o1_lam), inv_errors(t, o1_inv)


@pytest.mark.parametrize("acc", ["fma", "compensated"])
def test_buckets_of_4096(sweep, acc):
    import paper_2511_00292_amd as eig3
    c, t, al_all, ai_all = sweep
    a_dev = upload(c["a"], "soa")
    lam = download_lam(eig3.eig3_eigvals(a_dev, "general", acc, "soa"))
    inv = download_inv(eig3.eig3_invariants(a_dev, "general", acc))
    el_all, ei_all = lam_errors(t, lam), inv_errors(t, inv)
    bl_all, bi_all = t.bound_lam(), t.bound_inv()
    for v, name in enumerate(SPECTRA):
        for kappa in (1.0, 10.0, 100.0):
            sel = (c["variant"] == v) & (c["kappa"] == kappa)
            assert sel.sum() == PER_BUCKET, (name, kappa, int(sel.sum()))
            el, ei = el_all[sel], ei_all[sel]
            bl, bi = np.broadcast_to(bl_all[sel], el.shape), bi_all[sel]
            what = f"{name} kappa={kappa:g} {acc}"
            if acc == "compensated" or kappa <= 10.0:
                check(el, bl, what=f"{what} eigvals (G1)")
            else:
                check_g2(el, bl, al_all[sel], what=f"{what} eigvals (G2)", pool=True)
            # I1, J2, J3, Delta
            if acc == "compensated" or kappa == 1.0:
                check(ei, bi, what=f"{what} invariants (G1)")
            else:
                check_g2(ei, bi, ai_all[sel], what=f"{what} invariants (G2)")
