"""Full-size batches in the launch configuration the benchmark times:
sampled outputs against the exact oracle, properties on every output."""
import numpy as np
import pytest

import workloads as w
from accuracy import EPS64, Truth, check, check_g2, lam_errors
from gpu_util import download_lam, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


def _properties(a_gen, lam, kappa):
    """Ascending, finite, and sum(lambda) = tr(A) within 8x the bound on the
    sum of three eigenvalues."""
    assert np.isfinite(lam).all()
    assert np.all(np.diff(lam, axis=1) >= 0)
    tr = a_gen[:, 0] + a_gen[:, 4] + a_gen[:, 8]
    nrm = np.sqrt((a_gen * a_gen).sum(1))
    assert np.all(np.abs(lam.sum(1) - tr) <= 8 * 3 * kappa * nrm * EPS64 + 8 * 3 * nrm * EPS64)


@pytest.mark.parametrize("acc", ["fma", "compensated"])
def test_config2_full_2p24_sampled(eig3, plain_oracle, acc):
    n = 1 << 24
    c = w.config2(n)
    lam = download_lam(eig3.eig3_eigvals(upload(c["a"], "soa"), "general", acc, "soa"))
    _properties(c["a"], lam, c["kappa"][:, None][:, 0])
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, 1500, replace=False))
    t = Truth(c["a"][idx], c["kappa"][idx])
    el = lam_errors(t, lam[idx])
    bl = np.broadcast_to(t.bound_lam(), el.shape)
    good = c["kappa"][idx] <= 10
    check(el[good], bl[good], what=f"config2 2^24 kappa<=10 {acc}")
    al = lam_errors(t, plain_oracle.eigvals(c["a"][idx]))
    check_g2(el[~good], bl[~good], al[~good], what=f"config2 2^24 kappa=100 {acc} (G2)")


def test_config3_full_2p27_sampled(eig3):
    n = 1 << 27
    c = w.config3(n)
    s = c["s"]
    lam = download_lam(eig3.eig3_eigvals(upload(s, "soa"), "symmetric", "fma", "soa"))
    rng = np.random.default_rng(8)
    idx = np.sort(rng.choice(n, 1500, replace=False))
    a = w.symmetric_to_general(s[idx])
    t = Truth(a, np.ones(idx.size))
    check(lam_errors(t, lam[idx]), t.bound_lam(), what="config3 2^27 sampled")
    assert np.isfinite(lam).all()
    assert np.all(np.diff(lam, axis=1) >= 0)
    tr = s[:, 0] + s[:, 1] + s[:, 2]
    nrm = np.sqrt((s[:, :3] ** 2).sum(1) + 2 * (s[:, 3:] ** 2).sum(1))
    assert np.all(np.abs(lam.sum(1) - tr) <= 48 * nrm * EPS64)


@pytest.mark.parametrize("acc", ["fma", "compensated"])
def test_config4_full_2p27_f32_sampled(eig3, acc):
    from accuracy import EPS32
    n = 1 << 27
    s = w.config4(n)["s"]
    lam = download_lam(eig3.eig3_eigvals(upload(s, "soa"), "symmetric", acc, "soa"))
    assert np.isfinite(lam).all()
    assert np.all(np.diff(lam, axis=1) >= 0)
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(n, 1500, replace=False))
    a = w.symmetric_to_general(s[idx].astype(np.float64))
    t = Truth(a, np.ones(idx.size))
    check(lam_errors(t, lam[idx]), t.bound_lam(EPS32), what=f"config4 2^27 f32 sampled {acc}")
