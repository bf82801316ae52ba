"""GPU parity of the forward path (eig3_invariants, eig3_eigvals) against the
exact oracle, through the C ABI.  Gates G1/G2 are defined in tests/accuracy.py."""
import numpy as np
import pytest

import workloads as w
from accuracy import Truth, check, check_g2, inv_errors, lam_errors
from gpu_util import download_inv, download_lam, upload

pytestmark = pytest.mark.gpu

ACCS = ["fma", "compensated"]


@pytest.fixture(scope="module")
def eig3():
    import paper_2511_00292_amd as m
    return m


@pytest.fixture(scope="module")
def c1():
    c = w.haar_general(1200)
    return c, Truth(c["a"], c["kappa"])


@pytest.fixture(scope="module")
def c2():
    c = w.perturbation_sweep(9 * 200)
    return c, Truth(c["a"], c["kappa"])


@pytest.fixture(scope="module")
def c3():
    c = w.stress_tensors(1200)
    a = w.symmetric_to_general(c["s"])
    return c, Truth(a, np.ones(a.shape[0]))


@pytest.fixture(scope="module")
def c5():
    c = w.differentiation_batch(1200)
    return c, Truth(c["a"], c["kappa"])


@pytest.fixture(scope="module")
def plain(plain_oracle):
    return plain_oracle


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("out_layout", ["soa", "aos"])
def test_haar_general_eigvals(eig3, c1, acc, layout, out_layout):
    c, t = c1
    lam = download_lam(eig3.eig3_eigvals(upload(c["a"], layout), "general", acc, out_layout))
    check(lam_errors(t, lam), t.bound_lam(), what=f"Haar-similar batch eigvals {acc} {layout}->{out_layout}")
    assert np.all(np.diff(lam, axis=1) >= 0)


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_haar_general_invariants(eig3, c1, acc, layout):
    c, t = c1
    inv = download_inv(eig3.eig3_invariants(upload(c["a"], layout), "general", acc))
    check(inv_errors(t, inv), t.bound_inv(), what=f"Haar-similar batch invariants {acc} {layout}")


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("kappa", [1.0, 10.0, 100.0])
def test_perturbation_sweep_buckets(eig3, plain, c2, acc, kappa):
    """Perturbation sweep: all three spectra, delta in [1e-16, 1e-1]."""
    c, t = c2
    sel = c["kappa"] == kappa
    a = c["a"]
    lam = download_lam(eig3.eig3_eigvals(upload(a, "soa"), "general", acc, "soa"))
    inv = download_inv(eig3.eig3_invariants(upload(a, "soa"), "general", acc))
    o1_lam = plain.eigvals(a)
    o1_inv = np.stack(plain.invariants(a), axis=1)
    el, ei = lam_errors(t, lam)[sel], inv_errors(t, inv)[sel]
    bl, bi = t.bound_lam()[sel], t.bound_inv()[sel]
    al = lam_errors(t, o1_lam)[sel]
    ai = inv_errors(t, o1_inv)[sel]
    # compensated: within 8x the bounds at every kappa (consistent diagonal
    # differences and error-free products); fma: the paper's class, G2 where
    # the paper's own algorithm exceeds the bounds
    if kappa <= 10.0 or acc == "compensated":
        check(el, np.broadcast_to(bl, el.shape), what=f"perturbation sweep eigvals kappa={kappa} {acc} (G1)")
    else:
        check_g2(el, bl, al, what=f"perturbation sweep eigvals kappa={kappa} {acc} (G2)", pool=True)
    if kappa == 1.0 or acc == "compensated":
        check(ei, bi, what=f"perturbation sweep invariants kappa={kappa} {acc} (G1)")
    else:
        check_g2(ei, bi, ai, what=f"perturbation sweep invariants kappa={kappa} {acc} (G2)")


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_stress_tensors_symmetric(eig3, c3, acc, layout):
    c, t = c3
    s = upload(c["s"], layout)
    lam = download_lam(eig3.eig3_eigvals(s, "symmetric", acc, "soa"))
    check(lam_errors(t, lam), t.bound_lam(), what=f"stress tensors eigvals {acc} {layout}")
    inv = download_inv(eig3.eig3_invariants(s, "symmetric", acc))
    check(inv_errors(t, inv), t.bound_inv(), what=f"stress tensors invariants {acc} {layout}")
    assert np.all(inv[:, 3] >= 0)


@pytest.mark.parametrize("acc", ACCS)
def test_differentiation_batch_forward(eig3, plain, c5, acc):
    c, t = c5
    lam = download_lam(eig3.eig3_eigvals(upload(c["a"], "aos"), "general", acc, "aos"))
    el = lam_errors(t, lam)
    bl = np.broadcast_to(t.bound_lam(), el.shape)
    well = (c["kappa"] <= 10) | (acc == "compensated")
    check(el[well], bl[well], what=f"differentiation batch eigvals kappa<=10 or compensated {acc} (G1)")
    if well.all():
        return
    al = lam_errors(t, plain.eigvals(c["a"]))
    check_g2(el[~well], bl[~well], al[~well], what=f"differentiation batch eigvals kappa>10 {acc} (G2)", pool=True)


@pytest.mark.parametrize("acc", ACCS)
def test_paper_paths(eig3, acc):
    """The paper's own sweeps: D1 and D2 paths with U_symm and U_1 (within the
    bound, as the paper reports) over delta = 10^-16 .. 10^-1."""
    deltas = 10.0 ** np.linspace(-16, -1, 61)
    for path in ("D1", "D2"):
        for basis in ("symm", "U1"):
            c = w.paper_path(path, basis, deltas)
            t = Truth(c["a"], c["kappa"])
            lam = download_lam(eig3.eig3_eigvals(upload(c["a"], "soa"), "general", acc, "soa"))
            check(lam_errors(t, lam), t.bound_lam(), what=f"{path}/{basis} eigvals {acc}")
            inv = download_inv(eig3.eig3_invariants(upload(c["a"], "soa"), "general", acc))
            check(inv_errors(t, inv), t.bound_inv(), what=f"{path}/{basis} invariants {acc}")


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 511, 769, 1000])
@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_ragged_sizes(eig3, n, layout):
    """Sizes around the 64-lane wave and the 256-lane workgroup (LDS tile)."""
    c = w.haar_general(n, seed=99)
    t = Truth(c["a"], c["kappa"])
    lam = download_lam(eig3.eig3_eigvals(upload(c["a"], layout), "general", "fma", "aos"))
    check(lam_errors(t, lam), t.bound_lam(), what=f"ragged n={n} {layout}")
    s = w.stress_tensors(n, seed=98)
    ts = Truth(w.symmetric_to_general(s["s"]), np.ones(n))
    lam = download_lam(eig3.eig3_eigvals(upload(s["s"], layout), "symmetric", "fma", "soa"))
    check(lam_errors(ts, lam), ts.bound_lam(), what=f"ragged symmetric n={n} {layout}")


def test_aos_unaligned_offset(eig3):
    """AoS input starting at an odd element offset of a larger buffer."""
    import torch
    c = w.haar_general(700, seed=97)
    t = Truth(c["a"], c["kappa"])
    big = torch.zeros(700 * 9 + 5, dtype=torch.float64, device="cuda:0")
    big[3:3 + 700 * 9] = torch.from_numpy(c["a"].ravel()).to("cuda:0")
    view = big[3:3 + 700 * 9]
    lam = download_lam(eig3.eig3_eigvals(view, "general", "fma", "aos"))
    check(lam_errors(t, lam), t.bound_lam(), what="aos offset 3")
