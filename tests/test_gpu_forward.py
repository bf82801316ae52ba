"""GPU parity of the forward path (eig3_invariants, eig3_eigvals) against the
two oracles, through the C ABI.  Gates G1, G2 and T8 are defined in
tests/accuracy.py; every gate is elementwise.

Claims checked here: double_word and compensated within 8x the bounds of the
exact result (T8) and G1/G2 on every output at every kappa; fma T8 on the
eigenvalues and G1/G2 on every output for kappa <= 10 and symmetric input.
fma is not claimed at kappa = 100 (perturbation sweep) and kappa > 10
(differentiation batch), where it fails G1 and G2 on some elements (the
accuracy report lists how many)."""
import numpy as np
import pytest

import workloads as w
from accuracy import Truth, check, check_g12, inv_errors, lam_errors
from gpu_util import download_inv, download_lam, upload

pytestmark = pytest.mark.gpu

ACCS = ["fma", "compensated", "double_word"]
EXACT = ("compensated", "double_word")  # claimed within 8x at every kappa


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
    lam = download_lam(eig3.eig3_eigvals(upload(a, "soa"), "general", acc, "soa"))[sel]
    inv = download_inv(eig3.eig3_invariants(upload(a, "soa"), "general", acc))[sel]
    o1_lam = plain.eigvals(a)[sel]
    o1_inv = np.stack(plain.invariants(a), axis=1)[sel]
    bl, bi = t.bound_lam()[sel], t.bound_inv()[sel]
    if acc == "fma" and kappa > 10.0:
        # not claimed: only what holds for any evaluation
        assert np.all(np.isfinite(lam)) and np.all(np.diff(lam, axis=1) >= 0)
        return
    what = f"perturbation sweep kappa={kappa} {acc}"
    check_g12(lam, o1_lam, t.lam.real[sel], bl, what=f"{what} eigvals (G1/G2)")
    check_g12(inv, o1_inv, t.inv[sel], bi, what=f"{what} invariants (G1/G2)")
    check(np.abs(lam - t.lam.real[sel]), bl, what=f"{what} eigvals (T8)")
    if acc in EXACT or kappa == 1.0:
        check(np.abs(inv - t.inv[sel]), bi, what=f"{what} invariants (T8)")


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
    bl = t.bound_lam()
    # fma is claimed for kappa <= 10 only
    well = np.ones(c["a"].shape[0], bool) if acc in EXACT else c["kappa"] <= 10
    check_g12(lam[well], plain.eigvals(c["a"])[well], t.lam.real[well], bl[well],
              what=f"differentiation batch eigvals {acc} (G1/G2)")
    check(lam_errors(t, lam)[well], bl[well], what=f"differentiation batch eigvals {acc} (T8)")


@pytest.mark.parametrize("acc", ACCS)
def test_haar_general_full_size_g1(eig3, plain, acc):
    """The Haar-similar batch at its full 100,000 matrices: G1 against the
    plain binary64 oracle on every eigenvalue; where G1 misses, G2 against the
    exact eigenvalues of those matrices."""
    c = w.haar_general()
    assert c["a"].shape[0] == 100_000
    lam = download_lam(eig3.eig3_eigvals(upload(c["a"], "soa"), "general", acc, "soa"))
    o1 = plain.eigvals(c["a"])
    na = np.sqrt((c["a"] ** 2).sum(axis=1))
    bound = (na * 2.0 ** -53)[:, None]  # kappa = 1
    miss = np.abs(lam - o1) > 8 * bound
    rows = np.nonzero(miss.any(axis=1))[0]
    assert rows.size < 100, f"{rows.size} matrices miss G1"
    if rows.size:
        t = Truth(c["a"][rows], c["kappa"][rows])
        check_g12(lam[rows], o1[rows], t.lam.real, t.bound_lam(), what=f"Haar-similar batch {acc} G1 misses (G2)")


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
    lam = download_lam(eig3.eig3_eigvals(upload(c["a"], layout), "general", "double_word", "aos"))
    check(lam_errors(t, lam), t.bound_lam(), what=f"ragged n={n} {layout}")
    s = w.stress_tensors(n, seed=98)
    ts = Truth(w.symmetric_to_general(s["s"]), np.ones(n))
    lam = download_lam(eig3.eig3_eigvals(upload(s["s"], layout), "symmetric", "double_word", "soa"))
    check(lam_errors(ts, lam), ts.bound_lam(), what=f"ragged symmetric n={n} {layout}")


def test_aos_unaligned_offset(eig3):
    """AoS input starting at an odd element offset of a larger buffer."""
    import torch
    c = w.haar_general(700, seed=97)
    t = Truth(c["a"], c["kappa"])
    big = torch.zeros(700 * 9 + 5, dtype=torch.float64, device="cuda:0")
    big[3:3 + 700 * 9] = torch.from_numpy(c["a"].ravel()).to("cuda:0")
    view = big[3:3 + 700 * 9]
    lam = download_lam(eig3.eig3_eigvals(view, "general", "double_word", "aos"))
    check(lam_errors(t, lam), t.bound_lam(), what="aos offset 3")


def test_staggered_one_buffer_placement(eig3):
    """Arrays placed in one buffer at eig3.soa_stride (the library's default
    for its own outputs) give bitwise the results of separate allocations,
    forward and adjoint, with ragged n."""
    import torch
    n = 70_001
    c = w.differentiation_batch(n)
    a, g = np.ascontiguousarray(c["a"]), np.ascontiguousarray(c["g"])
    sep_a, sep_g = upload(a, "soa"), upload(g, "soa")
    one = eig3.empty_soa(n, 12, torch.float64, device=sep_a[0].device)
    for k in range(9):
        one[k].copy_(sep_a[k])
    for k in range(3):
        one[9 + k].copy_(sep_g[k])
    for acc in ("double_word", "fma"):
        lam_sep = download_lam(eig3.eig3_eigvals(sep_a, "general", acc, "soa"))
        lam_one = download_lam(eig3.eig3_eigvals(one[:9], "general", acc, "soa"))
        assert np.array_equal(lam_sep, lam_one)
        g_sep = download_inv(eig3.eig3_eigvals_backward(sep_a, sep_g, "general", acc))
        g_one = download_inv(eig3.eig3_eigvals_backward(one[:9], one[9:], "general", acc))
        assert np.array_equal(g_sep, g_one)
