"""Accuracy report: forward errors of every variant, in units of the paper's
stability bound, next to the paper's own algorithm (plain binary64) on the
same matrices.  With EIG3_ACCURACY_REPORT=<path> the table is written there as
JSON (the committed copy is profiles/accuracy.json, read by bench.py as the
stated error of each workload)."""
import json
import os

import numpy as np
import pytest

import workloads as w
from accuracy import EPS32, Truth, inv_errors, lam_errors
from gpu_util import download_inv, download_lam, download_matrix, upload
from oracle import exact

pytestmark = pytest.mark.gpu


def _ratios(err, bound):
    r = err / np.maximum(np.broadcast_to(bound, err.shape), 1e-300)
    r = np.where(np.broadcast_to(bound, err.shape) > 0, r, np.where(err > 0, np.inf, 0.0))
    return {"max": float(np.max(r)), "p99": float(np.percentile(r, 99)), "median": float(np.median(r))}


def test_accuracy_report(plain_oracle):
    import paper_2511_00292_amd as eig3
    rep = {"units": "forward error / stability bound (C = 1, Frobenius, second-order term included)",
           "rows": []}

    def row(name, n, gpu, paper=None, extra=None):
        d = {"workload": name, "n": int(n), "gpu": gpu}
        if paper is not None:
            d["paper_algorithm_plain_f64"] = paper
        d.update(extra or {})
        rep["rows"].append(d)

    # Haar-similar batch and the perturbation sweep buckets (general binary64)
    c1 = w.haar_general(1500, seed=12)
    t1 = Truth(c1["a"], c1["kappa"])
    o1 = plain_oracle.eigvals(c1["a"])
    for acc in ("fma", "compensated"):
        lam = download_lam(eig3.eig3_eigvals(upload(c1["a"], "soa"), "general", acc, "soa"))
        row(f"Haar-similar batch general f64 eigvals ({acc})", 1500, _ratios(lam_errors(t1, lam), t1.bound_lam()),
            _ratios(lam_errors(t1, o1), t1.bound_lam()))
    c2 = w.perturbation_sweep(9 * 300, seed=13)
    t2 = Truth(c2["a"], c2["kappa"])
    o2l = plain_oracle.eigvals(c2["a"])
    o2i = np.stack(plain_oracle.invariants(c2["a"]), axis=1)
    for acc in ("fma", "compensated"):
        lam = download_lam(eig3.eig3_eigvals(upload(c2["a"], "soa"), "general", acc, "soa"))
        inv = download_inv(eig3.eig3_invariants(upload(c2["a"], "soa"), "general", acc))
        for kappa in (1.0, 10.0, 100.0):
            sel = c2["kappa"] == kappa
            bl, bi = t2.bound_lam()[sel], t2.bound_inv()[sel]
            gi = inv_errors(t2, inv)[sel]
            pi = inv_errors(t2, o2i)[sel]
            row(f"perturbation sweep kappa={kappa:g} general f64 ({acc})", int(sel.sum()),
                {"eigvals": _ratios(lam_errors(t2, lam)[sel], bl),
                 **{k: _ratios(gi[:, j], bi[:, j]) for j, k in enumerate(("I1", "J2", "J3", "Delta"))}},
                {"eigvals": _ratios(lam_errors(t2, o2l)[sel], bl),
                 **{k: _ratios(pi[:, j], bi[:, j]) for j, k in enumerate(("I1", "J2", "J3", "Delta"))}})
    # the perturbation sweep by bucket: variant x kappa x delta range, 4096
    # matrices per (variant, kappa), eigenvalues of both modes and of the
    # paper's algorithm against the exact roots (max, p99, p99.99)
    cb = w.perturbation_sweep(9 * 4096, seed=16)
    tb = Truth(cb["a"], cb["kappa"])
    ob = lam_errors(tb, plain_oracle.eigvals(cb["a"])) / tb.bound_lam()
    gb = {acc: lam_errors(tb, download_lam(eig3.eig3_eigvals(upload(cb["a"], "soa"), "general", acc, "soa")))
          / tb.bound_lam() for acc in ("fma", "compensated")}
    names = {0: "diag(1, 1+d, 1+2d)", 1: "diag(1, 1, 1+d)", 2: "I + d S"}
    edges = [1e-16, 1e-13, 1e-10, 1e-7, 1e-4, 1e-1]
    rep["buckets"] = []
    for v in range(3):
        for kappa in (1.0, 10.0, 100.0):
            for lo, hi in zip(edges[:-1], edges[1:]):
                sel = (cb["variant"] == v) & (cb["kappa"] == kappa) & (cb["delta"] >= lo) & (cb["delta"] < hi)
                if not sel.any():
                    continue
                st = {}
                for key, r in (("gpu_fma", gb["fma"]), ("gpu_compensated", gb["compensated"]),
                               ("paper_algorithm_plain_f64", ob)):
                    x = r[sel].ravel()
                    st[key] = {"max": float(x.max()), "p99": float(np.percentile(x, 99)),
                               "p9999": float(np.percentile(x, 99.99))}
                rep["buckets"].append({"variant": names[v], "kappa": kappa, "delta": [lo, hi],
                                       "n": int(sel.sum()), **st})
    # stress tensors (symmetric binary64) and binary32 stress tensors (binary32)
    c3 = w.stress_tensors(1500, seed=14)
    a3 = w.symmetric_to_general(c3["s"])
    t3 = Truth(a3, np.ones(1500))
    o3 = plain_oracle.eigvals(a3)
    for acc in ("fma", "compensated"):
        lam = download_lam(eig3.eig3_eigvals(upload(c3["s"], "soa"), "symmetric", acc, "soa"))
        row(f"stress tensors symmetric f64 eigvals ({acc})", 1500, _ratios(lam_errors(t3, lam), t3.bound_lam()),
            _ratios(lam_errors(t3, o3), t3.bound_lam()))
    s4 = c3["s"].astype(np.float32)
    a4 = w.symmetric_to_general(s4.astype(np.float64))
    t4 = Truth(a4, np.ones(1500))
    for acc in ("fma", "compensated"):
        lam = download_lam(eig3.eig3_eigvals(upload(s4, "soa"), "symmetric", acc, "soa"))
        row(f"binary32 stress tensors symmetric f32 eigvals ({acc})", 1500, _ratios(lam_errors(t4, lam), t4.bound_lam(EPS32)),
            extra={"bound_eps": "2^-24"})
    # differentiation batch forward and backward
    c5 = w.differentiation_batch(1500, seed=15, with_basis=True)
    t5 = Truth(c5["a"], c5["kappa"])
    o5 = plain_oracle.eigvals(c5["a"])
    idx = np.arange(0, 1500, 10)
    gref = np.array([exact.eigvals_vjp(c5["a"][m], c5["g"][m]) for m in idx])
    ob = plain_oracle.eigvals_backward(c5["a"][idx], c5["g"][idx])
    for acc in ("fma", "compensated"):
        lam = download_lam(eig3.eig3_eigvals(upload(c5["a"], "soa"), "general", acc, "soa"))
        grad = download_matrix(eig3.eig3_eigvals_backward(upload(c5["a"][idx], "aos"), upload(c5["g"][idx], "aos"),
                                                          "general", acc), 9)
        rel = np.abs(grad - gref).max(1) / np.abs(gref).max(1)
        relp = np.abs(ob - gref).max(1) / np.abs(gref).max(1)
        row(f"differentiation batch general f64 ({acc})", 1500, {"eigvals": _ratios(lam_errors(t5, lam), t5.bound_lam()),
                                                    "grad_rel_err_max": float(rel.max())},
            {"eigvals": _ratios(lam_errors(t5, o5), t5.bound_lam()), "grad_rel_err_max": float(relp.max())})
    path = os.environ.get("EIG3_ACCURACY_REPORT")
    if path:
        import bench
        rep["source_sha256"] = bench.source_digest()
        with open(path, "w") as f:
            json.dump(rep, f, indent=1)
    assert len(rep["rows"]) >= 14
