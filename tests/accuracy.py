"""Error measurement against the exact oracle, shared by the GPU parity tests.

Gates (forward errors against the exact definitions of oracle/exact.py, bound
b = the paper's lowest-order stability bound with C = 1, Frobenius norms; for
eigenvalues b = kappa_2(V) ||A|| eps with kappa_2(V) known from the generator):

  G1: |x - truth| <= 8 b                       (8x the stability bound)
  G2: |x - truth| <= 8 b + |x_paper - truth|   (no worse than the paper's own
      algorithm in plain binary64, oracle/eig3_plain.c, plus the 8x allowance)

G1 applies where the paper's algorithms themselves meet their bounds
(orthogonal and well-conditioned eigenbases, kappa <= 10, and symmetric
input).  For ill-conditioned eigenbases (kappa = 100) the paper reports
violations of the J3, Delta and eigenvalue bounds, and G2 applies instead.
"""
from __future__ import annotations

import numpy as np

from oracle import exact

EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24
KEYS = ("I1", "J2", "J3", "Delta")


class Truth:
    """Exact invariants, eigenvalues and bound scales of a batch (slow)."""

    def __init__(self, a: np.ndarray, kappa: np.ndarray):
        a = np.asarray(a, dtype=np.float64).reshape(-1, 9)
        self.a = a
        self.kappa = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (a.shape[0],)).copy()
        n = a.shape[0]
        self.inv = np.empty((n, 4))
        self.scale = np.empty((n, 5))
        self.lam = np.empty((n, 3), dtype=np.complex128)
        for m in range(n):
            ex = exact.invariants(a[m])
            self.inv[m] = [float(x) for x in ex]
            b = exact.bound_scales(a[m])
            self.scale[m] = [b[k] for k in KEYS] + [b["lam"]]
            self.lam[m] = exact.eigvals_float(a[m])

    def bound_inv(self, eps=EPS64):
        return self.scale[:, :4] * eps

    def bound_lam(self, eps=EPS64):
        return (self.scale[:, 4] * self.kappa * eps)[:, None]


def inv_errors(t: Truth, inv) -> np.ndarray:
    """|inv - truth| per (matrix, invariant); inv: 4 arrays or (n, 4)."""
    inv = np.asarray(inv, dtype=np.float64)
    if inv.shape[0] == 4 and inv.shape[1] != 4:
        inv = inv.T
    return np.abs(inv - t.inv)


def lam_errors(t: Truth, lam) -> np.ndarray:
    return np.abs(np.asarray(lam, dtype=np.float64).reshape(-1, 3) - t.lam)


def check(err: np.ndarray, bound: np.ndarray, allowance: np.ndarray | None = None, factor: float = 8.0,
          what: str = "") -> None:
    """Assert err <= factor * bound (+ allowance) elementwise, reporting the worst."""
    lim = factor * bound + (0.0 if allowance is None else allowance)
    bad = err > lim
    if bad.any():
        ratio = np.where(bound > 0, err / np.maximum(bound, 1e-300), np.inf)
        idx = np.unravel_index(np.argmax(np.where(bad, ratio, -1)), err.shape)
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {err.size} values exceed the gate; worst at {idx}: "
            f"err={err[idx]:.3e} bound={bound[idx]:.3e} allowance="
            f"{(0.0 if allowance is None else allowance[idx]):.3e}")


def ratio_summary(err: np.ndarray, bound: np.ndarray) -> dict:
    r = err / np.maximum(bound, 1e-300)
    return {"max": float(r.max()) if r.size else 0.0,
            "p9999": float(np.percentile(r, 99.99)) if r.size else 0.0}
