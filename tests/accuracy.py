"""Error measurement against the exact oracle, shared by the GPU parity tests.

Gates (forward errors against the exact definitions of oracle/exact.py, bound
b = the paper's stability bound with C = 1 and Frobenius norms; for
eigenvalues b = kappa_2(V) ||A|| eps with kappa_2(V) known from the generator):

  b_I1 = ||A|| eps
  b_J2 = ||S||^2 eps + ||S||^2 eps^2            (S = dev A)
  b_J3 = ||dev cof S|| ||S|| eps + ||S||^3 eps^2
  b_D  = ||dev(12 J2^2 A^T - 54 J3 cof S)|| ||S|| eps + ||S||^6 eps^2
  b_l  = kappa_2 ||A|| eps

The paper's bounds are first order, "+ O(eps^2)"; the second-order term is
taken as eps^2 ||S||^k with k the degree of the invariant.  It matters only
where the first-order term vanishes: at an exactly repeated eigenvalue the
Jacobian of Delta is zero, and an FMA evaluation then returns a Delta of
order eps^2 ||S||^6 where the exact value is 0.

  G1: |x - truth| <= 8 b elementwise            (8x the stability bound)
  G2: max |x - truth|/b <= 8 + 2 max |x_paper - truth|/b over the bucket,
      per output: no worse than the paper's own algorithm in plain binary64
      (oracle/eig3_plain.c) in the worst case, up to a factor 2 for a
      different rounding order, plus the 8x allowance.

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
        ns = np.sqrt(self.scale[:, 1])  # ||dev A||
        second = np.stack([0.0 * ns, ns ** 2, ns ** 3, ns ** 6], axis=1) * eps * eps
        return self.scale[:, :4] * eps + second

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
    err = np.asarray(err)
    bound = np.broadcast_to(bound, err.shape)
    if allowance is not None:
        allowance = np.broadcast_to(allowance, err.shape)
    lim = factor * bound + (0.0 if allowance is None else allowance)
    bad = ~(err <= lim)  # a NaN error fails the gate
    if bad.any():
        ratio = np.where(bound > 0, err / np.maximum(bound, 1e-300), np.inf)
        idx = np.unravel_index(np.argmax(np.where(bad, ratio, -1)), err.shape)
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {err.size} values exceed the gate; worst at {idx}: "
            f"err={err[idx]:.3e} bound={bound[idx]:.3e} allowance="
            f"{(0.0 if allowance is None else allowance[idx]):.3e}")


def check_g2(err: np.ndarray, bound: np.ndarray, err_paper: np.ndarray, factor: float = 8.0,
             what: str = "", pool: bool = False) -> None:
    """G2: the worst ratio err / bound of x over a bucket is no worse than
    8 + 2x the worst ratio of the paper's algorithm over the same bucket.
    Per output column, or, with pool=True, over all columns together (the
    three eigenvalues of a bucket: at kappa(V) > 10 their worst ratios are
    heavy-tailed extremes whose position among the three carries no
    information)."""
    bound = np.broadcast_to(bound, err.shape)
    if err.size == 0:
        return
    tiny = np.maximum(bound, 1e-300)
    r = np.where(bound > 0, err / tiny, np.where(err > 0, np.inf, 0.0)).reshape(err.shape[0], -1)
    rp = np.where(bound > 0, err_paper / tiny, np.where(err_paper > 0, np.inf, 0.0)).reshape(err.shape[0], -1)
    if pool:
        r, rp = r.reshape(-1, 1), rp.reshape(-1, 1)
    lim = factor + 2.0 * rp.max(axis=0)
    worst = r.max(axis=0)
    if not np.all(worst <= lim):  # a NaN error fails the gate
        raise AssertionError(f"{what}: worst ratio {np.round(worst, 2)} exceeds 8 + 2 x paper's "
                             f"worst {np.round(rp.max(axis=0), 2)}")


def ratio_summary(err: np.ndarray, bound: np.ndarray) -> dict:
    r = err / np.maximum(bound, 1e-300)
    return {"max": float(r.max()) if r.size else 0.0,
            "p9999": float(np.percentile(r, 99.99)) if r.size else 0.0}
