"""Error measurement against the two oracles, shared by the GPU parity tests.

O1 is the paper's algorithms in plain binary64 (oracle/eig3_plain.c), O2 the
exact definitions (oracle/exact.py: exact invariants of the stored matrix,
80-digit eigenvalues).  Bounds b are the paper's stability bounds with C = 1
and Frobenius norms; for eigenvalues b = kappa_2(V) ||A|| eps with
kappa_2(V) known from the generator:

  b_I1 = ||A|| eps
  b_J2 = ||S||^2 eps + ||S||^2 eps^2            (S = dev A)
  b_J3 = ||dev cof S|| ||S|| eps + ||S||^3 eps^2
  b_D  = ||dev(12 J2^2 A^T - 54 J3 cof S)|| ||S|| eps + ||S||^6 eps^2
  b_l  = kappa_2 ||A|| eps

The paper's bounds are first order, "+ O(eps^2)"; the second-order term is
taken as eps^2 ||S||^k with k the degree of the invariant.  It matters only
where the first-order term vanishes: at an exactly repeated eigenvalue the
Jacobian of Delta is zero, and an evaluation with roundings returns a Delta
of order eps^2 ||S||^6 where the exact value is 0.

Gates, each elementwise (every matrix, every output, no pooling):

  G1: |x - O1| <= 8 b
  G2: where G1 misses, |x - O2| <= 8 b + |O1 - O2|: no worse than the paper's
      own algorithm plus the allowance (the paper reports its J3, Delta and
      eigenvalue errors above the bounds for ill-conditioned eigenbases, and
      an evaluation with better rounding may then differ from O1 by more
      than 8 b)
  T8: |x - O2| <= 8 b: within 8x the bound of the exact result, whatever O1
      does.  The claim of the double_word and compensated evaluations at
      every kappa, and of fma for symmetric input and the eigenvalues at
      kappa <= 10.
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


def check_g12(x: np.ndarray, o1: np.ndarray, truth: np.ndarray, bound: np.ndarray, what: str = "",
              factor: float = 8.0) -> None:
    """Assert G1 or, where G1 misses, G2, for every element of x."""
    x, o1, truth = (np.asarray(v, dtype=np.float64) for v in (x, o1, truth))
    bound = np.broadcast_to(bound, x.shape)
    g1 = np.abs(x - o1) <= factor * bound
    g2 = np.abs(x - truth) <= factor * bound + np.abs(o1 - truth)
    bad = ~(g1 | g2)  # a NaN fails both
    if bad.any():
        excess = np.where(bad, (np.abs(x - truth) - np.abs(o1 - truth)) / np.maximum(bound, 1e-300), -np.inf)
        idx = np.unravel_index(np.argmax(excess), x.shape)
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {x.size} values fail G1 and G2; worst at {idx}: "
            f"|x-O2|={abs(x[idx] - truth[idx]):.3e} |O1-O2|={abs(o1[idx] - truth[idx]):.3e} "
            f"|x-O1|={abs(x[idx] - o1[idx]):.3e} bound={bound[idx]:.3e}")


def g12_failures(x, o1, truth, bound, factor: float = 8.0) -> np.ndarray:
    """Boolean mask of the elements that fail both G1 and G2."""
    x, o1, truth = (np.asarray(v, dtype=np.float64) for v in (x, o1, truth))
    bound = np.broadcast_to(bound, x.shape)
    return ~((np.abs(x - o1) <= factor * bound) | (np.abs(x - truth) <= factor * bound + np.abs(o1 - truth)))


def ratio_summary(err: np.ndarray, bound: np.ndarray) -> dict:
    r = np.asarray(err) / np.maximum(np.broadcast_to(bound, np.shape(err)), 1e-300)
    return {"max": float(r.max()) if r.size else 0.0,
            "p9999": float(np.percentile(r, 99.99)) if r.size else 0.0}
