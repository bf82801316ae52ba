"""Seeded synthetic batches of real, diagonalizable 3x3 matrices.

This module only *builds inputs*: it contains none of the eigenvalue
method's arithmetic (no invariants, no discriminant, no trigonometric
formula).  Both the HIP path's tests/bench and the oracle's tests draw their
matrices from here.

Construction follows the paper's test-matrix recipe fl(A) = fl(U D U^-1)
(Sec. "Benchmarks", Eq. test-matrix): a prescribed spectrum D and a
nonsingular eigenbasis U, multiplied out in binary64.  The eigenbasis with a
chosen 2-norm condition number kappa is V = Q1 diag(1, kappa^-1/2, kappa^-1) Q2^T
with Q1, Q2 Haar-random orthogonal (Gram-Schmidt QR of a N(0,1) matrix with
a positive R diagonal), and its inverse is Q2 diag(1, kappa^1/2, kappa) Q1^T.
A = (V D) V^-1.

Every batch is generated in chunks of ``CHUNK`` matrices; chunk c draws from
``numpy.random.default_rng([seed, c])``, so matrix i is the same whatever the
batch size, and a sampled index can be regenerated alone.  All arrays are
row-major (n, 9) float64 (entries A00, A01, A02, A10, ..., A22) unless
stated otherwise; symmetric batches are (n, 6) with entries
A00, A11, A22, A01, A02, A12.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 18

GENERAL_ENTRIES = ("A00", "A01", "A02", "A10", "A11", "A12", "A20", "A21", "A22")
SYMMETRIC_ENTRIES = ("A00", "A11", "A22", "A01", "A02", "A12")
# positions of the symmetric entries inside the 9 row-major entries
SYMMETRIC_POS = (0, 4, 8, 1, 2, 5)

SEEDS = {"haar_general": 2511001, "perturbation_sweep": 2511002, "stress_tensors": 2511003,
         "stress_tensors_f32": 2511003, "differentiation_batch": 2511005}


# ----------------------------------------------------------------------------
# elementwise (struct-of-arrays) 3x3 helpers: a matrix is a list of 9 arrays
# ----------------------------------------------------------------------------

def _mm(x, y):
    return [x[3 * i] * y[j] + x[3 * i + 1] * y[3 + j] + x[3 * i + 2] * y[6 + j]
            for i in range(3) for j in range(3)]


def _t(x):
    return [x[0], x[3], x[6], x[1], x[4], x[7], x[2], x[5], x[8]]


def _haar(rng, n):
    """Q factor (positive R diagonal) of an N(0,1) 3x3 matrix: Haar measure.
    Classical Gram-Schmidt on the columns, applied twice for orthogonality."""
    g = rng.standard_normal((9, n))
    cols = [[g[0 + c], g[3 + c], g[6 + c]] for c in range(3)]
    q = []
    for c in range(3):
        v = cols[c]
        for _ in range(2):
            for u in q:
                p = v[0] * u[0] + v[1] * u[1] + v[2] * u[2]
                v = [v[k] - p * u[k] for k in range(3)]
        nv = np.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
        q.append([v[k] / nv for k in range(3)])
    # q[c] is column c
    return [q[j][i] for i in range(3) for j in range(3)]


def _basis(rng, n, kappa):
    """V with 2-norm condition number kappa (array or scalar) and its inverse."""
    kappa = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n,))
    q1 = _haar(rng, n)
    q2 = _haar(rng, n)
    s = [np.ones(n), kappa ** -0.5, 1.0 / kappa]
    si = [np.ones(n), np.sqrt(kappa), kappa]
    q2t = _t(q2)
    q1t = _t(q1)
    v = _mm([q1[3 * i + j] * s[j] for i in range(3) for j in range(3)], q2t)
    vinv = _mm([q2[3 * i + j] * si[j] for i in range(3) for j in range(3)], q1t)
    return v, vinv


def _similar(v, vinv, d):
    """fl((V D) V^-1) for a general (9-list) D."""
    return _mm(_mm(v, d), vinv)


def _diag(l0, l1, l2):
    z = np.zeros_like(l0)
    return [l0, z, z, z, l1, z, z, z, l2]


def _stack(m):
    return np.ascontiguousarray(np.stack(m, axis=1))


def _chunks(n, fn, seed, nthreads=None):
    """Run fn(rng, start, count) per chunk (in threads) and concatenate dicts."""
    nch = (n + CHUNK - 1) // CHUNK
    nthreads = nthreads or min(16, os.cpu_count() or 1, max(nch, 1))

    def one(c):
        rng = np.random.default_rng([seed, c])
        start = c * CHUNK
        out = fn(rng, start, CHUNK)
        cnt = min(CHUNK, n - start)
        return {k: v[:cnt] for k, v in out.items()}

    if nch == 0:
        parts = [{k: v[:0] for k, v in fn(np.random.default_rng([seed, 0]), 0, 1).items()}]
    elif nthreads > 1 and nch > 1:
        with ThreadPoolExecutor(nthreads) as ex:
            parts = list(ex.map(one, range(nch)))
    else:
        parts = [one(c) for c in range(nch)]
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def haar_general(n=100_000, seed=SEEDS["haar_general"]):
    """General matrices A = V diag(l) V^-1, V Haar orthogonal, l iid U[-1, 1].
    Returns a (n,9), lam (n,3) prescribed spectrum sorted, kappa (n,)."""
    def fn(rng, start, cnt):
        lam = np.sort(rng.uniform(-1.0, 1.0, (cnt, 3)), axis=1)
        v, vi = _basis(rng, cnt, 1.0)
        a = _similar(v, vi, _diag(lam[:, 0], lam[:, 1], lam[:, 2]))
        return {"a": _stack(a), "lam": lam, "kappa": np.ones(cnt)}
    return _chunks(n, fn, seed)


SWEEP_KAPPAS = (1.0, 10.0, 100.0)
SWEEP_SPECTRA = ("triple-spread", "double", "near-triple")


def perturbation_sweep(n=1 << 24, seed=SEEDS["perturbation_sweep"]):
    """Perturbation sweep.  Matrix i has variant i mod 3:
    0: D = diag(1, 1+d, 1+2d); 1: D = diag(1, 1, 1+d); 2: D = I + d S with S a
    symmetric matrix of 6 iid N(0,1) entries; and kappa = (1, 10, 100)[(i // 3) mod 3];
    d = 10^U(-16, -1).  Returns a, kappa, variant, delta, and lam (the
    prescribed spectrum, NaN for variant 2)."""
    def fn(rng, start, cnt):
        idx = np.arange(start, start + cnt)
        variant = idx % 3
        kappa = np.asarray(SWEEP_KAPPAS)[(idx // 3) % 3]
        delta = 10.0 ** rng.uniform(-16.0, -1.0, cnt)
        s6 = rng.standard_normal((6, cnt))
        v, vi = _basis(rng, cnt, kappa)
        one = np.ones(cnt)
        z = np.zeros(cnt)
        l1 = np.where(variant == 0, 1.0 + delta, 1.0)
        l2 = np.where(variant == 0, 1.0 + 2.0 * delta, 1.0 + delta)
        isn = variant == 2
        sd = delta * isn
        d = [np.where(isn, 1.0 + sd * s6[0], one), sd * s6[3], sd * s6[4],
             sd * s6[3], np.where(isn, 1.0 + sd * s6[1], l1), sd * s6[5],
             sd * s6[4], sd * s6[5], np.where(isn, 1.0 + sd * s6[2], l2)]
        a = _similar(v, vi, d)
        lam = np.stack([one, l1, l2], axis=1)
        lam[isn] = np.nan
        return {"a": _stack(a), "kappa": kappa, "variant": variant, "delta": delta, "lam": lam}
    return _chunks(n, fn, seed)


def stress_tensors(n=1 << 27, seed=SEEDS["stress_tensors"]):
    """Symmetric stress-like tensors, (n, 6) in SYMMETRIC_ENTRIES order.
    Half of each chunk has 6 iid N(0,1)*100 entries; the other half is
    p I + d S with p ~ N(0, 100^2), S symmetric with 6 iid N(0,1) entries,
    d = 10^U(-14, -2).  The halves are interleaved by a seeded permutation of
    an exact 50/50 mask.  Returns s (n,6) float64 and iso (n,) bool."""
    def fn(rng, start, cnt):
        mask = np.zeros(cnt, dtype=bool)
        mask[: cnt // 2] = True
        rng.shuffle(mask)
        gen = rng.standard_normal((6, cnt)) * 100.0
        p = rng.standard_normal(cnt) * 100.0
        sn = rng.standard_normal((6, cnt))
        delta = 10.0 ** rng.uniform(-14.0, -2.0, cnt)
        iso = [p + delta * sn[0], p + delta * sn[1], p + delta * sn[2],
               delta * sn[3], delta * sn[4], delta * sn[5]]
        s = np.stack([np.where(mask, iso[k], gen[k]) for k in range(6)], axis=1)
        return {"s": np.ascontiguousarray(s), "iso": mask}
    return _chunks(n, fn, seed)


def stress_tensors_f32(n=1 << 27, seed=SEEDS["stress_tensors_f32"]):
    """stress tensors rounded to binary32 (same matrices, same seed)."""
    out = stress_tensors(n, seed)
    out["s"] = out["s"].astype(np.float32)
    return out


def differentiation_batch(n=1 << 24, seed=SEEDS["differentiation_batch"], with_basis=False):
    """Differentiation batch: sorted l ~ U[-1, 1] with min gap >= 1e-3
    (rejection sampling), kappa = 10^U(0, 2), upstream gradient g ~ N(0,1)
    (n, 3).  Returns a, g, lam, kappa and, if with_basis, v and vinv (n, 9)."""
    def fn(rng, start, cnt):
        lam = np.sort(rng.uniform(-1.0, 1.0, (cnt, 3)), axis=1)
        bad = np.minimum(lam[:, 1] - lam[:, 0], lam[:, 2] - lam[:, 1]) < 1e-3
        while bad.any():
            lam[bad] = np.sort(rng.uniform(-1.0, 1.0, (int(bad.sum()), 3)), axis=1)
            bad = np.minimum(lam[:, 1] - lam[:, 0], lam[:, 2] - lam[:, 1]) < 1e-3
        kappa = 10.0 ** rng.uniform(0.0, 2.0, cnt)
        v, vi = _basis(rng, cnt, kappa)
        g = rng.standard_normal((cnt, 3))
        a = _similar(v, vi, _diag(lam[:, 0], lam[:, 1], lam[:, 2]))
        out = {"a": _stack(a), "g": g, "lam": lam, "kappa": kappa}
        if with_basis:
            out["v"] = _stack(v)
            out["vinv"] = _stack(vi)
        return out
    return _chunks(n, fn, seed)


# ----------------------------------------------------------------------------
# the paper's own benchmark paths (Sec. "Benchmarks")
# ----------------------------------------------------------------------------

def paper_basis(name: str, gamma: float = 1e-3):
    """U_symm (orthogonal), U_1 (kappa_2 = 2), U_2(gamma) (ill-conditioned) of
    Eq. transformation-matrices, as 3x3 float64 arrays."""
    r2 = np.sqrt(2.0)
    if name == "symm":
        return np.array([[1 / r2, -0.5, 0.5], [1 / r2, 0.5, -0.5], [0.0, 1 / r2, 1 / r2]])
    if name == "U1":
        return np.array([[1.0, -1.0, 1.0], [1.0, 1.0, 1.0], [-1.0, -1.0, 1.0]])
    if name == "U2":
        return np.array([[1.0, 1.0, 1.0], [1.0, 0.0, 1.0], [2.0, 1.0, 2.0 + gamma]])
    raise ValueError(name)


def paper_path(path: str, basis: str, deltas, gamma: float = 1e-3):
    """fl(U D U^-1) along D1 = diag(1, 1, 1+d) or D2 = diag(-1, 1, 1+d)
    (Sec. "Benchmarks"), with numpy.linalg.inv and matmul as the paper does.
    For U_symm the inverse is the transpose.  Returns a (n,9), lam (n,3)."""
    u = paper_basis(basis, gamma)
    ui = u.T.copy() if basis == "symm" else np.linalg.inv(u)
    deltas = np.asarray(deltas, dtype=np.float64)
    first = 1.0 if path == "D1" else -1.0
    if path not in ("D1", "D2"):
        raise ValueError(path)
    a = np.empty((deltas.size, 9))
    lam = np.empty((deltas.size, 3))
    for i, d in enumerate(deltas):
        dm = np.diag([first, 1.0, 1.0 + d])
        a[i] = (u @ dm @ ui).ravel()
        lam[i] = np.sort([first, 1.0, 1.0 + d])
    return {"a": a, "lam": lam, "kappa": np.full(deltas.size, np.linalg.cond(u))}


# ----------------------------------------------------------------------------
# layout helpers
# ----------------------------------------------------------------------------

def symmetric_to_general(s):
    """(n,6) symmetric entries -> (n,9) row-major full matrices."""
    s = np.asarray(s)
    a00, a11, a22, a01, a02, a12 = (s[:, k] for k in range(6))
    return np.ascontiguousarray(np.stack([a00, a01, a02, a01, a11, a12, a02, a12, a22], axis=1))


def to_soa(a):
    """(n,k) -> (k,n) contiguous (one array per entry)."""
    return np.ascontiguousarray(np.asarray(a).T)
