"""Host <-> device helpers for the GPU tests (layout conversion only)."""
from __future__ import annotations

import numpy as np

import workloads as w

DEV = "cuda:0"


def upload(a: np.ndarray, layout: str, structure: str = "general", dtype=None):
    """(n,9) or (n,6) host array -> device batch in the given layout."""
    import torch

    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a).to(DEV)
    if dtype is not None:
        t = t.to(dtype)
    if layout == "aos":
        return t.contiguous()
    return [t[:, k].contiguous() for k in range(a.shape[1])]


def download_lam(res) -> np.ndarray:
    if isinstance(res, (list, tuple)):
        return np.stack([r.double().cpu().numpy() for r in res], axis=1)
    return res.double().cpu().numpy().reshape(-1, 3)


def download_inv(res) -> np.ndarray:
    return np.stack([r.double().cpu().numpy() for r in res], axis=1)


def download_matrix(res, k: int) -> np.ndarray:
    if isinstance(res, (list, tuple)):
        return np.stack([r.double().cpu().numpy() for r in res], axis=1)
    return res.double().cpu().numpy().reshape(-1, k)


def sym_to_gen(s):
    return w.symmetric_to_general(s)
