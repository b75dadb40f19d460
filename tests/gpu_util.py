"""Helpers of the GPU parity tests: error metrics and device round trips."""
from __future__ import annotations

import numpy as np


def rel_err(mesh, U, R, blocks=None) -> float:
    """max over cells c and variables v of |U - R| / max(|R(c,v)|, 1e-6 max_c |R(., v)|)."""
    ids = range(mesh.nblocks) if blocks is None else blocks
    worst = 0.0
    for v in range(5):
        ref = [mesh.block_view(R, b)[v] for b in ids]
        got = [mesh.block_view(U, b)[v] for b in ids]
        scale = max(float(np.abs(r).max()) for r in ref)
        if scale == 0.0:
            worst = max(worst, max(float(np.abs(g).max()) for g in got))
            continue
        for g, r in zip(got, ref):
            worst = max(worst, float((np.abs(g - r) / np.maximum(np.abs(r), 1e-6 * scale)).max()))
    return worst


def l1_rho(mesh, U, R, blocks=None) -> float:
    """sum_c |rho - rho_ref| V_c / sum_c |rho_ref| V_c."""
    ids = range(mesh.nblocks) if blocks is None else blocks
    num = den = 0.0
    for b in ids:
        vol = float(np.prod(mesh.dx[b]))
        r = mesh.block_view(R, b)[0]
        num += float(np.abs(mesh.block_view(U, b)[0] - r).sum()) * vol
        den += float(np.abs(r).sum()) * vol
    return num / den


def to_dev(U):
    import torch

    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()
