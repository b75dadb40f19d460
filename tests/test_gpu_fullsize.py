"""GPU parity at the benchmark configurations' full sizes.

The whole mesh runs on the GPU through the C ABI in the batched launch
configuration the benchmark times; the oracle recomputes what it can afford:
  * one step from the initial state on sampled blocks (their domain of
    dependence is their face neighbours), with the global dt computed by the
    oracle over the full mesh;
  * for the large Sedov-plus-noise run, 20 steps on the centred 512-block
    subset, the oracle running the 18^3-block region that contains the
    subset's domain of dependence (four cells per step).
Properties that hold at any size are checked on the full GPU result:
conservation of the totals on periodic meshes, in both precisions.
"""
import math

import numpy as np
import pytest

from gpu_util import l1_rho, rel_err
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _blocks_to_host(arena, mesh, ids):
    import torch

    torch.cuda.synchronize()
    U = np.zeros(mesh.arena_len)
    for i in ids:
        o, n = int(mesh.offset[i]), 5 * int(mesh.ncells[i])
        U[o:o + n] = arena[o:o + n].cpu().numpy()
    return U


def _one_step_sampled(P, ids, tune=False):
    import torch

    dt = O.dt(P.mesh, P.U0, P.gamma, P.cfl)
    ref = O.step_subset(P.mesh, P.U0, dt, P.gamma, ids)
    U0 = torch.from_numpy(P.U0).cuda()
    arena = U0.clone()
    mesh = H.Mesh(P.mesh, arena)
    out = {}
    for prec in (H.FP64, H.FP32_FP64):
        arena.copy_(U0)
        b = H.Batch([H.Packet(mesh, p, prec) for p in P.packets])
        if tune:
            b.autotune(P.gamma, reps=2)
        t = b.run(1, P.cfl, P.gamma)
        assert abs(t - dt) <= 1e-12 * dt
        U = _blocks_to_host(arena, P.mesh, ids)
        out[prec] = (rel_err(P.mesh, U, ref, ids), l1_rho(P.mesh, U, ref, ids))
        b.close()
    mesh.close()
    return out


def test_smooth_full_size_one_step_sampled():
    P = I.smooth3d()
    ids = sorted(set(np.random.default_rng(5).choice(P.mesh.nblocks, 8, replace=False).tolist()) | {0, 4095})
    out = _one_step_sampled(P, ids)
    assert out[H.FP64][0] <= 1e-12
    assert out[H.FP32_FP64][1] <= 1e-5


def test_uneven_full_size_one_step_sampled_autotuned():
    P = I.uneven()
    rng = np.random.default_rng(6)
    ids = []
    for e in (8, 16, 32):
        cls = np.nonzero(P.mesh.n[:, 0] == e)[0]
        ids += rng.choice(cls, 4, replace=False).tolist()
    out = _one_step_sampled(P, sorted(ids), tune=True)
    assert out[H.FP64][0] <= 1e-12
    assert out[H.FP32_FP64][1] <= 1e-5


def test_large_run_subset_after_20_steps_and_conservation():
    import torch

    P = I.sedov_noise()
    steps = 20
    # oracle: the region around the centred subset covering 20 steps of dependence
    nbx = P.mesh.grid[0]
    width, margin = 8, -(-4 * steps // 16)
    lo, hi = (nbx - width) // 2 - margin, (nbx - width) // 2 + width + margin
    region = np.asarray([(z * nbx + y) * nbx + x for z in range(lo, hi) for y in range(lo, hi)
                         for x in range(lo, hi)])
    m = P.mesh.subset(region)
    R = P.mesh.gather(P.U0, region)
    O.run(m, R, steps, P.cfl, P.gamma)
    pos = {int(b): k for k, b in enumerate(region)}
    inner = [pos[int(b)] for b in P.meta["subset"]]
    ms = m.subset(inner)
    Rin = m.gather(R, inner)

    U0 = torch.from_numpy(P.U0).cuda()
    arena = U0.clone()
    mesh = H.Mesh(P.mesh, arena)
    vol = float(np.prod(P.mesh.dx[0]))
    tot0 = [math.fsum(P.U0.reshape(P.mesh.nblocks, 5, -1)[:, v].ravel()) for v in range(5)]
    for prec in (H.FP64, H.FP32_FP64):
        arena.copy_(U0)
        b = H.Batch([H.Packet(mesh, p, prec) for p in P.packets])
        b.run(steps, P.cfl, P.gamma)
        torch.cuda.synchronize()
        G = np.concatenate([arena[int(P.mesh.offset[i]):int(P.mesh.offset[i]) + 5 * 4096].cpu().numpy()
                            for i in P.meta["subset"]])
        if prec == H.FP64:
            assert rel_err(ms, G, Rin) <= 1e-12
        else:
            assert l1_rho(ms, G, Rin) <= 1e-5
        # totals of the whole periodic mesh (sums on the GPU in FP64, then fsum of block sums)
        blocks = arena.view(P.mesh.nblocks, 5, -1)
        for v in range(5):
            s = math.fsum(blocks[:, v, :].sum(dim=1).cpu().numpy().tolist())
            scale = math.fsum(blocks[:, v, :].abs().sum(dim=1).cpu().numpy().tolist())
            assert abs(s - tot0[v]) * vol <= 1e-13 * steps * max(scale, 1.0) * vol, (prec, v, s, tot0[v])
        b.close()
    mesh.close()
