"""GPU parity over the full duration of the smooth and uneven benchmark
configurations, at full size, every cell compared.

* Smooth random flow: 4096 blocks of 16^3 (256^3 cells, periodic), 64 packets
  of 64, 100 steps, batched graph path.
* Uneven batch: 6000 self-periodic blocks of 8^3/16^3/32^3 in packets of 1 to
  256 blocks, 20 steps, batched graph path after the autotuner has picked the
  tilings.

Bars: the FP64 path within 1e-12 relative per cell (floored as in the other
parity tests) and its simulated time within 1e-12; the mixed path within
1e-5 relative in L1(rho).  The mixed path's time step comes from its own FP64
rate of its own (FP32-fluxed) state, so its time differs from the oracle's by
the state's error at the fastest cell, not by rounding: after n steps
|t_mixed - t_ref| / t_ref is at most the largest relative error of any
step's dt, which is bounded by the relative error of the rate (|u| + c)/dx at
the fastest cell.  On this smooth flow the state errors are O(1e-8) (FP32
fluxes, unit roundoff 6e-8, accumulated over the steps), so the bound
stated and tested here, 1e-6, has a margin of about two orders.

The oracle runs the whole mesh on the host cores (about a minute for the
smooth case on 16 cores).
"""
import numpy as np
import pytest

from gpu_util import l1_rho, rel_err
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL_L1_MIXED = 1e-5
TOL_T_MIXED = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _oracle(P):
    R = P.U0.copy()
    dts, t = O.run(P.mesh, R, P.nsteps, P.cfl, P.gamma)
    return R, dts, t


def _gpu_run(P, prec, tune=False, fused=False):
    import torch

    arena = torch.from_numpy(P.U0).cuda()
    mesh = H.Mesh(P.mesh, arena)
    pks = [H.Packet(mesh, p, prec) for p in P.packets]
    b = H.Batch(pks)
    if tune:
        b.autotune(P.gamma, reps=2)
    if fused:
        b.set_tiling(8, 5)
    t = b.run(P.nsteps, P.cfl, P.gamma)
    torch.cuda.synchronize()
    U = arena.cpu().numpy()
    b.close()
    mesh.close()
    return U, t


def _check(P, R, t_ref, tune=False, fused=False):
    U, t = _gpu_run(P, H.FP64, tune, fused)
    e64 = rel_err(P.mesh, U, R)
    U, tm = _gpu_run(P, H.FP32_FP64, tune, fused)
    l1 = l1_rho(P.mesh, U, R)
    et = abs(tm - t_ref) / t_ref
    print(f"{P.name}: fp64 max rel err {e64:.3e}, t err {abs(t - t_ref) / t_ref:.3e}; "
          f"mixed L1(rho) {l1:.3e}, t err {et:.3e}", flush=True)
    assert e64 <= TOL64
    assert abs(t - t_ref) <= TOL64 * t_ref
    assert l1 <= TOL_L1_MIXED
    assert et <= TOL_T_MIXED


def test_smooth_full_size_100_steps():
    P = I.smooth3d()
    assert P.mesh.nblocks == 4096 and P.nsteps == 100
    R, _, t_ref = _oracle(P)
    _check(P, R, t_ref)


@pytest.fixture(scope="module")
def uneven_ref():
    P = I.uneven()
    assert P.mesh.nblocks == 6000 and P.nsteps == 20
    R, _, t_ref = _oracle(P)
    return P, R, t_ref


def test_uneven_full_size_20_steps_autotuned(uneven_ref):
    P, R, t_ref = uneven_ref
    _check(P, R, t_ref, tune=True)


def test_uneven_full_size_20_steps_fused(uneven_ref):
    """The same with the 8^3 class on the fused step (tiling code 5)."""
    P, R, t_ref = uneven_ref
    _check(P, R, t_ref, fused=True)


def test_packet_dt_mixed_and_fp64_against_oracle():
    """hydro_packet_reduce_dt of a packet holding the whole smooth mesh (a
    reduced 4^3-block copy): FP64 equals the oracle's dt to 1e-12; the mixed
    packet's rate (refined hardware reciprocal square root) to 1e-14 on the
    same state, and to the mixed time bound after 30 mixed steps taken with
    its own dt."""
    import torch

    P = I.smooth3d(nblk=(4, 4, 4), nsteps=30)
    R = P.U0.copy()
    dts, _ = O.run(P.mesh, R, P.nsteps, P.cfl, P.gamma)
    dt_end = O.dt(P.mesh, R, P.gamma, P.cfl)
    for prec in (H.FP64, H.FP32_FP64):
        arena = torch.from_numpy(P.U0).cuda()
        mesh = H.Mesh(P.mesh, arena)
        pk = H.Packet(mesh, range(P.mesh.nblocks), prec)
        dt0 = pk.reduce_dt(P.gamma, P.cfl)
        tol0 = TOL64 if prec == H.FP64 else 1e-14
        assert abs(dt0 - dts[0]) <= tol0 * dts[0], (prec, dt0, dts[0])
        for s in range(P.nsteps):
            dt = pk.reduce_dt(P.gamma, P.cfl)
            pk.advance(dt, P.gamma)
        dt = pk.reduce_dt(P.gamma, P.cfl)
        tol = TOL64 if prec == H.FP64 else TOL_T_MIXED
        assert abs(dt - dt_end) <= tol * dt_end, (prec, dt, dt_end)
        pk.close()
        mesh.close()
