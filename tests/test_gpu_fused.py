"""GPU parity of the fused step (both RK stages of a self-periodic 8^3 block
in one workgroup, the block on chip; tiling code 5 of the 8^3 class) through
the C ABI, against the FP64 oracle: FP64 within 1e-12 relative per cell (the
oracle's operations in its order), mixed within 1e-5 relative in L1(rho) on
smooth flow; a uniform state stays fixed bitwise; mass, momentum and energy of
every block are conserved; the failure contract of the graph path holds; the
class refuses the fused step unless every block is 3D, 8^3 and periodic on
itself."""
import math

import numpy as np
import pytest

from gpu_util import l1_rho, rel_err, to_dev, to_host
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


def _fused_batch(mesh, P, prec):
    b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
    b.set_tiling(8, 5)
    assert {c["edge"]: c["tile"] for c in b.config()["classes"]}[8] == 5
    return b


@pytest.fixture(scope="module")
def uneven():
    P = I.uneven(nblocks=150, nsteps=20)
    R = P.U0.copy()
    _, t = O.run(P.mesh, R, P.nsteps, P.cfl, P.gamma)
    return P, R, t


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_fused_uneven_20_steps(uneven, prec):
    P, R, t_ref = uneven
    assert (P.mesh.n[:, 0] == 8).sum() > 20
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    b = _fused_batch(mesh, P, prec)
    t = b.run(P.nsteps, P.cfl, P.gamma)
    U = to_host(arena)
    if prec == H.FP64:
        assert rel_err(P.mesh, U, R) <= 1e-12
        assert abs(t - t_ref) <= 1e-12 * t_ref
    else:
        assert l1_rho(P.mesh, U, R) <= 1e-5
        assert abs(t - t_ref) <= 1e-6 * t_ref
    # each self-periodic block conserves its own totals
    for blk in np.nonzero(P.mesh.n[:, 0] == 8)[0][:40]:
        f0, f1 = P.mesh.block_view(P.U0, blk), P.mesh.block_view(U, blk)
        for v in range(5):
            scale = max(math.fsum(np.abs(f0[v]).ravel()), math.fsum(np.abs(f1[v]).ravel()), 1e-300)
            assert abs(math.fsum(f1[v].ravel()) - math.fsum(f0[v].ravel())) <= 1e-13 * P.nsteps * scale
    mesh.close()


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_fused_equals_two_launch_step(uneven, prec):
    """The fused step against the two stage launches of the same batch: FP64
    bitwise; mixed to the L1 bar (the mixed tile forms its z faces from a
    carried slope, the fused kernel from the four cells)."""
    P = uneven[0]
    outs = []
    for fused in (False, True):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        if fused:
            b.set_tiling(8, 5)
        b.run(5, P.cfl, P.gamma)
        outs.append(to_host(arena))
        mesh.close()
    if prec == H.FP64:
        assert np.array_equal(outs[0], outs[1])
    else:
        assert l1_rho(P.mesh, outs[1], outs[0]) <= 1e-6


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_fused_uniform_state_bitwise(prec):
    m = I.independent_blocks([8] * 12, 3)
    U0 = I.uniform_state(m, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, gamma=1.4)
    arena = to_dev(U0)
    mesh = H.Mesh(m, arena)
    b = H.Batch([H.Packet(mesh, range(m.nblocks), prec)])
    b.set_tiling(8, 5)
    b.run(4, 0.4, 1.4)
    assert np.array_equal(to_host(arena), U0)
    mesh.close()


def test_fused_failure_contract():
    """A non-physical cell in one fused block: the run reports ENONPHYS naming
    the block and leaves the whole arena untouched."""
    m = I.independent_blocks([8] * 6, 3)
    U0 = I.random_smooth_state(m, 5, 1.4)
    m.block_view(U0, 4)[4, 3, 2, 1] = 0.0
    for prec in (H.FP64, H.FP32_FP64):
        arena = to_dev(U0)
        mesh = H.Mesh(m, arena)
        b = H.Batch([H.Packet(mesh, range(m.nblocks), prec)])
        b.set_tiling(8, 5)
        with pytest.raises(H.HydroError) as e:
            b.run(3, 0.4, 1.4)
        assert e.value.code == H.ENONPHYS and "block 4" in str(e.value)
        assert np.array_equal(to_host(arena), U0)
        mesh.close()


def test_fused_refused_for_other_blocks():
    cases = [
        (I.block_grid((2, 2, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3), H.FP64),  # linked, not self
        (I.independent_blocks([8, 8], 2), H.FP64),  # 2D
        (I.independent_blocks([8, 8], 3), H.FP64 | H.EINFELDT),  # a method variant
    ]
    for m, prec in cases:
        U0 = I.uniform_state(m, gamma=1.4)
        arena = to_dev(U0)
        mesh = H.Mesh(m, arena)
        b = H.Batch([H.Packet(mesh, range(m.nblocks), prec)])
        with pytest.raises(H.HydroError) as e:
            b.set_tiling(8, 5)
        assert e.value.code == H.EINVAL
        mesh.close()


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_graph_replays_match_eager_steps(uneven, prec):
    """The captured step graph (stage launches plus the fused branch) replayed
    one step at a time, with eager work and synchronisations between the
    replays, equals the same steps launched eagerly (hydro_batch_time_kernels),
    bitwise after every step."""
    P = uneven[0]
    arena_g, arena_e = to_dev(P.U0), to_dev(P.U0)
    mesh_g, mesh_e = H.Mesh(P.mesh, arena_g), H.Mesh(P.mesh, arena_e)
    bg = _fused_batch(mesh_g, P, prec)
    be = _fused_batch(mesh_e, P, prec)
    for s in range(4):
        bg.run(1, P.cfl, P.gamma)  # one graph replay (the graph is captured once, on the first call)
        be.time_kernels(1, P.cfl, P.gamma)  # the same step, eager launches
        scratch = to_dev(np.arange(1000, dtype=np.float64)) * 2.0  # eager work of the program between replays
        assert float(scratch.sum()) == 999000.0
        assert np.array_equal(to_host(arena_g), to_host(arena_e)), s
    mesh_g.close()
    mesh_e.close()
