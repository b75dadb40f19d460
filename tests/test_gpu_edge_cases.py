"""GPU parity on mesh shapes the benchmark configurations do not exercise.

Each case runs the HIP path through the C ABI and the FP64 oracle on the same
seeded state: FP64 <= 1e-12 relative per cell (floored, as in the other parity
tests), mixed FP32/FP64 L1(rho) <= 1e-5.
  * linked blocks of different extents along the link axis (the guard source
    has another row length than the block itself);
  * ragged blocks that only the 8x8 tiling covers (x/y extents multiples of 8
    but not of 16, an odd three-plane z extent), with outflow faces and
    partly filled four-tile work items;
  * blocks two planes thin along z, linked to each other, so the two guard
    layers are the whole neighbour;
  * a 2D mesh of non-square blocks;
  * a one-block self-periodic packet through the packet path and the graph
    path;
  * supersonic flow, every x face on the upwind branch of HLLC;
  * a block at the maximum x extent;
  * zero steps (graph and host-resident paths): t = 0, the state untouched.
"""
import numpy as np
import pytest

from gpu_util import l1_rho, rel_err, to_dev, to_host
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu

GAMMA = 1.4
CFL = 0.4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def chain_mesh(ns, axis, dx, ndim=3):
    """Blocks of extents `ns` linked in a periodic chain along `axis`; every
    other face is periodic onto the block itself (outflow on the unused z
    faces in 2D)."""
    nb = len(ns)
    n = np.asarray(ns, dtype=np.int32)
    kind = np.full((nb, 6), I.PERIODIC_SELF, dtype=np.int32)
    if ndim == 2:
        kind[:, 4:] = I.OUTFLOW
    nbr = np.full((nb, 6), -1, dtype=np.int32)
    origin = np.zeros((nb, 3))
    for b in range(nb):
        kind[b, 2 * axis] = kind[b, 2 * axis + 1] = I.NBR
        nbr[b, 2 * axis] = (b - 1) % nb
        nbr[b, 2 * axis + 1] = (b + 1) % nb
        if b:
            origin[b, axis] = origin[b - 1, axis] + n[b - 1, axis] * dx
    dxs = np.full((nb, 3), dx)
    if ndim == 2:
        dxs[:, 2] = 1.0
    sizes = 5 * n.prod(axis=1).astype(np.int64)
    offset = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return I.BlockMesh(ndim, n, dxs, kind, nbr, offset, origin)


def smooth_state(mesh, seed=7):
    prims = I.grid_field(mesh, lambda x, y, z: I.smooth_fields(np.random.default_rng(seed), x, y, z))
    if mesh.ndim == 2:
        for w in prims:
            w[3] = 0.0
    return I.conserved_arena(mesh, prims, GAMMA)


def check_both(mesh, U0, nsteps, packets=None):
    R = U0.copy()
    _, t_ref = O.run(mesh, R, nsteps, CFL, GAMMA)
    packets = packets or [list(range(mesh.nblocks))]
    for prec in (H.FP64, H.FP32_FP64):
        arena = to_dev(U0)
        m = H.Mesh(mesh, arena)
        b = H.Batch([H.Packet(m, p, prec) for p in packets])
        t = b.run(nsteps, CFL, GAMMA)
        U = to_host(arena)
        if prec == H.FP64:
            assert abs(t - t_ref) <= 1e-12 * t_ref
            assert rel_err(mesh, U, R) <= 1e-12
        else:
            assert l1_rho(mesh, U, R) <= 1e-5
        b.close()
        m.close()


def test_links_between_blocks_of_different_extent():
    mesh = chain_mesh([(32, 16, 16), (16, 16, 16), (48, 16, 16)], axis=0, dx=1.0 / 96)
    check_both(mesh, smooth_state(mesh), 8, packets=[[0], [1, 2]])


def test_ragged_blocks_eight_wide_tiles_three_planes():
    mesh = I.block_grid((3, 1, 2), (24, 40, 3), (0, 0, 0), (1, 1, 1), "outflow", 3)
    check_both(mesh, smooth_state(mesh), 8)


def test_two_plane_blocks_linked_along_z():
    mesh = chain_mesh([(16, 16, 2)] * 3, axis=2, dx=1.0 / 16)
    check_both(mesh, smooth_state(mesh), 8)


def test_2d_non_square_blocks():
    mesh = chain_mesh([(16, 32, 1), (48, 32, 1)], axis=0, dx=1.0 / 64, ndim=2)
    check_both(mesh, smooth_state(mesh), 10)


def test_single_self_periodic_block_packet_and_graph():
    mesh = I.independent_blocks([32], 3)
    U0 = smooth_state(mesh)
    R = U0.copy()
    dts, _ = O.run(mesh, R, 5, CFL, GAMMA)
    for path in ("packet", "graph"):
        arena = to_dev(U0)
        m = H.Mesh(mesh, arena)
        pk = H.Packet(m, [0], H.FP64)
        if path == "packet":
            for s in range(5):
                dt = pk.reduce_dt(GAMMA, CFL)
                assert abs(dt - dts[s]) <= 1e-12 * dts[s]
                pk.advance(dt, GAMMA)
        else:
            b = H.Batch([pk])
            b.run(5, CFL, GAMMA)
        assert rel_err(mesh, to_host(arena), R) <= 1e-12


def test_supersonic_flow_every_face_upwind():
    """Mach ~3.4 flow along x over a density wave: every x face takes the
    upwind (left-state) branch of HLLC."""
    mesh = I.block_grid((2, 1, 1), (16, 16, 8), (0, 0, 0), (1, 0.5, 0.25), "periodic", 3)
    prims = I.grid_field(mesh, lambda x, y, z: (1.0 + 0.2 * np.sin(2 * np.pi * x), 4.0, 0.0, 0.0, 1.0))
    check_both(mesh, I.conserved_arena(mesh, prims, GAMMA), 10)


def test_widest_block_accepted():
    """A block at the maximum x extent (16384 cells), eight rows, two planes."""
    mesh = I.block_grid((1, 1, 1), (16384, 8, 2), (0, 0, 0), (1, 8.0 / 16384, 2.0 / 16384), "periodic", 3)
    check_both(mesh, smooth_state(mesh), 3)


def test_zero_steps_leave_the_state_untouched():
    """nsteps = 0 through the graph path and the host-resident path, in both
    precisions: t = 0 and the state bit for bit as it was."""
    import torch

    mesh = I.block_grid((2, 2, 2), (16, 16, 16), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = smooth_state(mesh)
    for prec in (H.FP64, H.FP32_FP64):
        arena = to_dev(U0)
        m = H.Mesh(mesh, arena)
        b = H.Batch([H.Packet(m, list(range(mesh.nblocks)), prec)])
        assert b.run(0, CFL, GAMMA) == 0.0
        assert np.array_equal(to_host(arena), U0)
        b.close()
        m.close()
        host = torch.from_numpy(U0.copy()).pin_memory()
        hs = H.HostStream(mesh, host, [list(range(mesh.nblocks))], prec, 2)
        assert hs.run(0, CFL, GAMMA) == 0.0
        hs.close()
        assert np.array_equal(host.numpy(), U0)
