"""GPU parity of the method variants -- HLLC wave-speed bounds
(HYDRO_SPEEDS_EINFELDT, HYDRO_SPEEDS_PVRS) and PLM on conserved variables
(HYDRO_RECON_CONSERVED, alone and with Einfeldt bounds) and on characteristic
variables (HYDRO_RECON_CHARACTERISTIC, alone and with PVRS bounds) and the gas +
radiation equation of state (HYDRO_EOS_GAS_RADIATION, FP64 only) -- against the oracle
run with the same options, through the C ABI: FP64 <= 1e-12 relative per cell
(floored), mixed L1(rho) <= 1e-5 on smooth flow; uniform states bitwise;
conservation on a periodic blast; the host-resident packet path with each
variant; a non-physical face state of conserved reconstruction reported."""
import math

import numpy as np
import pytest

from gpu_util import l1_rho, rel_err, to_dev, to_host
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu

# (library flags, oracle options)
VARIANTS = {
    "einfeldt": (H.EINFELDT, dict(speeds=O.EINFELDT)),
    "pvrs": (H.PVRS, dict(speeds=O.PVRS)),
    "conserved": (H.CONSERVED, dict(recon=O.CONSERVED)),
    "conserved-einfeldt": (H.CONSERVED | H.EINFELDT, dict(speeds=O.EINFELDT, recon=O.CONSERVED)),
    "characteristic": (H.CHARACTERISTIC, dict(recon=O.CHARACTERISTIC)),
    "characteristic-pvrs": (H.CHARACTERISTIC | H.PVRS, dict(speeds=O.PVRS, recon=O.CHARACTERISTIC)),
    "gas-radiation": (H.GAS_RADIATION, dict(eos=O.GAS_RADIATION)),
}
FP64_ONLY = {H.GAS_RADIATION}


def precisions(flags):
    return (H.FP64,) if flags in FP64_ONLY else (H.FP64, H.FP32_FP64)


@pytest.fixture(params=sorted(VARIANTS), scope="module")
def variant(request):
    return VARIANTS[request.param]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def oracle_run(mesh, U0, nsteps, cfl, gamma, opts):
    R = U0.copy()
    dts, t = O.run(mesh, R, nsteps, cfl, gamma, **opts)
    return R, dts, t


@pytest.mark.parametrize("tile", [0, 1], ids=["t16", "t8"])
def test_smooth_fp64_and_mixed(variant, tile):
    EF, opts = variant
    P = I.smooth3d(nblk=(3, 3, 3), nsteps=15)
    R, dts, t_ref = oracle_run(P.mesh, P.U0, P.nsteps, P.cfl, P.gamma, opts)
    for prec in precisions(EF):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, prec | EF) for ids in P.packets])
        b.set_tiling(16, tile, 0)
        t = b.run(P.nsteps, P.cfl, P.gamma)
        U = to_host(arena)
        if prec == H.FP64:
            assert abs(t - t_ref) <= 1e-12 * t_ref
            assert rel_err(P.mesh, U, R) <= 1e-12
        else:
            assert l1_rho(P.mesh, U, R) <= 1e-5
        b.close()
        mesh.close()


def test_2d_smooth_fp64_and_mixed(variant):
    """The 2D kernels of the variant: self-periodic blocks of 16^2 and 32^2
    (16x16 tiles and z-free faces), smooth random flow."""
    EF, opts = variant
    m = I.independent_blocks([16, 32, 16], 2)
    U0 = I.random_smooth_state(m, 5, 1.4)
    R, dts, t_ref = oracle_run(m, U0, 10, 0.4, 1.4, opts)
    for prec in precisions(EF):
        arena = to_dev(U0)
        mesh = H.Mesh(m, arena)
        b = H.Batch([H.Packet(mesh, range(m.nblocks), prec | EF)])
        t = b.run(10, 0.4, 1.4)
        U = to_host(arena)
        if prec == H.FP64:
            assert abs(t - t_ref) <= 1e-12 * t_ref
            assert rel_err(m, U, R) <= 1e-12
        else:
            assert l1_rho(m, U, R) <= 1e-5
        b.close()
        mesh.close()


def test_ragged_blocks_partly_filled_items(variant):
    """Blocks only the 8x8 tiling covers (24x40, three planes, outflow), so
    some four-tile items carry empty slots, whose garbage LDS must neither
    reach a result nor raise a non-physical flag."""
    EF, opts = variant
    m = I.block_grid((3, 1, 2), (24, 40, 3), (0, 0, 0), (1, 1, 1), "outflow", 3)
    prims = I.grid_field(m, lambda x, y, z: (1 + 0.2 * np.sin(2 * np.pi * (x + y)), 0.3 * np.cos(2 * np.pi * y),
                                             0.2 * np.sin(2 * np.pi * x), 0.1 + 0 * x, 1 + 0.3 * np.cos(2 * np.pi * z)))
    U0 = I.conserved_arena(m, prims, 1.4)
    R, dts, t_ref = oracle_run(m, U0, 6, 0.4, 1.4, opts)
    for prec in precisions(EF):
        arena = to_dev(U0)
        mesh = H.Mesh(m, arena)
        b = H.Batch([H.Packet(mesh, range(m.nblocks), prec | EF)])
        t = b.run(6, 0.4, 1.4)
        U = to_host(arena)
        if prec == H.FP64:
            assert abs(t - t_ref) <= 1e-12 * t_ref
            assert rel_err(m, U, R) <= 1e-12
        else:
            assert l1_rho(m, U, R) <= 1e-5
        b.close()
        mesh.close()


def test_sod2d_packet_path_fp64(variant):
    EF, opts = variant
    P = I.sod2d()
    R, dts, _ = oracle_run(P.mesh, P.U0, P.nsteps, P.cfl, P.gamma, opts)
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    pk = H.Packet(mesh, range(P.mesh.nblocks), H.FP64 | EF)
    for s in range(P.nsteps):
        dt = pk.reduce_dt(P.gamma, P.cfl)
        assert abs(dt - dts[s]) <= 1e-12 * dts[s]
        pk.advance(dt, P.gamma)
    assert rel_err(P.mesh, to_host(arena), R) <= 1e-12


def test_blast_plain_path_conservation(variant):
    EF, opts = variant
    gamma = 1.4
    m = I.block_grid((3, 3, 3), (16, 16, 16), (0, 0, 0), (1, 1, 1), "periodic", 3)
    prims = I.grid_field(m, lambda x, y, z: (1.0, 0.0, 0.0, 0.0, 1e-3))
    I.sedov_deposit(m, prims, 1.0, 2.0, (0.5, 0.5, 0.5), gamma)
    U0 = I.conserved_arena(m, prims, gamma)
    R, dts, _ = oracle_run(m, U0, 10, 0.4, gamma, opts)
    arena = to_dev(U0)
    mesh = H.Mesh(m, arena)
    pks = [H.Packet(mesh, range(9 * k, 9 * k + 9), H.FP64 | EF) for k in range(3)]
    b = H.Batch(pks)
    for s in range(10):
        dt = min(pk.reduce_dt(gamma, 0.4) for pk in pks)
        assert abs(dt - dts[s]) <= 1e-12 * dts[s]
        b.advance_plain(dt, gamma)
    U = to_host(arena)
    assert rel_err(m, U, R) <= 1e-12
    for v in range(5):
        a = U0.reshape(m.nblocks, 5, -1)[:, v].ravel()
        c = U.reshape(m.nblocks, 5, -1)[:, v].ravel()
        scale = max(math.fsum(np.abs(a)), math.fsum(np.abs(c)))
        assert abs(math.fsum(c) - math.fsum(a)) <= 1e-13 * 10 * scale


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_uniform_state_bitwise(variant, prec):
    EF, _ = variant
    if prec not in precisions(EF):
        pytest.skip("this variant runs in FP64 only")
    m = I.block_grid((2, 1, 2), (16, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = I.uniform_state(m, gamma=1.4)
    arena = to_dev(U0)
    mesh = H.Mesh(m, arena)
    b = H.Batch([H.Packet(mesh, range(m.nblocks), prec | EF)])
    b.run(3, 0.4, 1.4)
    assert np.array_equal(to_host(arena), U0)


def test_host_resident_packets(variant):
    import torch

    EF, opts = variant
    P = I.uneven(nblocks=40, nsteps=6)
    R, _, t_ref = oracle_run(P.mesh, P.U0, P.nsteps, P.cfl, P.gamma, opts)
    host = torch.from_numpy(P.U0.copy()).pin_memory()
    hs = H.HostStream(P.mesh, host, P.packets, H.FP64 | EF, 2)
    t = hs.run(P.nsteps, P.cfl, P.gamma)
    hs.close()
    assert abs(t - t_ref) <= 1e-12 * t_ref
    assert rel_err(P.mesh, host.numpy(), R) <= 1e-12


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_conserved_reconstruction_reports_non_physical_face_state(prec):
    """Velocity shear at low pressure: every cell is physical, but conserved
    reconstruction gives face states with p < 0 (the oracle reports them);
    the step must fail with HYDRO_ENONPHYS, and primitive reconstruction of
    the same state must not."""
    m = I.block_grid((1, 1, 1), (16, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    prims = I.grid_field(m, lambda x, y, z: (1.0, 5 * np.sin(2 * np.pi * x), 0.0, 0.0, 0.1))
    U0 = I.conserved_arena(m, prims, 1.4)
    O.run(m, U0.copy(), 1, 0.4, 1.4)  # primitive reconstruction: a physical step
    with pytest.raises(O.OracleError) as e:
        O.run(m, U0.copy(), 1, 0.4, 1.4, recon=O.CONSERVED)
    assert e.value.code == O.ENONPHYS
    for flags, ok in ((0, True), (H.CONSERVED, False)):
        arena = to_dev(U0)
        mesh = H.Mesh(m, arena)
        b = H.Batch([H.Packet(mesh, range(m.nblocks), prec | flags)])
        if ok:
            b.run(1, 0.4, 1.4)
        else:
            with pytest.raises(H.HydroError) as e:
                b.run(1, 0.4, 1.4)
            assert e.value.code == H.ENONPHYS
        b.close()
        mesh.close()
