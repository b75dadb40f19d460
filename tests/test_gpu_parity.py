"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars: FP64 path <= 1e-12 relative per cell (floored: the denominator is
max(|ref|, 1e-6 max|ref| of that variable), so a momentum crossing zero is
compared on the field's scale); mixed FP32/FP64 path L1(rho) <= 1e-5 relative
on smooth flow.  Bitwise invariants (uniform state, 2D row identity) hold
exactly on the GPU as in the oracle.
"""
import math

import numpy as np
import pytest

from gpu_util import l1_rho, rel_err, to_dev, to_host
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL_L1_MIXED = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def oracle_run(P, nsteps, fixed_dt=0.0):
    R = P.U0.copy()
    dts, t = O.run(P.mesh, R, nsteps, P.cfl, P.gamma, fixed_dt)
    return R, dts, t


# ------------------------------------------------------------------- C1 Sod
def test_sod2d_packet_path_fp64():
    P = I.sod2d()
    R, dts, t_ref = oracle_run(P, P.nsteps)
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    pk = H.Packet(mesh, range(P.mesh.nblocks), H.FP64)
    for s in range(P.nsteps):
        dt = pk.reduce_dt(P.gamma, P.cfl)
        assert abs(dt - dts[s]) <= TOL64 * dts[s], (s, dt, dts[s])
        pk.advance(dt, P.gamma)
    U = to_host(arena)
    assert rel_err(P.mesh, U, R) <= TOL64


def test_sod2d_graph_path_fp64_and_rows():
    P = I.sod2d()
    R, dts, t_ref = oracle_run(P, P.nsteps)
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    b = H.Batch([H.Packet(mesh, range(P.mesh.nblocks), H.FP64)])
    t = b.run(P.nsteps, P.cfl, P.gamma)
    U = to_host(arena)
    assert abs(t - t_ref) <= TOL64 * t_ref
    assert rel_err(P.mesh, U, R) <= TOL64
    # bitwise: every row identical, rho*v exactly 0
    for blk in range(P.mesh.nblocks):
        f = P.mesh.block_view(U, blk)
        assert np.all(f[2] == 0.0)
        assert all(np.array_equal(f[0, 0, 0], f[0, 0, j]) for j in range(f.shape[2]))


# ----------------------------------------------------------- uniform states
@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
@pytest.mark.parametrize(
    "mk",
    [
        lambda: I.block_grid((2, 2, 1), (16, 16, 1), (0, 0, 0), (1, 1, 1), "outflow", 2),
        lambda: I.block_grid((2, 1, 2), (16, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3),
        lambda: I.block_grid((1, 2, 1), (32, 16, 6), (0, 0, 0), (1, 1, 1), "outflow", 3),
        lambda: I.independent_blocks([8, 16, 32], 3),
    ],
    ids=["2d-outflow", "3d-periodic", "3d-outflow-thin", "3d-selfperiodic"],
)
def test_uniform_state_bitwise(mk, prec):
    mesh_ = mk()
    U0 = I.uniform_state(mesh_, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, gamma=1.4)
    arena = to_dev(U0)
    mesh = H.Mesh(mesh_, arena)
    b = H.Batch([H.Packet(mesh, range(mesh_.nblocks), prec)])
    b.run(4, 0.4, 1.4)
    b.advance_plain(1e-3, 1.4)
    assert np.array_equal(to_host(arena), U0)


# ------------------------------------------------------------- C2 Sedov
@pytest.fixture(scope="module")
def sedov():
    P = I.sedov3d()
    R, dts, t = oracle_run(P, P.nsteps)
    return P, R, dts, t


def test_sedov_plain_per_packet_fp64(sedov):
    P, R, dts, t_ref = sedov
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    pks = [H.Packet(mesh, ids, H.FP64) for ids in P.packets]
    b = H.Batch(pks)
    for s in range(P.nsteps):
        dt = min(pk.reduce_dt(P.gamma, P.cfl) for pk in pks)
        assert abs(dt - dts[s]) <= TOL64 * dts[s], (s, dt, dts[s])
        b.advance_plain(dt, P.gamma)
    U = to_host(arena)
    assert rel_err(P.mesh, U, R) <= TOL64


def test_sedov_graph_fp64_conservation_and_mirror(sedov):
    P, R, dts, t_ref = sedov
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    b = H.Batch([H.Packet(mesh, ids, H.FP64) for ids in P.packets])
    t = b.run(P.nsteps, P.cfl, P.gamma)
    U = to_host(arena)
    assert abs(t - t_ref) <= TOL64 * t_ref
    assert rel_err(P.mesh, U, R) <= TOL64
    # conservation of the totals (periodic mesh)
    vol = float(np.prod(P.mesh.dx[0]))
    for v in range(5):
        a = P.U0.reshape(P.mesh.nblocks, 5, -1)[:, v].ravel()
        c = U.reshape(P.mesh.nblocks, 5, -1)[:, v].ravel()
        # momenta start at exactly 0: scale by the larger of the initial and final sum |U|
        scale = max(math.fsum(np.abs(a)), math.fsum(np.abs(c)))
        assert abs(math.fsum(c) - math.fsum(a)) <= 1e-13 * P.nsteps * scale, v
    # mirror symmetry about x = 1/2 of the centred blast
    from test_oracle_scheme import assemble

    rho = assemble(P.mesh, U, 0)
    assert np.abs(np.flip(rho, axis=2) - rho).max() <= 1e-12 * np.abs(rho).max()


# ------------------------------------------------------ C3 smooth (reduced)
@pytest.mark.parametrize("tile,zchunk", [(0, 0), (1, 0), (0, 4), (3, 0)], ids=["t16", "t8", "t16-z4", "t16-run3"])
def test_smooth_fp64_and_mixed(tile, zchunk):
    P = I.smooth3d(nblk=(4, 4, 4), nsteps=30)
    R, dts, t_ref = oracle_run(P, P.nsteps)
    for prec, check in ((H.FP64, "rel"), (H.FP32_FP64, "l1")):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        b.set_tiling(16, tile, zchunk)
        t = b.run(P.nsteps, P.cfl, P.gamma)
        U = to_host(arena)
        if check == "rel":
            assert rel_err(P.mesh, U, R) <= TOL64
            assert abs(t - t_ref) <= TOL64 * t_ref
        else:
            assert l1_rho(P.mesh, U, R) <= TOL_L1_MIXED
        b.close()
        mesh.close()


# ------------------------------------------------------- C4 uneven (reduced)
def test_uneven_fp64_and_mixed_autotuned():
    P = I.uneven(nblocks=120, nsteps=20)
    R, dts, t_ref = oracle_run(P, P.nsteps)
    for prec in (H.FP64, H.FP32_FP64):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        b.autotune(P.gamma, reps=2)
        cfg = b.config()
        assert {c["edge"] for c in cfg["classes"]} == {8, 16, 32}
        t = b.run(P.nsteps, P.cfl, P.gamma)
        U = to_host(arena)
        if prec == H.FP64:
            assert rel_err(P.mesh, U, R) <= TOL64
            assert abs(t - t_ref) <= TOL64 * t_ref
        else:
            assert l1_rho(P.mesh, U, R) <= TOL_L1_MIXED
        b.close()
        mesh.close()


# -------------------------------------------------------------- errors
def test_nonphysical_state_reported():
    m = I.block_grid((2, 1, 1), (16, 16, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = I.uniform_state(m, gamma=1.4)
    m.block_view(U0, 1)[4, 3, 5, 7] = 0.0  # E < rho|v|^2/2
    arena = to_dev(U0)
    mesh = H.Mesh(m, arena)
    pk = H.Packet(mesh, range(m.nblocks), H.FP64)
    with pytest.raises(H.HydroError) as e:
        pk.reduce_dt(1.4, 0.4)
    assert e.value.code == H.ENONPHYS and "block 1" in str(e.value)
    b = H.Batch([pk])
    with pytest.raises(H.HydroError) as e:
        b.run(2, 0.4, 1.4)
    assert e.value.code == H.ENONPHYS


def test_bad_initial_state_leaves_the_arena_untouched():
    """A non-physical initial state is caught by the rate reduction before the
    first step: every stage launch of the run then returns at once, so the
    arena (and, through staging slots, the host arena) is bitwise unchanged."""
    import torch

    m = I.block_grid((2, 1, 1), (16, 16, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = I.uniform_state(m, gamma=1.4)
    m.block_view(U0, 1)[4, 3, 5, 7] = 0.0  # E < rho|v|^2/2
    for prec in (H.FP64, H.FP32_FP64):
        arena = to_dev(U0)
        mesh = H.Mesh(m, arena)
        b = H.Batch([H.Packet(mesh, range(m.nblocks), prec)])
        with pytest.raises(H.HydroError) as e:
            b.run(5, 0.4, 1.4)
        assert e.value.code == H.ENONPHYS and "block 1" in str(e.value)
        assert np.array_equal(to_host(arena), U0)
        mesh.close()
        host = torch.from_numpy(U0.copy()).pin_memory()
        hs = H.HostStream(m, host, [[0, 1]], prec, 2)
        with pytest.raises(H.HydroError) as e:
            hs.run(5, 0.4, 1.4)
        assert e.value.code == H.ENONPHYS
        hs.close()
        assert np.array_equal(host.numpy(), U0)


def _unstable_sod():
    """2D Sod at CFL 2.3, far above the scheme's stable limit: the growing
    instability makes a pressure negative.  The oracle's state after the
    failing step is finite and non-physical (its next rate reduction
    reports it)."""
    P = I.sod2d()
    cfl = 2.3
    R = P.U0.copy()
    t = 0.0
    for k in range(40):
        try:
            dt = O.dt(P.mesh, R, P.gamma, cfl)
        except O.OracleError as e:
            assert e.code == O.ENONPHYS
            return P, cfl, R, k, t
        O.step(P.mesh, R, dt, P.gamma)
        t += dt
    raise AssertionError("the unstable run did not fail")


def test_failing_step_result_kept_fp64():
    """Graph path and host-resident packets: a run of 20 steps whose k-th step
    makes the state non-physical returns ENONPHYS with the arena holding the
    result of step k (equal to the oracle's state after k steps, finite) and
    t the time at its end; the replays after it touch nothing."""
    import torch

    P, cfl, R, k, t_ref = _unstable_sod()
    assert 2 <= k < 20 and np.isfinite(R).all()
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    b = H.Batch([H.Packet(mesh, range(P.mesh.nblocks), H.FP64)])
    t = C_double_run(b, 20, cfl, P.gamma)
    U = to_host(arena)
    assert np.isfinite(U).all()
    assert rel_err(P.mesh, U, R) <= TOL64
    assert abs(t - t_ref) <= TOL64 * t_ref
    mesh.close()
    host = torch.from_numpy(P.U0.copy()).pin_memory()
    hs = H.HostStream(P.mesh, host, [list(range(P.mesh.nblocks))], H.FP64, 2)
    with pytest.raises(H.HydroError) as e:
        hs.run(20, cfl, P.gamma)
    assert e.value.code == H.ENONPHYS
    hs.close()
    assert rel_err(P.mesh, host.numpy(), R) <= TOL64


def C_double_run(b, nsteps, cfl, gamma):
    """hydro_batch_run expected to fail with ENONPHYS; returns the t it reports."""
    import ctypes as C

    t = C.c_double(-1.0)
    rc = H.lib().hydro_batch_run(b.h, int(nsteps), float(cfl), float(gamma), C.byref(t))
    assert rc == H.ENONPHYS, rc
    return t.value


def test_failing_step_result_kept_mixed():
    """The mixed path fails at its own step j of the unstable run (the first
    run length n for which a run from the initial state reports ENONPHYS):
    a run of 20 steps leaves bitwise the state and time of the run of j
    steps, i.e. the steps after the failing one touch nothing."""
    P, cfl, _, _, _ = _unstable_sod()
    arena = to_dev(P.U0)
    mesh = H.Mesh(P.mesh, arena)
    b = H.Batch([H.Packet(mesh, range(P.mesh.nblocks), H.FP32_FP64)])
    j = None
    for n in range(1, 20):
        arena.copy_(to_dev(P.U0))
        try:
            b.run(n, cfl, P.gamma)
        except H.HydroError as e:
            assert e.code == H.ENONPHYS
            j = n
            break
    assert j is not None and j >= 2
    U_j = to_host(arena)
    arena.copy_(to_dev(P.U0))
    t_j = C_double_run(b, j, cfl, P.gamma)
    assert np.array_equal(to_host(arena), U_j)
    arena.copy_(to_dev(P.U0))
    t_20 = C_double_run(b, 20, cfl, P.gamma)
    assert np.array_equal(to_host(arena), U_j) and t_20 == t_j
    mesh.close()


def test_open_packet_refuses_advance_and_batch_is_stage_synchronous():
    m = I.block_grid((2, 1, 1), (16, 16, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = I.random_smooth_state(m, 3, 1.4)
    arena = to_dev(U0)
    mesh = H.Mesh(m, arena)
    p0, p1 = H.Packet(mesh, [0], H.FP64), H.Packet(mesh, [1], H.FP64)
    with pytest.raises(H.HydroError) as e:
        p0.advance(1e-3, 1.4)
    assert e.value.code == H.ESTATE
    b = H.Batch([p0, p1])
    b.advance_plain(1e-3, 1.4)
    R = U0.copy()
    O.step(m, R, 1e-3, 1.4)
    assert rel_err(m, to_host(arena), R) <= TOL64


def test_deterministic_bitwise():
    P = I.smooth3d(nblk=(2, 2, 2), nsteps=5)
    outs = []
    for _ in range(2):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, range(P.mesh.nblocks), H.FP32_FP64)])
        b.run(P.nsteps, P.cfl, P.gamma)
        outs.append(to_host(arena))
        b.close()
        mesh.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_autotune_leaves_the_state_untouched(prec):
    """The tuner launches both RK stages of every candidate; they write only
    the library's scratch buffer, so the caller's arena is bitwise unchanged
    and a run afterwards equals a run without tuning."""
    P = I.smooth3d(nblk=(2, 2, 4), nsteps=3)
    outs = []
    for tune in (False, True):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, range(P.mesh.nblocks), prec)])
        if tune:
            b.autotune(P.gamma, reps=1)
            assert np.array_equal(to_host(arena), P.U0)
        b.run(P.nsteps, P.cfl, P.gamma)
        outs.append(to_host(arena))
        b.close()
        mesh.close()
    if prec == H.FP64:  # any tiling reproduces the oracle's rounding
        assert np.array_equal(outs[0], outs[1])
    else:
        assert l1_rho(P.mesh, outs[1], outs[0]) <= 1e-6


def test_timed_run_matches_run_and_reports_step_times():
    """hydro_batch_run_timed replays the same graph as hydro_batch_run (same
    state and time, bitwise) and returns one positive device time per step."""
    P = I.smooth3d(nblk=(2, 2, 2), nsteps=5)
    outs, times = [], []
    for timed in (False, True):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, range(P.mesh.nblocks), H.FP32_FP64)])
        if timed:
            t, ms = b.run_timed(P.nsteps, P.cfl, P.gamma)
            assert len(ms) == P.nsteps and all(x > 0.0 for x in ms)
        else:
            t = b.run(P.nsteps, P.cfl, P.gamma)
        outs.append(to_host(arena))
        times.append(t)
        b.close()
        mesh.close()
    assert np.array_equal(outs[0], outs[1]) and times[0] == times[1]


# ---------------------------------------------------- host-resident packets
def test_host_resident_packets_match_device_batch_and_oracle():
    """Packets kept in pinned host memory, streamed through device slots (copy
    in, two stage launches, copy back on one stream per slot), one packet per
    transfer unit or consecutive packets merged into units of at least 1 MiB
    and of at least 64 MiB (all GPU packets in one unit): the result equals
    the device-resident batch bit for bit and, in FP64, the oracle."""
    import torch

    P = I.uneven(nblocks=150, nsteps=8)
    R, dts, t_ref = oracle_run(P, P.nsteps)
    for prec in (H.FP64, H.FP32_FP64):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        t_dev = b.run(P.nsteps, P.cfl, P.gamma)
        U_dev = to_host(arena)
        mesh.close()
        for nslots, unit in ((1, 0), (3, 0), (3, 1 << 20), (2, 64 << 20)):
            host = torch.from_numpy(P.U0.copy()).pin_memory()
            hs = H.HostStream(P.mesh, host, P.packets, prec, nslots)
            if unit:
                hs.set_unit_bytes(unit)
            t = hs.run(P.nsteps, P.cfl, P.gamma)
            hs.close()
            U = host.numpy()
            assert np.array_equal(U, U_dev) and t == t_dev, (prec, nslots, unit)
        if prec == H.FP64:
            assert rel_err(P.mesh, U_dev, R) <= TOL64


def test_autotune_results_cached_as_json(tmp_path):
    """The tuned configuration is stored under the batch's key; a second batch
    of the same shape takes it from the file without timing and computes the
    same result."""
    import json

    P = I.uneven(nblocks=60, nsteps=4)
    cache = str(tmp_path / "tuning.json")
    outs = []
    for k in range(2):
        arena = to_dev(P.U0)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, H.FP32_FP64) for ids in P.packets])
        cfg = b.autotune(P.gamma, reps=1, cache=cache)
        assert b.config() == cfg
        with open(cache) as f:
            assert json.load(f)[b.tuning_key()] == cfg
        b.run(P.nsteps, P.cfl, P.gamma)
        outs.append((cfg, to_host(arena)))
        b.close()
        mesh.close()
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("prec", [H.FP64, H.FP32_FP64], ids=["fp64", "mixed"])
def test_checkpoint_resume_bitwise(prec, tmp_path):
    """20 steps in one run equal 10 steps, a save of the arena to a file, a new
    mesh and batch over the loaded state, and 10 more steps -- bit for bit:
    the run keeps no state but the arena and the time (the resumed run's
    first dt is a fresh reduction, the same rate its stage 2 reduces)."""
    P = I.smooth3d(nblk=(2, 2, 2), nsteps=20)

    def run(U, n):
        arena = to_dev(U)
        mesh = H.Mesh(P.mesh, arena)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        t = b.run(n, P.cfl, P.gamma)
        out = to_host(arena)
        mesh.close()
        return out, t

    U20, t20 = run(P.U0, 20)
    U10, t10 = run(P.U0, 10)
    path = tmp_path / "state.npy"
    np.save(path, U10)
    Ur, tr = run(np.load(path), 10)
    assert np.array_equal(Ur, U20)
    assert abs((t10 + tr) - t20) <= 1e-15 * t20
