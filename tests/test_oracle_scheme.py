"""Pins of the whole oracle step (guard fill + recovery + PLM + HLLC + SSP-RK2 +
CFL dt) against what the mathematics fixes:

* a uniform state (any velocity) is a fixed point, bitwise, for every kind of
  face (linked, periodic, outflow) in 2D and 3D;
* a mesh split into linked blocks gives bitwise the result of one big block
  (guard fill = the neighbour's interior);
* conservation of mass, momentum and energy to round-off on periodic meshes;
* Sod shock tube: rows stay bit-identical and rho*v == 0 in 2D; the solution
  converges to the exact Riemann solution; the shock sits where the exact
  shock speed puts it;
* the x, y and z sweeps are the same operator (axis permutation is bitwise a
  transpose; a 3D x-problem reproduces the 2D rows bitwise);
* mirror symmetry of a centred blast;
* smooth advection converges at better than first order to the translated
  exact solution, keeping u and p uniform;
* the CFL rate of a uniform state has its closed form; non-physical states
  are reported; a subset step equals the whole-mesh step on its blocks; the
  result does not depend on the number of OpenMP threads.
"""
import math

import numpy as np
import pytest

from oracle import exact_riemann as ER
from oracle import oracle as O
from paper_2507_09337_amd import inputs as I


def prims_of(mesh, U, gamma):
    out = []
    for b in range(mesh.nblocks):
        blk = mesh.block_view(U, b)
        rho = blk[0]
        u, v, w = blk[1] / rho, blk[2] / rho, blk[3] / rho
        p = (gamma - 1) * (blk[4] - 0.5 * rho * (u * u + v * v + w * w))
        out.append(np.stack([rho, u, v, w, p]))
    return out


def assemble(mesh, U, var=0):
    """Global (Z, Y, X) field of one variable on a uniform block grid."""
    nbx, nby, nbz = mesh.grid
    nx, ny, nz = (int(v) for v in mesh.n[0])
    out = np.empty((nbz * nz, nby * ny, nbx * nx))
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                b = (bz * nby + by) * nbx + bx
                out[bz * nz:(bz + 1) * nz, by * ny:(by + 1) * ny, bx * nx:(bx + 1) * nx] = mesh.block_view(U, b)[var]
    return out


def field_state(mesh, f, gamma):
    return I.conserved_arena(mesh, I.grid_field(mesh, f), gamma)


# --------------------------------------------------------------- uniform
@pytest.mark.parametrize(
    "mesh",
    [
        I.block_grid((4, 2, 1), (8, 8, 1), (0, 0, 0), (1, 0.5, 1), "outflow", 2),
        I.block_grid((2, 2, 2), (4, 4, 4), (0, 0, 0), (1, 1, 1), "periodic", 3),
        I.block_grid((2, 1, 2), (4, 6, 4), (0, 0, 0), (1, 1, 1), "outflow", 3),
        I.independent_blocks([4, 8], 3),
        I.independent_blocks([6], 2),
    ],
    ids=["2d-outflow", "3d-periodic", "3d-outflow", "3d-selfperiodic", "2d-selfperiodic"],
)
def test_uniform_state_is_fixed_point_bitwise(mesh):
    gamma = 1.4
    U0 = I.uniform_state(mesh, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, gamma=gamma)
    U = U0.copy()
    O.run(mesh, U, 5, 0.4, gamma)
    assert np.array_equal(U, U0)


def test_cfl_rate_of_uniform_state_closed_form():
    gamma = 1.4
    mesh = I.block_grid((2, 1, 1), (4, 4, 4), (0, 0, 0), (1, 0.5, 0.25), "periodic", 3)
    U = I.uniform_state(mesh, rho=2.0, vel=(0.3, -0.2, 0.1), p=0.7, gamma=gamma)
    c = math.sqrt(gamma * 0.7 / 2.0)
    dx = mesh.dx[0]
    want = (0.3 + c) / dx[0] + (0.2 + c) / dx[1] + (0.1 + c) / dx[2]
    assert O.max_lambda(mesh, U, gamma) == pytest.approx(want, rel=1e-14)


# ---------------------------------------------------- block decomposition
def test_linked_blocks_equal_one_block_3d():
    gamma = 5.0 / 3.0
    one = I.independent_blocks([16], 3)
    split = I.block_grid((2, 2, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    f = lambda x, y, z: (1 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y), 0.3 * np.cos(2 * np.pi * z),
                         -0.2 * np.sin(2 * np.pi * (x + y)), 0.1 + 0 * x, 1 + 0.1 * np.cos(2 * np.pi * (x - z)))
    U1, U8 = field_state(one, f, gamma), field_state(split, f, gamma)
    d1, _ = O.run(one, U1, 3, 0.4, gamma)
    d8, _ = O.run(split, U8, 3, 0.4, gamma)
    assert np.array_equal(d1, d8)
    for v in range(5):
        assert np.array_equal(one.block_view(U1, 0)[v], assemble(split, U8, v))


def test_linked_blocks_equal_one_block_2d_outflow():
    gamma = 1.4
    one = I.block_grid((1, 1, 1), (32, 16, 1), (0, 0, 0), (1, 0.5, 1), "outflow", 2)
    split = I.block_grid((4, 2, 1), (8, 8, 1), (0, 0, 0), (1, 0.5, 1), "outflow", 2)
    f = lambda x, y, z: (np.where((x - 0.4) ** 2 + (y - 0.2) ** 2 < 0.02, 2.0, 1.0), 0.2 + 0 * x, -0.1 + 0 * x, 0.0,
                         np.where(x < 0.6, 1.0, 0.3))
    U1, U8 = field_state(one, f, gamma), field_state(split, f, gamma)
    O.run(one, U1, 6, 0.4, gamma)
    O.run(split, U8, 6, 0.4, gamma)
    for v in range(5):
        assert np.array_equal(assemble(one, U1, v), assemble(split, U8, v))


# ------------------------------------------------------------ conservation
@pytest.mark.parametrize("kind", ["grid", "selfperiodic"])
def test_conservation_periodic(kind):
    gamma = 1.4
    if kind == "grid":
        mesh = I.block_grid((2, 2, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    else:
        mesh = I.independent_blocks([8, 12], 3)
    U = I.random_smooth_state(mesh, 7, gamma)
    # add a strong pressure pulse so that shocks and limiter switching occur
    for b in range(mesh.nblocks):
        blk = mesh.block_view(U, b)
        blk[4, 1:3, 2:4, 1:3] += 5.0
    vol = np.repeat(mesh.dx.prod(axis=1), mesh.ncells)

    def totals(U):
        out = []
        for v in range(5):
            vals = np.concatenate([mesh.block_view(U, b)[v].ravel() for b in range(mesh.nblocks)])
            out.append((math.fsum(vals * vol), math.fsum(np.abs(vals) * vol)))
        return out

    t0 = totals(U)
    O.run(mesh, U, 10, 0.4, gamma)
    t1 = totals(U)
    for v in range(5):
        assert abs(t1[v][0] - t0[v][0]) <= 1e-13 * t0[v][1] * 10, (v, t1[v][0] - t0[v][0])


# ---------------------------------------------------------------------- Sod
def sod_mesh(ncell_x, block=16):
    nb = ncell_x // block
    return I.block_grid((nb, 1, 1), (block, 2, 1), (0, 0, 0), (1, 2.0 / ncell_x, 1), "outflow", 2)


def sod_state(mesh, gamma=1.4):
    return field_state(mesh, lambda x, y, z: (np.where(x < 0.5, 1.0, 0.125), 0.0, 0.0, 0.0,
                                              np.where(x < 0.5, 1.0, 0.1)), gamma)


def run_to(mesh, U, t_end, gamma, cfl=0.4):
    t = 0.0
    while t < t_end:
        dt = min(O.dt(mesh, U, gamma, cfl), t_end - t)
        O.step(mesh, U, dt, gamma)
        t += dt
    return t


def sod_l1(ncell):
    gamma = 1.4
    mesh = sod_mesh(ncell)
    U = sod_state(mesh, gamma)
    run_to(mesh, U, 0.2, gamma)
    rho = assemble(mesh, U, 0)[0]
    x = (np.arange(ncell) + 0.5) / ncell
    star = ER.star_state(1, 0, 1, 0.125, 0, 0.1, gamma)
    exact = np.array([ER.sample((xi - 0.5) / 0.2, 1, 0, 1, 0.125, 0, 0.1, gamma, star=star)[0] for xi in x])
    return float(np.abs(rho[0] - exact).sum() / ncell), rho, x, mesh, U


def test_sod_converges_to_exact_solution():
    errs = [sod_l1(n)[0] for n in (64, 128, 256)]
    assert errs[0] <= 2e-2
    assert errs[0] / errs[1] >= 1.5 and errs[1] / errs[2] >= 1.5, errs


def test_sod_shock_position_and_rows():
    err, rho, x, mesh, U = sod_l1(256)
    full = assemble(mesh, U, 0)[0]
    assert all(np.array_equal(full[0], full[j]) for j in range(full.shape[0]))
    assert np.all(assemble(mesh, U, 2) == 0.0)
    # shock: the steepest density drop right of the contact
    s_exact = 0.5 + ER.wave_speeds(1, 0, 1, 0.125, 0, 0.1, 1.4)["r_shock"] * 0.2
    right = x > 0.8
    jump = np.abs(np.diff(rho[0]))[right[:-1]]
    xs = x[:-1][right[:-1]][np.argmax(jump)] + 0.5 / 256
    assert abs(xs - s_exact) <= 2.0 / 256


def test_sod2d_config_rows_bit_identical():
    P = I.sod2d()
    U = P.U0.copy()
    O.run(P.mesh, U, P.nsteps, P.cfl, P.gamma)
    rho = assemble(P.mesh, U, 0)
    assert all(np.array_equal(rho[0, 0], rho[0, j]) for j in range(rho.shape[1]))
    assert np.all(assemble(P.mesh, U, 2) == 0.0)
    assert not np.array_equal(U, P.U0)


# -------------------------------------------------------- axis permutation
def test_axis_permutation_and_2d_3d_consistency():
    gamma, dt, steps = 1.4, 2e-3, 8

    def sod_along(axis):
        ncell = [4, 4, 4]
        ncell[axis] = 32
        mesh = I.block_grid(tuple(2 if a == axis else 1 for a in range(3)),
                            tuple(16 if a == axis else 4 for a in range(3)), (0, 0, 0), (1, 1, 1), "outflow", 3)
        c = [None] * 3

        def f(x, y, z):
            q = (x, y, z)[axis]
            vel = [0.0, 0.0, 0.0]
            return np.where(q < 0.5, 1.0, 0.125), vel[0], vel[1], vel[2], np.where(q < 0.5, 1.0, 0.1)

        U = field_state(mesh, f, gamma)
        O.run(mesh, U, steps, 0.4, gamma, fixed_dt=dt)
        return [np.moveaxis(assemble(mesh, U, v), 2 - axis, 2) for v in range(5)]

    X, Y, Z = sod_along(0), sod_along(1), sod_along(2)
    # density and energy identical; the normal momentum moves to the swept axis
    for v in (0, 4):
        assert np.array_equal(X[v], Y[v]) and np.array_equal(X[v], Z[v])
    assert np.array_equal(X[1], Y[2]) and np.array_equal(X[1], Z[3])
    # 2D x-problem reproduces the 3D rows bitwise
    mesh2 = I.block_grid((2, 1, 1), (16, 4, 1), (0, 0, 0), (1, 1, 1), "outflow", 2)
    U2 = field_state(mesh2, lambda x, y, z: (np.where(x < 0.5, 1.0, 0.125), 0.0, 0.0, 0.0,
                                             np.where(x < 0.5, 1.0, 0.1)), gamma)
    O.run(mesh2, U2, steps, 0.4, gamma, fixed_dt=dt)
    for v in range(5):
        two = assemble(mesh2, U2, v)[0]
        for k in range(X[v].shape[0]):
            assert np.array_equal(X[v][k], two)


# -------------------------------------------------------------- mirror blast
def test_centred_blast_mirror_symmetry():
    gamma = 1.4
    mesh = I.block_grid((2, 2, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    prims = I.grid_field(mesh, lambda x, y, z: (1.0, 0.0, 0.0, 0.0, 1e-3))
    I.sedov_deposit(mesh, prims, 1.0, 2.0, (0.5, 0.5, 0.5), gamma)
    U = I.conserved_arena(mesh, prims, gamma)
    O.run(mesh, U, 6, 0.4, gamma)
    F = [assemble(mesh, U, v) for v in range(5)]  # (z, y, x)
    for axis in range(3):  # numpy axis 2 - axis is the physical axis
        ax = 2 - axis
        for v in range(5):
            ref = F[v]
            scale = np.abs(ref).max()
            mir = np.flip(ref, axis=ax) * (-1.0 if v == 1 + axis else 1.0)
            assert np.abs(mir - ref).max() <= 1e-12 * scale, (axis, v)
    # x <-> y transposition maps the field onto itself (momenta swapped)
    assert np.abs(np.swapaxes(F[0], 1, 2) - F[0]).max() <= 1e-12 * np.abs(F[0]).max()
    assert np.abs(np.swapaxes(F[1], 1, 2) - F[2]).max() <= 1e-12 * np.abs(F[1]).max()


# ---------------------------------------------------------- smooth advection
def advection_l1(ncell, t_end=0.25):
    gamma = 1.4
    mesh = I.block_grid((ncell // 16, 1, 1), (16, 2, 1), (0, 0, 0), (1, 2.0 / ncell, 1), "periodic", 2)
    U = field_state(mesh, lambda x, y, z: (1 + 0.1 * np.sin(2 * np.pi * x), 1.0 + 0 * x, 0.0, 0.0, 1.0 + 0 * x), gamma)
    run_to(mesh, U, t_end, gamma)
    rho = assemble(mesh, U, 0)[0, 0]
    x = (np.arange(ncell) + 0.5) / ncell
    # exact cell average of the translated wave
    exact = 1 + 0.1 * (np.cos(2 * np.pi * (x - 0.5 / ncell - t_end)) - np.cos(2 * np.pi * (x + 0.5 / ncell - t_end))) \
        / (2 * np.pi / ncell)
    W = prims_of(mesh, U, gamma)
    u_dev = max(np.abs(w[1] - 1.0).max() for w in W)
    p_dev = max(np.abs(w[4] - 1.0).max() for w in W)
    return float(np.abs(rho - exact).mean()), u_dev, p_dev


def test_smooth_advection_order():
    res = [advection_l1(n) for n in (32, 64, 128)]
    errs = [r[0] for r in res]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.5, (errs, orders)
    for _, u_dev, p_dev in res:
        assert u_dev <= 1e-12 and p_dev <= 1e-12


# ------------------------------------------------------------ outflow faces
def _euler_flux(W, gamma, axis):
    r, vel, p = W[0], W[1:4], W[4]
    un = vel[axis]
    E = p / (gamma - 1) + 0.5 * r * (vel ** 2).sum(axis=0)
    F = [r * un, None, None, None, un * (E + p)]
    for d in range(3):
        F[1 + d] = r * un * vel[d] + (p if d == axis else 0.0)
    return np.stack(F)


@pytest.mark.parametrize("ndim,axis", [(2, 0), (2, 1), (3, 2)])
def test_outflow_faces_pass_physical_flux_of_edge_cell(ndim, axis):
    """Zero-gradient guards make both face states at an outflow face equal the
    edge cell, so the face flux is that cell's physical flux.  Over one tiny
    step the change of the totals is then dt times the net physical flux
    through the two outflow faces (the other axes are periodic)."""
    gamma = 1.4
    n = 12
    mesh = I.independent_blocks([n], ndim)
    mesh.dx[:] = np.where(np.arange(3) < ndim, 1.0 / n, 1.0)
    mesh.kind[0, 2 * axis:2 * axis + 2] = I.OUTFLOW
    U = I.random_smooth_state(mesh, 11, gamma)
    W = prims_of(mesh, U, gamma)[0]  # (5, nz, ny, nx)
    ax = 3 - axis  # numpy axis of the physical axis in (5, z, y, x)
    lo = np.take(W, 0, axis=ax)
    hi = np.take(W, n - 1, axis=ax)
    face_area = float(np.prod([mesh.dx[0, d] for d in range(ndim) if d != axis]))
    net = (_euler_flux(lo, gamma, axis) - _euler_flux(hi, gamma, axis)).reshape(5, -1).sum(axis=1) * face_area
    vol = float(np.prod(mesh.dx[0]))
    before = mesh.block_view(U, 0).reshape(5, -1).sum(axis=1) * vol
    dt = 1e-7
    O.step(mesh, U, dt, gamma)
    after = mesh.block_view(U, 0).reshape(5, -1).sum(axis=1) * vol
    change = after - before
    for v in range(5):
        assert abs(change[v] - dt * net[v]) <= 1e-4 * dt * (abs(net[v]) + 1e-3 * np.abs(net).max()) + 1e-13, v


# ------------------------------------------------------ errors and plumbing
def test_nonphysical_state_is_reported():
    gamma = 1.4
    mesh = I.block_grid((2, 1, 1), (4, 4, 4), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U = I.uniform_state(mesh, gamma=gamma)
    mesh.block_view(U, 1)[4, 1, 2, 3] = 0.0  # E < rho |v|^2 / 2  ->  p < 0
    with pytest.raises(O.OracleError) as e:
        O.max_lambda(mesh, U, gamma)
    assert e.value.code == O.ENONPHYS
    with pytest.raises(O.OracleError) as e:
        O.step(mesh, U, 1e-3, gamma)
    assert e.value.code == O.ENONPHYS


def test_invalid_meshes_rejected():
    good = I.block_grid((2, 1, 1), (4, 4, 4), (0, 0, 0), (1, 1, 1), "periodic", 3)
    assert O.validate(good) == O.OK
    bad = I.block_grid((2, 1, 1), (4, 4, 4), (0, 0, 0), (1, 1, 1), "periodic", 3)
    bad.nbr[0, 1] = 7
    assert O.validate(bad) == O.EINVAL
    bad = I.block_grid((2, 1, 1), (4, 4, 4), (0, 0, 0), (1, 1, 1), "periodic", 3)
    bad.n[1] = (4, 5, 4)  # face extents no longer match
    assert O.validate(bad) == O.EINVAL


def test_subset_step_equals_full_step():
    gamma = 1.4
    mesh = I.block_grid((3, 3, 3), (4, 4, 4), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U = I.random_smooth_state(mesh, 3, gamma)
    dt = O.dt(mesh, U, gamma, 0.4)
    full = U.copy()
    O.step(mesh, full, dt, gamma)
    targets = [0, 13, 26]
    sub = O.step_subset(mesh, U, dt, gamma, targets)
    for b in range(mesh.nblocks):
        want = full if b in targets else U
        assert np.array_equal(mesh.block_view(sub, b), mesh.block_view(want, b))


def test_result_independent_of_thread_count():
    gamma = 1.4
    mesh = I.block_grid((2, 2, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = I.random_smooth_state(mesh, 5, gamma)
    n0 = O.num_threads()
    try:
        outs = []
        for nt in (1, max(2, n0)):
            O.set_num_threads(nt)
            U = U0.copy()
            O.run(mesh, U, 3, 0.4, gamma)
            outs.append(U)
    finally:
        O.set_num_threads(n0)
    assert np.array_equal(outs[0], outs[1])
