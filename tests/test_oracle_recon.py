"""Pins of the conserved-variable reconstruction variant of the oracle.

With this option PLM (minmod) runs on (rho, rho u, rho v, rho w, E) and the
two face states are recovered to primitives afterwards (van Leer's MUSCL on
the conserved variables); a non-physical face state is an error, as a
non-physical cell is.  Pinned without re-typing the formulas:
  * linear conserved data: both face states are the primitive state of the
    conserved midpoint value (exact for a linear profile);
  * a conserved extremum: that variable's slope is 0, the others are the
    linear midpoint values;
  * strong velocity shear at low pressure: the conserved face energy keeps
    the cell's value while the face momentum is interpolated, so the face
    pressure goes negative -- the classic failure of conserved
    reconstruction -- and the step reports it; primitive reconstruction
    keeps the face pressure positive on the same data;
  * advection of a density wave at uniform velocity and pressure: rho u and
    E are affine in rho, so the face states keep u and p and the scheme
    reproduces primitive reconstruction to rounding, and converges at better
    than first order;
  * the scheme keeps uniform states bitwise, conserves, keeps blast mirror
    symmetry and converges on Sod; the option reaches the step.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2507_09337_amd import inputs as I
from test_oracle_einfeldt import check_scheme_invariants, sod_l1
from test_oracle_scheme import assemble, field_state, prims_of

CONS = O.CONSERVED


def prim_of(U, g):
    r, m, E = U[0], U[1:4], U[4]
    return np.array([r, *(m / r), (g - 1.0) * (E - 0.5 * float(m @ m) / r)])


def random_state(rng):
    r = rng.uniform(0.5, 2.0)
    vel = rng.normal(0, 1, 3)
    p = rng.uniform(0.5, 2.0)
    return np.array([r, *(r * vel), p / 0.4 + 0.5 * r * float(vel @ vel)])


def test_linear_conserved_data_gives_midpoint_states():
    rng = np.random.default_rng(31)
    for _ in range(100):
        # cells on the segment from a towards b: convex combinations of two
        # physical states, so every cell and the midpoint are physical
        a = random_state(rng)
        d = 0.2 * (random_state(rng) - a)
        u4 = np.array([a + s * d for s in range(4)])
        wl, wr = O.face_states(u4, 1.4, CONS)
        ref = prim_of(a + 1.5 * d, 1.4)
        scale = np.abs(ref) + np.abs(ref).max()
        assert np.all(np.abs(wl - ref) <= 1e-14 * scale) and np.all(np.abs(wr - ref) <= 1e-14 * scale)
        # primitive reconstruction of the same cells differs (W is not linear in U)
        pl, pr = O.face_states(u4, 1.4, O.PRIMITIVE)
        assert not np.allclose(pl, wl, rtol=1e-10, atol=0)


def test_conserved_extremum_has_zero_slope():
    rng = np.random.default_rng(32)
    for _ in range(100):
        a = random_state(rng)
        d = 0.1 * (random_state(rng) - a)
        u4 = np.array([a + s * d for s in range(4)])
        u4[1, 4] += 0.5 * abs(a[4])  # energy maximum at cell 1
        wl, _ = O.face_states(u4, 1.4, CONS)
        mid = a + 1.5 * d
        uL = np.array([mid[0], mid[1], mid[2], mid[3], u4[1, 4]])  # left state: E of cell 1 itself
        ref = prim_of(uL, 1.4)
        assert np.all(np.abs(wl - ref) <= 1e-14 * (np.abs(ref) + np.abs(ref).max()))


def test_shear_at_low_pressure_gives_non_physical_face_state():
    # rho = 1, u = 10 (s - 1), p = 0.1: at the face between cells 1 and 2 the
    # momentum is interpolated to 5 while E keeps E_1 (an energy minimum), so
    # the face pressure is (gamma - 1)(0.25 - 12.5) < 0
    g = 1.4
    u4 = np.array([[1.0, 10.0 * (s - 1), 0, 0, 0.1 / (g - 1) + 50.0 * (s - 1) ** 2] for s in range(4)])
    assert O.face_states(u4, g, CONS) is None
    wl, wr = O.face_states(u4, g, O.PRIMITIVE)
    assert wl[4] > 0 and wr[4] > 0
    mesh = I.block_grid((1, 1, 1), (16, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    for recon, ok in ((O.PRIMITIVE, True), (CONS, False)):
        U = field_state(mesh, lambda x, y, z: (1.0 + 0 * x, 10 * np.sin(2 * np.pi * x), 0 * x, 0 * x, 0.01 + 0 * x), g)
        try:
            O.step(mesh, U, 1e-4, g, O.DAVIS, recon)
            assert ok
        except O.OracleError as e:
            assert not ok and e.code == O.ENONPHYS


def advect(ncell, recon, t_end=0.25):
    gamma = 1.4
    mesh = I.block_grid((ncell // 16, 1, 1), (16, 2, 1), (0, 0, 0), (1, 2.0 / ncell, 1), "periodic", 2)
    U = field_state(mesh, lambda x, y, z: (1 + 0.1 * np.sin(2 * np.pi * x), 1.0 + 0 * x, 0.0, 0.0, 1.0 + 0 * x), gamma)
    t = 0.0
    while t < t_end:
        dt = min(O.dt(mesh, U, gamma, 0.4), t_end - t)
        O.step(mesh, U, dt, gamma, O.DAVIS, recon)
        t += dt
    return mesh, U


def test_advected_density_wave_matches_primitive_reconstruction():
    res = {}
    for recon in (O.PRIMITIVE, CONS):
        mesh, U = advect(64, recon)
        res[recon] = U
    a, b = res[O.PRIMITIVE], res[CONS]
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    W = prims_of(mesh, b, 1.4)
    assert max(np.abs(w[1] - 1.0).max() for w in W) <= 1e-12
    assert max(np.abs(w[4] - 1.0).max() for w in W) <= 1e-12
    # and the scheme converges at better than first order on it
    errs = []
    for n in (32, 64, 128):
        mesh, U = advect(n, CONS)
        rho = assemble(mesh, U, 0)[0, 0]
        x = (np.arange(n) + 0.5) / n
        exact = 1 + 0.1 * (np.cos(2 * np.pi * (x - 0.5 / n - 0.25)) - np.cos(2 * np.pi * (x + 0.5 / n - 0.25))) \
            / (2 * np.pi / n)
        errs.append(float(np.abs(rho - exact).mean()))
    assert min(math.log2(errs[i] / errs[i + 1]) for i in range(2)) >= 1.5, errs


def test_scheme_with_conserved_reconstruction_converges_on_sod():
    errs = [sod_l1(n, O.DAVIS, CONS)[0] for n in (64, 128, 256)]
    assert errs[0] <= 2e-2
    assert errs[0] / errs[1] >= 1.5 and errs[1] / errs[2] >= 1.5, errs
    # the option reaches the step: it changes the result
    assert not np.array_equal(sod_l1(64, O.DAVIS, CONS)[1], sod_l1(64, O.DAVIS)[1])


def test_scheme_with_conserved_reconstruction_invariants():
    check_scheme_invariants(O.DAVIS, CONS)


def test_unknown_reconstruction_rejected():
    mesh = I.block_grid((1, 1, 1), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    assert O.validate(mesh, O.DAVIS, 2) == O.EINVAL and O.validate(mesh, O.DAVIS, -1) == O.EINVAL
    assert O.validate(mesh, O.PVRS, CONS) == O.OK
