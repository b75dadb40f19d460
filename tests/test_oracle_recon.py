"""Pins of the reconstruction variants of the oracle: PLM on the conserved
variables, and PLM on the characteristic variables.

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

Characteristic reconstruction limits, per cell, the amplitudes of the
one-sided differences on the waves of the primitive system along the face
normal (u - c, entropy, two shear waves, u + c) and maps the limited
amplitudes back.  Pinned through an eigen-decomposition of the primitive
Jacobian built here and solved with numpy (acoustic eigenvectors from
numpy.linalg.eig, the three-fold eigenvalue u spanned by the density-only
and tangential-velocity vectors; minmod is odd-homogeneous, so the scaling
of the eigenvectors does not matter), in every direction; linear data and a
contact at rest reduce to primitive reconstruction; an acoustic extremum
keeps a slope that primitive reconstruction clips.
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
    assert O.validate(mesh, O.DAVIS, 3) == O.EINVAL and O.validate(mesh, O.DAVIS, -1) == O.EINVAL
    assert O.validate(mesh, O.PVRS, CONS) == O.OK and O.validate(mesh, O.EINFELDT, O.CHARACTERISTIC) == O.OK


# ------------------------------------------------------ characteristic PLM
CHAR = O.CHARACTERISTIC


def cons_of(W, g):
    r, vel, p = W[0], np.asarray(W[1:4]), W[4]
    return np.array([r, *(r * vel), p / (g - 1.0) + 0.5 * r * float(vel @ vel)])


def minmod(a, b):
    return np.where((a > 0) & (b > 0), np.minimum(a, b), np.where((a < 0) & (b < 0), np.maximum(a, b), 0.0))


def eig_slope(W, da, db, g, direction):
    """Limited characteristic slope of cell W from an eigen-decomposition of
    the primitive Jacobian along `direction`, computed with numpy."""
    n = 1 + direction
    r, un, p = W[0], W[n], W[4]
    c2 = g * p / r
    # (rho, u_n, p) block of the Jacobian; the tangential velocities are
    # advected (eigenvalue u_n)
    A = np.array([[un, r, 0.0], [0.0, un, 1.0 / r], [0.0, r * c2, un]])
    lam, V = np.linalg.eig(A)
    order = np.argsort(lam.real)
    V = V[:, order].real  # columns: u - c, u (entropy), u + c
    R = np.zeros((5, 5))
    idx = [0, n, 4]
    tang = [k for k in (1, 2, 3) if k != n]
    R[idx, 0] = V[:, 0]               # acoustic waves from numpy
    R[idx, 4] = V[:, 2]
    R[0, 1] = 1.0                     # entropy wave: density only
    R[tang[0], 2] = 1.0               # shear waves
    R[tang[1], 3] = 1.0
    a = np.linalg.solve(R, da)
    b = np.linalg.solve(R, db)
    return R @ minmod(a, b)


def random_prims(rng):
    return np.array([rng.uniform(0.5, 2.0), *rng.normal(0, 1, 3), rng.uniform(0.5, 2.0)])


def test_characteristic_slopes_match_eigen_decomposition():
    rng = np.random.default_rng(41)
    g = 1.4
    checked = 0
    for _ in range(300):
        direction = int(rng.integers(0, 3))
        base = random_prims(rng)
        W = [base + 0.15 * rng.normal(0, 1, 5) for _ in range(4)]
        if min(w[0] for w in W) <= 0.1 or min(w[4] for w in W) <= 0.1:
            continue
        u4 = np.array([cons_of(w, g) for w in W])
        res = O.face_states(u4, g, CHAR, direction)
        Wr = [O.prim(u, g) for u in u4]  # the oracle's own recovered cells
        s1 = eig_slope(Wr[1], Wr[1] - Wr[0], Wr[2] - Wr[1], g, direction)
        s2 = eig_slope(Wr[2], Wr[2] - Wr[1], Wr[3] - Wr[2], g, direction)
        el, er = Wr[1] + 0.5 * s1, Wr[2] - 0.5 * s2
        if min(el[0], el[4], er[0], er[4]) <= 0:
            assert res is None
            continue
        wl, wr = res
        scale = np.abs(np.concatenate([w for w in Wr])).max()
        assert np.abs(wl - el).max() <= 1e-13 * scale and np.abs(wr - er).max() <= 1e-13 * scale
        checked += 1
    assert checked >= 150


def test_characteristic_equals_primitive_on_linear_data_and_contacts():
    rng = np.random.default_rng(42)
    g = 1.4
    for _ in range(100):
        base = random_prims(rng)
        d = 0.05 * rng.normal(0, 1, 5)
        u4 = np.array([cons_of(base + s * d, g) for s in range(4)])
        direction = int(rng.integers(0, 3))
        cl, cr = O.face_states(u4, g, CHAR, direction)
        pl, pr = O.face_states(u4, g, O.PRIMITIVE, direction)
        # the recovered cells are linear only to rounding: compare to it
        scale = np.abs(base).max()
        assert np.abs(cl - pl).max() <= 1e-12 * scale and np.abs(cr - pr).max() <= 1e-12 * scale
    # contact at rest: density jumps, u and p uniform -> only the entropy wave
    W = [np.array([r, 0.3, -0.2, 0.1, 1.0]) for r in (1.0, 1.0, 0.125, 0.125)]
    u4 = np.array([cons_of(w, g) for w in W])
    for direction in range(3):
        cl, cr = O.face_states(u4, g, CHAR, direction)
        pl, pr = O.face_states(u4, g, O.PRIMITIVE, direction)
        assert np.abs(cl - pl).max() <= 1e-15 and np.abs(cr - pr).max() <= 1e-15


def test_characteristic_keeps_acoustic_slope_at_pressure_extremum():
    """A right-going acoustic wave plus a left-going one of opposite
    curvature: the pressure has an extremum at cell 1, so primitive PLM clips
    the pressure slope to 0, while both acoustic amplitudes keep a slope of
    one sign; here rho = 1, c = 1 and the limited slopes are computed by hand:
    d_lo = (du, dp) = (0.1, 0.05), d_hi = (0.1, -0.05) give amplitudes
    a_+ = (0.075, 0.025), a_- = (-0.025, -0.075), limited 0.025 and -0.025,
    so du = (c/rho)(0.025 + 0.025) = 0.05 and dp = 0."""
    g = 1.4
    p1 = 1.0 / g  # c = sqrt(g p / rho) = 1
    W1 = np.array([1.0, 0.0, 0.0, 0.0, p1])
    W0 = W1 - np.array([0.05, 0.1, 0, 0, 0.05])  # d_rho = d_p / c^2: no entropy wave
    W2 = W1 + np.array([-0.05, 0.1, 0, 0, -0.05])
    W3 = W2 + (W2 - W1)
    u4 = np.array([cons_of(w, g) for w in (W0, W1, W2, W3)])
    Wr = [O.prim(u, g) for u in u4]
    wl, _ = O.face_states(u4, g, CHAR, 0)
    pl, _ = O.face_states(u4, g, O.PRIMITIVE, 0)
    assert abs(pl[1] - (Wr[1][1] + 0.05)) <= 1e-12 and abs(pl[4] - Wr[1][4]) <= 1e-12
    assert abs(wl[1] - (Wr[1][1] + 0.025)) <= 1e-12 and abs(wl[4] - Wr[1][4]) <= 1e-12


def test_scheme_with_characteristic_reconstruction():
    # Sod: converges, and the option reaches the step
    errs = [sod_l1(n, O.DAVIS, CHAR)[0] for n in (64, 128, 256)]
    assert errs[0] <= 2e-2
    assert errs[0] / errs[1] >= 1.5 and errs[1] / errs[2] >= 1.5, errs
    assert not np.array_equal(sod_l1(64, O.DAVIS, CHAR)[1], sod_l1(64, O.DAVIS)[1])
    # advection at uniform u, p: only the entropy wave, so primitive PLM to rounding
    a = advect(64, O.PRIMITIVE)[1]
    b = advect(64, CHAR)[1]
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    check_scheme_invariants(O.DAVIS, CHAR)

