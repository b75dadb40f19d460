"""Pins of the gas + radiation equation of state of the oracle (a method
variant standing in for a heavier, iterated EOS).

Model, in units with gas and radiation constants 1: p = rho T + T^4/3 and
rho e = rho T/(gamma - 1) + T^4; sound speed from the first adiabatic
exponent of the mixture.  Pinned by other routes:
  * both temperature solves invert the defining relations to rounding over
    eight decades of rho and T (the forward relations are the definition of
    the model; the oracle's work is the inverse);
  * limits: with negligible radiation the EOS is the gamma-law gas (p,
    sound speed, the whole step within rounding); with negligible gas the
    pressure is a third of the energy density and Gamma1 = 4/3;
  * Gamma1 is the logarithmic slope of p along an adiabat, found here by
    integrating the first law de = (p / rho^2) d rho (s fixed) with RK4 and
    differencing -- thermodynamics, not the closed form;
  * the HLLC flux keeps consistency, the stationary contact and upwinding;
  * the scheme keeps uniform states bitwise, conserves, keeps blast mirror
    symmetry and self-converges on Sod; the option reaches the step.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09337_amd import inputs as I
from test_oracle_einfeldt import check_scheme_invariants, euler_flux
from test_oracle_scheme import assemble, sod_mesh, sod_state

GR = O.GAS_RADIATION


def cons(rho, vel, rhoe):
    vel = np.asarray(vel, dtype=float)
    return np.array([rho, *(rho * vel), rhoe + 0.5 * rho * float(vel @ vel)])


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_temperature_solves_invert_the_definition(g):
    rng = np.random.default_rng(51)
    for _ in range(3000):
        rho = 10 ** rng.uniform(-4, 4)
        T = 10 ** rng.uniform(-4, 4)
        rhoe = rho * T / (g - 1) + T ** 4
        p = rho * T + T ** 4 / 3
        assert abs(O.gr_temperature_e(rho, rhoe, g) - T) <= 4e-15 * T
        assert abs(O.gr_temperature_p(rho, p) - T) <= 4e-15 * T
        W = O.prim_eos(cons(rho, (0.3, -0.2, 0.1), rhoe), g, GR)
        cond = 1.0 + 0.5 * rho * 0.14 / rhoe  # E - rho |v|^2 / 2 cancels when the kinetic part dominates
        assert abs(W[4] - p) <= 1e-14 * cond * p
        c, e = O.thermo(W, g, GR)
        assert abs(e - rhoe) <= 1e-14 * cond * rhoe


def test_limits_gas_and_radiation():
    g = 1.4
    # gas dominated: T = 1e-3, rho = 1e3 -> radiation share ~ 1e-15
    W = np.array([1e3, 0.2, 0.0, 0.0, 1.0])
    c, e = O.thermo(W, g, GR)
    ci, ei = O.thermo(W, g, O.IDEAL)
    assert abs(c - ci) <= 1e-12 * ci and abs(e - ei) <= 1e-12 * ei
    # radiation dominated: rho = 1e-6, T ~ 10 -> gas share ~ 1e-10
    rho, T = 1e-6, 10.0
    p = rho * T + T ** 4 / 3
    c, e = O.thermo(np.array([rho, 0, 0, 0, p]), g, GR)
    assert abs(p - e / 3) <= 1e-8 * p
    assert abs(c * c * rho / p - 4.0 / 3.0) <= 1e-8


def test_gamma1_is_the_adiabatic_slope():
    """d ln p / d ln rho at fixed entropy, from the first law integrated with
    RK4 (de/drho = p / rho^2 for the specific energy e) in both directions."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(52)

    def p_of(rho, e_spec):
        return O.prim_eos(cons(rho, (0, 0, 0), rho * e_spec), g, GR)[4]

    def adiabat(rho0, e0, rho1, n=20):
        h = (rho1 - rho0) / n
        rho, e = rho0, e0
        f = lambda r, s: p_of(r, s) / (r * r)
        for _ in range(n):
            k1 = f(rho, e)
            k2 = f(rho + h / 2, e + h / 2 * k1)
            k3 = f(rho + h / 2, e + h / 2 * k2)
            k4 = f(rho + h, e + h * k3)
            e += h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            rho += h
        return e

    for _ in range(20):
        rho = 10 ** rng.uniform(-2, 2)
        T = 10 ** rng.uniform(-1, 1) * rho ** (1 / 3)  # straddle beta ~ 1/2
        e0 = (rho * T / (g - 1) + T ** 4) / rho
        eps = 1e-4
        rp, rm = rho * (1 + eps), rho * (1 - eps)
        pp, pm = p_of(rp, adiabat(rho, e0, rp)), p_of(rm, adiabat(rho, e0, rm))
        g1_num = (math.log(pp) - math.log(pm)) / (math.log(rp) - math.log(rm))
        p = rho * T + T ** 4 / 3
        c, _ = O.thermo(np.array([rho, 0, 0, 0, p]), g, GR)
        assert abs(c * c * rho / p - g1_num) <= 1e-7, (rho, T)


def test_hllc_with_gas_radiation_exact_properties():
    g = 1.4
    rng = np.random.default_rng(53)
    for _ in range(100):
        W = np.array([rng.uniform(0.1, 3), rng.normal(), rng.normal(), rng.normal(), rng.uniform(0.1, 3)])
        c, rhoe = O.thermo(W, g, GR)
        r, u, v, w, p = W
        E = rhoe + 0.5 * r * (u * u + v * v + w * w)
        ref = np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])
        F = O.hllc(W, W, g, O.DAVIS, GR)
        assert np.all(np.abs(F - ref) <= 1e-13 * (np.abs(ref) + np.abs(W).max()))
        # the gamma-law flux differs (the energy differs): the option reaches HLLC
        assert not np.allclose(F, euler_flux(W, g), rtol=1e-9, atol=0)
        WL = np.array([rng.uniform(0.1, 3), 0.0, rng.normal(), rng.normal(), p])
        WR = np.array([rng.uniform(0.1, 3), 0.0, rng.normal(), rng.normal(), p])
        Fc = O.hllc(WL, WR, g, O.DAVIS, GR)
        assert abs(Fc[0]) <= 1e-15 and abs(Fc[1] - p) <= 1e-14 * p and abs(Fc[4]) <= 1e-14 * p
        WL = W.copy()
        WL[1] = 6.0 * c
        WR = WL.copy()
        WR[0] *= 1.5
        WR[4] *= 0.8
        FL = O.hllc(WL, WR, g, O.DAVIS, GR)
        _, eL = O.thermo(WL, g, GR)
        EL = eL + 0.5 * WL[0] * float(WL[1:4] @ WL[1:4])
        refL = np.array([WL[0] * WL[1], WL[0] * WL[1] ** 2 + WL[4], WL[0] * WL[1] * WL[2], WL[0] * WL[1] * WL[3],
                         WL[1] * (EL + WL[4])])
        assert np.allclose(FL, refL, rtol=1e-14, atol=0)


def test_gas_dominated_step_is_the_gamma_law_step():
    """rho ~ 1e4 and p ~ 1: radiation pressure ~ 1e-17 of the total, so one
    step with either EOS agrees to rounding."""
    mesh = I.block_grid((2, 1, 1), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    prims = I.grid_field(mesh, lambda x, y, z: (1e4 * (1 + 0.1 * np.sin(2 * np.pi * x)), 0.01 + 0 * x, 0 * x,
                                                0 * x, 1.0 + 0.1 * np.cos(2 * np.pi * x)))
    U = I.conserved_arena(mesh, prims, 1.4)
    a, b = U.copy(), U.copy()
    O.step(mesh, a, 1e-3, 1.4)
    O.step(mesh, b, 1e-3, 1.4, eos=GR)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_scheme_with_gas_radiation():
    g = 1.4
    # Sod with the mixture: self-convergence (no exact solution here)
    def sod(n):
        mesh = sod_mesh(n)
        U = sod_state(mesh, g)
        t = 0.0
        while t < 0.2:
            dt = min(O.dt(mesh, U, g, 0.4, GR), 0.2 - t)
            O.step(mesh, U, dt, g, eos=GR)
            t += dt
        return assemble(mesh, U, 0)[0].ravel()

    r64, r128, r256 = sod(64), sod(128), sod(256)
    c = lambda fine: fine.reshape(-1, 2).mean(axis=1)
    d1 = np.abs(r64 - c(r128)).mean()
    d2 = np.abs(r128 - c(r256)).mean()
    assert d1 / d2 >= 1.5, (d1, d2)
    # the option reaches the step: the gamma-law density profile differs
    assert np.abs(r64 - assemble(*sod_ideal(64), 0)[0].ravel()).max() > 1e-3
    check_scheme_invariants(O.DAVIS, O.PRIMITIVE, eos=GR)


def sod_ideal(n):
    g = 1.4
    mesh = sod_mesh(n)
    U = sod_state(mesh, g)
    t = 0.0
    while t < 0.2:
        dt = min(O.dt(mesh, U, g, 0.4), 0.2 - t)
        O.step(mesh, U, dt, g)
        t += dt
    return mesh, U


def test_step_assembles_from_the_pointwise_pieces():
    """One SSP-RK2 step of a y-uniform, x-periodic 2D row with the mixture,
    rebuilt here from the pinned pointwise functions (EOS recovery, PLM,
    HLLC with the EOS, the flux differences in the oracle's order); the y
    fluxes cancel exactly.  Also the CFL rate against (|u| + c)/dx +
    (|v| + c)/dy with the EOS sound speed."""
    g, n = 1.4, 16
    mesh = I.block_grid((1, 1, 1), (n, 8, 1), (0, 0, 0), (1, 0.5, 1), "periodic", 2)
    x = (np.arange(n) + 0.5) / n
    rng = np.random.default_rng(54)
    row = np.stack([1 + 0.3 * np.sin(2 * np.pi * x + rng.uniform(0, 6)), 0.4 * np.cos(2 * np.pi * x),
                    0.2 + 0 * x, 0 * x, 2 + np.sin(4 * np.pi * x)])
    Ucells = np.array([cons(row[0, i], row[1:4, i], row[4, i]) for i in range(n)])  # (n, 5), rho e given

    def arena_of(Uc):
        arena = np.zeros(mesh.arena_len)
        view = mesh.block_view(arena, 0)
        for v in range(5):
            view[v, 0] = np.repeat(Uc[:, v][None], 8, axis=0)
        return arena

    arena = arena_of(Ucells)
    dt, dx = 2e-3, 1.0 / n

    def L(U):
        W = np.array([O.prim_eos(U[i], g, GR) for i in range(n)])
        F = np.zeros((n + 1, 5))
        for f in range(n + 1):  # face f between cells f-1 and f
            w4 = np.array([W[(f + k) % n] for k in (-2, -1, 0, 1)])
            wl, wr = O.plm_face(w4)
            F[f] = O.hllc(wl, wr, g, O.DAVIS, GR)
        return F

    def stage(src, un, k):
        F = L(src)
        out = np.empty_like(src)
        for i in range(n):
            d = (dt / dx) * (F[i] - F[i + 1])
            out[i] = src[i] + d if k == 1 else 0.5 * un[i] + 0.5 * (src[i] + d)
        return out

    U1 = stage(Ucells, Ucells, 1)
    U2 = stage(U1, Ucells, 2)
    O.step(mesh, arena, dt, g, eos=GR)
    got = mesh.block_view(arena, 0)[:, 0]  # (5, 8, n)
    for j in range(8):
        assert np.abs(got[:, j, :].T - U2).max() <= 1e-15 * np.abs(U2).max()
    # CFL rate
    W = [O.prim_eos(Ucells[i], g, GR) for i in range(n)]
    lam = max((abs(w[1]) + O.thermo(w, g, GR)[0]) / dx + (abs(w[2]) + O.thermo(w, g, GR)[0]) / (0.5 / 8)
              for w in W)
    assert abs(O.max_lambda(mesh, arena_of(Ucells), g, GR) - lam) <= 1e-14 * lam


def test_eos_option_validation():
    mesh = I.block_grid((1, 1, 1), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    assert O.validate(mesh, eos=GR) == O.OK
    assert O.validate(mesh, eos=2) == O.EINVAL
    # the variants of the wave speeds and of the reconstruction assume the gamma law
    assert O.validate(mesh, O.PVRS, eos=GR) == O.EINVAL
    assert O.validate(mesh, O.DAVIS, O.CONSERVED, eos=GR) == O.EINVAL
