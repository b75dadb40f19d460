"""Pins of the Einfeldt wave-speed variant of the oracle's HLLC.

Einfeldt's bounds (Toro 2009, sec. 10.5.1) are u_bar -+ d_bar with u_bar the
sqrt(rho)-weighted mean normal velocity and d_bar^2 a sqrt(rho)-weighted mean
of c^2 plus a term in the normal-velocity jump.  They are pinned to the Roe
average of the enthalpy, a different route to the same number:
  * if every velocity component agrees on both sides, d_bar equals the Roe
    sound speed c~ = sqrt((gamma-1)(H~ - |v~|^2/2)), H~ the sqrt(rho)-weighted
    mean of H = (E + p)/rho (any gamma);
  * for gamma = 2 the identity also holds across a jump in the normal
    velocity (the jump term is exactly the Roe average's);
  * the mean of the bounds satisfies the Roe linearisation of the jump in
    rho u (which fixes the sqrt(rho) weights);
  * Galilean shift and mirror symmetry of the bounds;
and the HLLC flux built on them keeps the solver's exact properties
(consistency, stationary contact, supersonic upwinding).  The whole scheme
with these bounds keeps the uniform-state, conservation and mirror invariants
and converges to the exact Sod solution.
"""
import math

import numpy as np
import pytest

from oracle import exact_riemann as ER
from oracle import oracle as O
from paper_2507_09337_amd import inputs as I
from test_oracle_scheme import assemble, sod_mesh, sod_state

E = O.EINFELDT


def roe_sound_speed(WL, WR, gamma):
    """c~ from the sqrt(rho)-weighted averages of velocity and enthalpy."""
    def H(W):
        r, u, v, w, p = W
        return (p / (gamma - 1.0) + 0.5 * r * (u * u + v * v + w * w) + p) / r

    sL, sR = math.sqrt(WL[0]), math.sqrt(WR[0])
    avg = lambda a, b: (sL * a + sR * b) / (sL + sR)
    Ht = avg(H(WL), H(WR))
    q2 = sum(avg(WL[k], WR[k]) ** 2 for k in (1, 2, 3))
    return math.sqrt((gamma - 1.0) * (Ht - 0.5 * q2))


def random_pair(rng, same_normal, same_tangential):
    rL, rR = rng.uniform(0.05, 5.0, 2)
    pL, pR = rng.uniform(0.05, 5.0, 2)
    uL, uR = rng.normal(0, 2, 2)
    vL, vR, wL, wR = rng.normal(0, 1, 4)
    if same_normal:
        uR = uL
    if same_tangential:
        vR, wR = vL, wL
    return np.array([rL, uL, vL, wL, pL]), np.array([rR, uR, vR, wR, pR])


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0, 1.1])
def test_equal_velocities_give_roe_sound_speed(gamma):
    rng = np.random.default_rng(11)
    for _ in range(200):
        WL, WR = random_pair(rng, True, True)
        SL, SR = O.wave_speeds(WL, WR, gamma, E)
        c = roe_sound_speed(WL, WR, gamma)
        assert abs(0.5 * (SL + SR) - WL[1]) <= 1e-13 * (abs(WL[1]) + c)
        assert abs(0.5 * (SR - SL) - c) <= 1e-13 * c


def test_mean_velocity_is_the_roe_velocity():
    """(S_L + S_R)/2 satisfies the Roe linearisation of the mass-flux jump:
    rho_R u_R - rho_L u_L = u~ (rho_R - rho_L) + sqrt(rho_L rho_R) (u_R - u_L)."""
    rng = np.random.default_rng(15)
    for _ in range(200):
        WL, WR = random_pair(rng, False, False)
        SL, SR = O.wave_speeds(WL, WR, 1.4, E)
        ut = 0.5 * (SL + SR)
        lhs = WR[0] * WR[1] - WL[0] * WL[1]
        rhs = ut * (WR[0] - WL[0]) + math.sqrt(WL[0] * WR[0]) * (WR[1] - WL[1])
        scale = (WL[0] + WR[0]) * (abs(WL[1]) + abs(WR[1]) + abs(SL) + abs(SR))
        assert abs(lhs - rhs) <= 1e-13 * scale


def test_gamma_two_normal_jump_gives_roe_sound_speed():
    rng = np.random.default_rng(12)
    for _ in range(200):
        WL, WR = random_pair(rng, False, True)
        SL, SR = O.wave_speeds(WL, WR, 2.0, E)
        c = roe_sound_speed(WL, WR, 2.0)
        assert abs(0.5 * (SR - SL) - c) <= 1e-13 * c


def test_galilean_shift_and_mirror():
    rng = np.random.default_rng(13)
    for _ in range(100):
        WL, WR = random_pair(rng, False, False)
        SL, SR = O.wave_speeds(WL, WR, 1.4, E)
        V = rng.normal(0, 3)
        sh = np.array([0, V, 0, 0, 0])
        SL2, SR2 = O.wave_speeds(WL + sh, WR + sh, 1.4, E)
        scale = abs(SL) + abs(SR) + abs(V)
        assert abs(SL2 - (SL + V)) <= 1e-13 * scale and abs(SR2 - (SR + V)) <= 1e-13 * scale
        M = np.array([1, -1, 1, 1, 1])
        mL, mR = O.wave_speeds(WR * M, WL * M, 1.4, E)
        assert mL == -SR and mR == -SL
        # both bound choices give an ordered pair
        dL, dR = O.wave_speeds(WL, WR, 1.4, O.DAVIS)
        assert SL < SR and dL < dR


def euler_flux(W, gamma):
    r, u, v, w, p = W
    E_ = p / (gamma - 1.0) + 0.5 * r * (u * u + v * v + w * w)
    return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E_ + p)])


def check_hllc_exact_properties(E):
    """Consistency, stationary contact and supersonic upwinding of the HLLC
    flux with wave-speed option E."""
    rng = np.random.default_rng(14)
    g = 1.4
    for _ in range(100):
        W = np.array([rng.uniform(0.1, 3), rng.normal(0, 1), rng.normal(0, 1), rng.normal(0, 1), rng.uniform(0.1, 3)])
        F = O.hllc(W, W, g, E)
        ref = euler_flux(W, g)
        assert np.all(np.abs(F - ref) <= 1e-13 * (np.abs(ref) + np.abs(W).max()))
        # stationary contact: density jump at rest under equal pressure
        WL = np.array([rng.uniform(0.1, 3), 0.0, rng.normal(), rng.normal(), W[4]])
        WR = np.array([rng.uniform(0.1, 3), 0.0, rng.normal(), rng.normal(), W[4]])
        Fc = O.hllc(WL, WR, g, E)
        assert abs(Fc[0]) <= 1e-15 and abs(Fc[1] - W[4]) <= 1e-14 * W[4] and abs(Fc[4]) <= 1e-14 * W[4]
        # supersonic to the right: the flux is the left state's, bitwise
        c = math.sqrt(g * W[4] / W[0])
        WL = W.copy()
        WL[1] = 6.0 * c
        WR = WL.copy()
        WR[0] *= 1.5
        WR[4] *= 0.8
        assert O.wave_speeds(WL, WR, g, E)[0] >= 0.0
        assert np.array_equal(O.hllc(WL, WR, g, E), euler_flux(WL, g))


def test_hllc_with_einfeldt_speeds_exact_properties():
    check_hllc_exact_properties(E)


def run_to(mesh, U, t_end, gamma, speeds, cfl=0.4, recon=O.PRIMITIVE):
    t = 0.0
    while t < t_end:
        dt = min(O.dt(mesh, U, gamma, cfl), t_end - t)
        O.step(mesh, U, dt, gamma, speeds, recon)
        t += dt
    return t


def sod_l1(ncell, speeds, recon=O.PRIMITIVE):
    gamma = 1.4
    mesh = sod_mesh(ncell)
    U = sod_state(mesh, gamma)
    run_to(mesh, U, 0.2, gamma, speeds, recon=recon)
    rho = assemble(mesh, U, 0)[0]
    x = (np.arange(ncell) + 0.5) / ncell
    star = ER.star_state(1, 0, 1, 0.125, 0, 0.1, gamma)
    exact = np.array([ER.sample((xi - 0.5) / 0.2, 1, 0, 1, 0.125, 0, 0.1, gamma, star=star)[0] for xi in x])
    return float(np.abs(rho[0] - exact).sum() / ncell), U


def test_scheme_with_einfeldt_speeds_converges_on_sod():
    errs = [sod_l1(n, E)[0] for n in (64, 128, 256)]
    assert errs[0] <= 2e-2
    assert errs[0] / errs[1] >= 1.5 and errs[1] / errs[2] >= 1.5, errs
    # the variant reaches the step: it changes the result
    assert not np.array_equal(sod_l1(64, E)[1], sod_l1(64, O.DAVIS)[1])


def check_scheme_invariants(E, recon=O.PRIMITIVE, eos=O.IDEAL):
    """Uniform state, conservation and blast mirror symmetry of the whole
    scheme with wave-speed option E, reconstruction option recon and
    equation of state eos."""
    gamma = 1.4
    # uniform state: bitwise fixed point
    mesh = I.block_grid((2, 1, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = I.uniform_state(mesh, gamma=gamma)
    U = U0.copy()
    O.run(mesh, U, 4, 0.4, gamma, speeds=E, recon=recon, eos=eos)
    assert np.array_equal(U, U0)
    # conservation on a periodic mesh with a strong pulse
    mesh = I.block_grid((2, 2, 2), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U = I.random_smooth_state(mesh, 7, gamma)
    for b in range(mesh.nblocks):
        mesh.block_view(U, b)[4, 1:3, 2:4, 1:3] += 5.0
    vol = float(np.prod(mesh.dx[0]))
    t0 = [math.fsum(U.reshape(mesh.nblocks, 5, -1)[:, v].ravel()) * vol for v in range(5)]
    s0 = [math.fsum(np.abs(U.reshape(mesh.nblocks, 5, -1)[:, v].ravel())) * vol for v in range(5)]
    O.run(mesh, U, 10, 0.4, gamma, speeds=E, recon=recon, eos=eos)
    for v in range(5):
        t1 = math.fsum(U.reshape(mesh.nblocks, 5, -1)[:, v].ravel()) * vol
        assert abs(t1 - t0[v]) <= 1e-13 * s0[v] * 10
    # centred blast: mirror symmetry
    prims = I.grid_field(mesh, lambda x, y, z: (1.0, 0.0, 0.0, 0.0, 1e-3))
    I.sedov_deposit(mesh, prims, 1.0, 2.0, (0.5, 0.5, 0.5), gamma)
    U = I.conserved_arena(mesh, prims, gamma)
    O.run(mesh, U, 6, 0.4, gamma, speeds=E, recon=recon, eos=eos)
    for axis in range(3):
        ax = 2 - axis
        for v in range(5):
            ref = assemble(mesh, U, v)
            mir = np.flip(ref, axis=ax) * (-1.0 if v == 1 + axis else 1.0)
            assert np.abs(mir - ref).max() <= 1e-12 * np.abs(ref).max()


def test_scheme_with_einfeldt_speeds_invariants():
    check_scheme_invariants(E)


def test_unknown_speed_option_rejected():
    mesh = I.block_grid((1, 1, 1), (8, 8, 8), (0, 0, 0), (1, 1, 1), "periodic", 3)
    assert O.validate(mesh, 3) == O.EINVAL and O.validate(mesh, -1) == O.EINVAL
    for ok in (O.DAVIS, E, O.PVRS):
        assert O.validate(mesh, ok) == O.OK
