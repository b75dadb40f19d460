"""Pins of the pressure-based (PVRS) wave-speed variant of the oracle's HLLC.

Toro (2009, sec. 10.5.2) bounds the waves with S_L = u_L - c_L q_L and
S_R = u_R + c_R q_R: q_K = 1 where the star pressure p* does not exceed p_K
(the wave is a rarefaction and its head moves at the acoustic speed) and
otherwise the factor that turns c_K into the speed of a shock of pressure
p*; p* comes from the primitive-variable (PVRS) linearisation about the
arithmetic means rho_bar, c_bar, clipped at zero.  The pins reach the same
numbers by other routes:
  * p* is the star pressure of the linear acoustic Riemann problem of the
    primitive-variable Euler system frozen at (rho_bar, c_bar), solved here by
    an eigen-decomposition of that Jacobian (numpy);
  * the shock speed for a given p* follows from the Rankine-Hugoniot
    conditions (mass and momentum flux through the shock, with the shock
    Hugoniot density ratio), not from the closed form of q_K;
  * in separating flow both bounds are the acoustic speeds u -+ c exactly;
  * Galilean shift and mirror symmetry; small jumps approach the exact
    solver's wave speeds at second order;
and the flux and the whole scheme keep the exact properties and invariants of
the other wave-speed options and converge on Sod.
"""
import math

import numpy as np
import pytest

from oracle import exact_riemann as ER
from oracle import oracle as O
from test_oracle_einfeldt import check_hllc_exact_properties, check_scheme_invariants, random_pair, sod_l1

P = O.PVRS


def sound(W, g):
    return math.sqrt(g * W[4] / W[0])


def linear_star_pressure(WL, WR, g):
    """Star pressure of the linearised Riemann problem: the 1D primitive
    system W_t + A W_x = 0 for W = (rho, u, p) with A frozen at rho_bar, c_bar
    (the arithmetic means of the two sides), solved by eigenvectors:
    W* = W_L + (the jump carried by the left-moving eigenvector)."""
    rb = 0.5 * (WL[0] + WR[0])
    cb = 0.5 * (sound(WL, g) + sound(WR, g))
    ub = 0.5 * (WL[1] + WR[1])
    A = np.array([[ub, rb, 0.0], [0.0, ub, 1.0 / rb], [0.0, rb * cb * cb, ub]])
    lam, R = np.linalg.eig(A)
    order = np.argsort(lam.real)
    R = R[:, order].real
    dW = np.array([WR[0] - WL[0], WR[1] - WL[1], WR[4] - WL[4]])
    alpha = np.linalg.solve(R, dW)
    star = np.array([WL[0], WL[1], WL[4]]) + alpha[0] * R[:, 0]
    return max(0.0, float(star[2]))


def shock_speed(W, ps, g, sign):
    """Speed of the shock that raises the pressure of the still state W to ps,
    moving into W in direction `sign` (-1 left, +1 right): the Hugoniot
    density ratio rho*/rho = (ps/p + mu)/(mu ps/p + 1), mu = (g-1)/(g+1), and
    the mass flux m through the shock from the momentum jump,
    m^2 (1/rho - 1/rho*) = ps - p."""
    mu = (g - 1.0) / (g + 1.0)
    ratio = ps / W[4]
    rs = W[0] * (ratio + mu) / (mu * ratio + 1.0)
    m = math.sqrt((ps - W[4]) / (1.0 / W[0] - 1.0 / rs))
    return W[1] + sign * m / W[0]


def rh_condition(W, ps):
    """Error amplification of the Rankine-Hugoniot route for a weak shock:
    (ps - p) and (1/rho - 1/rho*) cancel as ps -> p."""
    return 1.0 + W[4] / (ps - W[4])


def expected_bounds(WL, WR, g):
    """Expected (S_L, S_R) and the conditioning of each."""
    ps = linear_star_pressure(WL, WR, g)
    out, cond = [], []
    for W, sign in ((WL, -1.0), (WR, 1.0)):
        if ps > W[4] * (1.0 + 1e-9):
            out.append(shock_speed(W, ps, g, sign))
            cond.append(rh_condition(W, ps))
        else:
            out.append(W[1] + sign * sound(W, g))
            cond.append(1.0)
    return out, cond


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0, 1.1])
def test_bounds_follow_linear_star_pressure_and_rankine_hugoniot(g):
    rng = np.random.default_rng(21)
    nshock = 0
    for _ in range(400):
        WL, WR = random_pair(rng, False, False)
        SL, SR = O.wave_speeds(WL, WR, g, P)
        (eL, eR), (kL, kR) = expected_bounds(WL, WR, g)
        scale = abs(WL[1]) + abs(WR[1]) + sound(WL, g) + sound(WR, g)
        ps = linear_star_pressure(WL, WR, g)
        nshock += (ps > WL[4]) + (ps > WR[4])
        assert abs(SL - eL) <= 1e-13 * kL * scale and abs(SR - eR) <= 1e-13 * kR * scale
    assert 200 <= nshock <= 600  # both branches exercised


def test_separating_flow_gives_acoustic_speeds():
    rng = np.random.default_rng(22)
    for _ in range(200):
        WL, WR = random_pair(rng, False, False)
        WL[1] = -abs(WL[1]) - 3.0
        WR[1] = abs(WR[1]) + 3.0  # strong expansion: the linear p* is negative, clipped to 0
        SL, SR = O.wave_speeds(WL, WR, 1.4, P)
        assert SL == WL[1] - sound(WL, 1.4) and SR == WR[1] + sound(WR, 1.4)


def test_equal_velocities_shock_side_from_rankine_hugoniot():
    """u_L = u_R: p* is the mean pressure; the higher-pressure side moves at
    its acoustic speed and the other bound is the Rankine-Hugoniot speed."""
    rng = np.random.default_rng(23)
    for _ in range(200):
        WL, WR = random_pair(rng, True, False)
        SL, SR = O.wave_speeds(WL, WR, 1.4, P)
        ps = 0.5 * (WL[4] + WR[4])
        scale = abs(WL[1]) + sound(WL, 1.4) + sound(WR, 1.4)
        if WL[4] > WR[4]:
            assert SL == WL[1] - sound(WL, 1.4)
            assert abs(SR - shock_speed(WR, ps, 1.4, 1.0)) <= 1e-14 * rh_condition(WR, ps) * scale
        else:
            assert abs(SL - shock_speed(WL, ps, 1.4, -1.0)) <= 1e-14 * rh_condition(WL, ps) * scale
            assert SR == WR[1] + sound(WR, 1.4)


def test_small_jumps_approach_exact_wave_speeds_at_second_order():
    """A weak collision: both exact waves are shocks; the bounds differ from
    the exact shock speeds by O(eps^2)."""
    g = 1.4
    errs = []
    for eps in (4e-2, 2e-2, 1e-2):
        WL = np.array([1.0 + 0.5 * eps, 0.3 + eps, 0.0, 0.0, 1.0 + 0.2 * eps])
        WR = np.array([1.0 - 0.3 * eps, 0.3 - eps, 0.0, 0.0, 1.0 - 0.1 * eps])
        ex = ER.wave_speeds(WL[0], WL[1], WL[4], WR[0], WR[1], WR[4], g)
        SL, SR = O.wave_speeds(WL, WR, g, P)
        errs.append(max(abs(SL - ex["l_shock"]), abs(SR - ex["r_shock"])))
    assert errs[0] / errs[1] >= 3.0 and errs[1] / errs[2] >= 3.0, errs


def test_galilean_shift_and_mirror():
    rng = np.random.default_rng(24)
    for _ in range(100):
        WL, WR = random_pair(rng, False, False)
        SL, SR = O.wave_speeds(WL, WR, 1.4, P)
        V = rng.normal(0, 3)
        sh = np.array([0, V, 0, 0, 0])
        SL2, SR2 = O.wave_speeds(WL + sh, WR + sh, 1.4, P)
        scale = abs(SL) + abs(SR) + abs(V)
        assert abs(SL2 - (SL + V)) <= 1e-13 * scale and abs(SR2 - (SR + V)) <= 1e-13 * scale
        M = np.array([1, -1, 1, 1, 1])
        mL, mR = O.wave_speeds(WR * M, WL * M, 1.4, P)
        assert mL == -SR and mR == -SL


def test_bounds_ordered_unless_strong_collision():
    """The linear p* grows like the velocity jump while a strong shock's
    pressure grows like its square, so in a strong collision the bounds can
    cross (S_L > S_R); below that they are ordered."""
    rng = np.random.default_rng(25)
    for _ in range(200):
        WL, WR = random_pair(rng, False, False)
        if WL[1] - WR[1] < 0.5 * min(sound(WL, 1.4), sound(WR, 1.4)):
            SL, SR = O.wave_speeds(WL, WR, 1.4, P)
            assert SL < SR
    WL = np.array([1.0, 20.0, 0, 0, 1.0])
    WR = np.array([1.0, -20.0, 0, 0, 1.0])
    SL, SR = O.wave_speeds(WL, WR, 1.4, P)
    assert SL > SR


def test_hllc_with_pvrs_speeds_exact_properties():
    check_hllc_exact_properties(P)


def test_scheme_with_pvrs_speeds_converges_on_sod():
    errs = [sod_l1(n, P)[0] for n in (64, 128, 256)]
    assert errs[0] <= 2e-2
    assert errs[0] / errs[1] >= 1.5 and errs[1] / errs[2] >= 1.5, errs
    # the option reaches the step: it changes the result
    a = sod_l1(64, P)[1]
    assert not np.array_equal(a, sod_l1(64, O.DAVIS)[1]) and not np.array_equal(a, sod_l1(64, O.EINFELDT)[1])


def test_scheme_with_pvrs_speeds_invariants():
    check_scheme_invariants(P)
