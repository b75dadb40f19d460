"""Pins of the oracle's pointwise functions against properties fixed by the
mathematics of each method (not by retyping the oracle's formulas).

minmod (Roe 1986)      -- closed-form cases, symmetry, magnitude/sign bounds.
PLM (van Leer 1979)    -- exact on linear data, first order at extrema.
HLLC (Toro 2009 ch.10) -- consistency F(W, W) = physical flux; exact upwinding
                          of supersonic states; exact resolution of stationary
                          and moving contacts; mirror symmetry; and the contact
                          structure of the star state recovered from the flux:
                          F = S* U* + p* (0, 1, 0, 0, S*) with tangential
                          velocity preserved.
Recovery (ideal gas)   -- inverse of the input generator's conserved form.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09337_amd import inputs

RNG = np.random.default_rng(12345)


@pytest.fixture(autouse=True)
def _reseed(request):
    """Each test draws from its own seeded stream, whatever the test order."""
    global RNG
    RNG = np.random.default_rng(sum(map(ord, request.node.name)))


def euler_flux(W, gamma):
    """Physical Euler flux along the first velocity component, from its definition."""
    r, u, v, w, p = W
    E = p / (gamma - 1) + 0.5 * r * (u * u + v * v + w * w)
    return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])


def cons(W, gamma):
    r, u, v, w, p = W
    return np.array([r, r * u, r * v, r * w, p / (gamma - 1) + 0.5 * r * (u * u + v * v + w * w)])


def rand_state(subsonic=True):
    r = RNG.uniform(0.1, 3.0)
    p = RNG.uniform(0.05, 5.0)
    vel = RNG.uniform(-0.5, 0.5, 3) if subsonic else RNG.uniform(-5, 5, 3)
    return np.array([r, vel[0], vel[1], vel[2], p])


# ------------------------------------------------------------------ minmod
@pytest.mark.parametrize(
    "a,b,want",
    [(1.0, 2.0, 1.0), (2.0, 1.0, 1.0), (-1.0, -3.0, -1.0), (-3.0, -1.0, -1.0), (1.0, -1.0, 0.0),
     (-2.0, 5.0, 0.0), (0.0, 3.0, 0.0), (3.0, 0.0, 0.0), (0.0, -0.0, 0.0), (2.5, 2.5, 2.5), (-1e-300, -1e-300, -1e-300)],
)
def test_minmod_cases(a, b, want):
    assert O.minmod(a, b) == want


def test_minmod_properties():
    for _ in range(2000):
        a, b = RNG.normal(size=2) * 10.0 ** RNG.integers(-20, 20, size=2)
        m = O.minmod(a, b)
        assert m == O.minmod(b, a)
        assert abs(m) <= min(abs(a), abs(b))
        if a * b > 0:
            assert m in (a, b) and np.sign(m) == np.sign(a)
        else:
            assert m == 0.0
    # no product is formed: tiny same-sign slopes whose product underflows still give a slope
    assert O.minmod(1e-200, 2e-200) == 1e-200


# --------------------------------------------------------------------- PLM
def test_plm_exact_on_linear_data():
    for _ in range(100):
        base = RNG.normal(size=5)
        slope = RNG.normal(size=5)
        w = np.array([base + slope * s for s in range(4)])
        wl, wr = O.plm_face(w)
        face = base + slope * 1.5  # the face between cells 1 and 2
        assert np.allclose(wl, face, rtol=0, atol=1e-12)
        assert np.allclose(wr, face, rtol=0, atol=1e-12)


def test_plm_constant_and_extremum():
    w = np.tile(np.array([1.0, 0.2, -0.3, 0.4, 2.0]), (4, 1))
    wl, wr = O.plm_face(w)
    assert np.array_equal(wl, w[1]) and np.array_equal(wr, w[2])
    # a local maximum at cell 1 and a local minimum at cell 2: both slopes limited to zero
    w = np.array([[0.0] * 5, [1.0] * 5, [0.5] * 5, [2.0] * 5])
    wl, wr = O.plm_face(w)
    assert np.array_equal(wl, w[1]) and np.array_equal(wr, w[2])


def test_plm_face_values_bounded_by_neighbours():
    """With minmod, both face states at a face lie between the two cells that
    share it (no new extrema; |slope| <= the jump across the face)."""
    for _ in range(2000):
        w = RNG.normal(size=(4, 5))
        wl, wr = O.plm_face(w)
        lo = np.minimum(w[1], w[2])
        hi = np.maximum(w[1], w[2])
        assert np.all((wl >= lo) & (wl <= hi)) and np.all((wr >= lo) & (wr <= hi))


# -------------------------------------------------------------------- HLLC
@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_hllc_consistency(gamma):
    for _ in range(300):
        W = rand_state(subsonic=bool(RNG.integers(2)))
        F = O.hllc(W, W, gamma)
        ref = euler_flux(W, gamma)
        assert np.allclose(F, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_hllc_supersonic_upwinding(gamma):
    for _ in range(200):
        WL, WR = rand_state(), rand_state()
        cmax = max(math.sqrt(gamma * WL[4] / WL[0]), math.sqrt(gamma * WR[4] / WR[0]))
        shift = 1.5 * cmax + 1.0
        WL[1] += shift
        WR[1] += shift
        assert np.array_equal(O.hllc(WL, WR, gamma), euler_flux(WL, gamma))
        WL[1] -= 2 * shift
        WR[1] -= 2 * shift
        assert np.array_equal(O.hllc(WL, WR, gamma), euler_flux(WR, gamma))


def test_hllc_stationary_contact():
    gamma = 1.4
    for _ in range(200):
        p = RNG.uniform(0.1, 3)
        WL = np.array([RNG.uniform(0.1, 3), 0.0, RNG.normal(), RNG.normal(), p])
        WR = np.array([RNG.uniform(0.1, 3), 0.0, RNG.normal(), RNG.normal(), p])
        F = O.hllc(WL, WR, gamma)
        assert abs(F[0]) <= 1e-14 * WL[0]
        assert F[1] == pytest.approx(p, rel=1e-14)
        assert abs(F[4]) <= 1e-13 * p


def test_hllc_moving_contact_is_upwind():
    """A contact moving at u with equal pressure is resolved exactly: the flux is
    the physical flux of the upwind state."""
    gamma = 1.4
    for _ in range(200):
        u, p = RNG.uniform(-0.8, 0.8), RNG.uniform(0.1, 3)
        WL = np.array([RNG.uniform(0.1, 3), u, RNG.normal(), RNG.normal(), p])
        WR = np.array([RNG.uniform(0.1, 3), u, RNG.normal(), RNG.normal(), p])
        F = O.hllc(WL, WR, gamma)
        ref = euler_flux(WL if u > 0 else WR, gamma)
        assert np.allclose(F, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_hllc_mirror_symmetry():
    """Reflecting the problem (swap sides, negate the normal velocity) negates
    every flux component except the normal momentum flux."""
    gamma = 1.4
    M = np.array([1.0, -1.0, 1.0, 1.0, 1.0])
    S = np.array([-1.0, 1.0, -1.0, -1.0, -1.0])
    for _ in range(500):
        WL, WR = rand_state(bool(RNG.integers(2))), rand_state(bool(RNG.integers(2)))
        F = O.hllc(WL, WR, gamma)
        G = O.hllc(M * WR, M * WL, gamma)
        assert np.allclose(G, S * F, rtol=1e-12, atol=1e-12 * np.abs(F).max())


def test_hllc_star_state_contact_structure():
    """HLLC's middle wave is a contact at speed S* with one star pressure p* on
    both sides: p* = p_K + rho_K (S_K - u_K)(S* - u_K) for K = L and K = R
    (Toro 2009 eq. 10.36), which fixes S* as the root of a linear equation.
    Taking that S*, the side K it selects, and U*_K recovered from the flux
    through the outer wave's jump relation F = F_K + S_K (U*_K - U_K), the
    star state must move with S*, carry side K's tangential velocities, and
    the flux must have the contact form F = S* U*_K + p* (0, 1, 0, 0, S*)."""
    gamma = 1.4
    checked = 0
    for _ in range(2000):
        WL, WR = rand_state(), rand_state()
        cL, cR = math.sqrt(gamma * WL[4] / WL[0]), math.sqrt(gamma * WR[4] / WR[0])
        SL = min(WL[1] - cL, WR[1] - cR)  # Davis bounds
        SR = max(WL[1] + cL, WR[1] + cR)
        if not (SL < 0.0 < SR):  # a supersonic pair has no star state at the face
            continue
        checked += 1
        # p_L + aL (S - u_L) = p_R + aR (S - u_R), a_K = rho_K (S_K - u_K)
        aL, aR = WL[0] * (SL - WL[1]), WR[0] * (SR - WR[1])
        s_star = (WR[4] - WL[4] + aL * WL[1] - aR * WR[1]) / (aL - aR)
        W, S = (WL, SL) if s_star >= 0 else (WR, SR)
        p_star = W[4] + W[0] * (S - W[1]) * (s_star - W[1])
        F = O.hllc(WL, WR, gamma)
        Us = cons(W, gamma) + (F - euler_flux(W, gamma)) / S
        scale = np.abs(cons(W, gamma)).max() + np.abs(euler_flux(W, gamma)).max()
        assert Us[1] / Us[0] == pytest.approx(s_star, rel=1e-10, abs=1e-12)
        assert Us[2] / Us[0] == pytest.approx(W[2], rel=1e-10, abs=1e-12)
        assert Us[3] / Us[0] == pytest.approx(W[3], rel=1e-10, abs=1e-12)
        want = s_star * Us + p_star * np.array([0.0, 1.0, 0.0, 0.0, s_star])
        assert np.allclose(F, want, rtol=1e-10, atol=1e-11 * scale)
    assert checked >= 1500


# ---------------------------------------------------------------- recovery
@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_recovery_inverts_generator(gamma):
    mesh = inputs.independent_blocks([4], 3)
    prims = [np.stack([RNG.uniform(0.1, 2, (4, 4, 4)), RNG.normal(size=(4, 4, 4)), RNG.normal(size=(4, 4, 4)),
                       RNG.normal(size=(4, 4, 4)), RNG.uniform(0.1, 2, (4, 4, 4))])]
    U = inputs.conserved_arena(mesh, prims, gamma)
    blk = mesh.block_view(U, 0).reshape(5, -1)
    ref = prims[0].reshape(5, -1)
    for c in range(blk.shape[1]):
        W = O.prim(blk[:, c], gamma)
        assert np.allclose(W, ref[:, c], rtol=1e-12, atol=1e-12)
