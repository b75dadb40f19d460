"""Pins of the exact Riemann solver (oracle/exact_riemann.py).

* Toro's printed star states for his five standard tests (tests/golden).
* The sampled solution satisfies the Rankine-Hugoniot jump conditions across
  every shock and the isentropic relation plus the Riemann invariant through
  every rarefaction fan; pressure and velocity are continuous at the contact.
"""
import json
import math
import os

import pytest

from oracle import exact_riemann as ER

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "toro_riemann_star.json")


def _tol(printed: str) -> float:
    """Half a unit in the last printed digit, plus 5e-6 relative: test 5 starts
    from the star states of tests 3 and 4 as printed to six digits, so its own
    star state is only defined to that input precision."""
    dec = len(printed.split(".")[1]) if "." in printed else 0
    return 0.5 * 10.0 ** (-dec) + 5e-6 * abs(float(printed)) + 1e-12


def _cases():
    g = json.load(open(GOLDEN))
    return [(g["gamma"], t) for t in g["tests"]]


@pytest.mark.parametrize("gamma,case", _cases(), ids=lambda c: str(c["id"]) if isinstance(c, dict) else "")
def test_star_state_matches_toro_table(gamma, case):
    s = ER.star_state(*case["left"], *case["right"], gamma)
    for attr, key in (("p", "p_star"), ("u", "u_star"), ("rho_l", "rho_star_l"), ("rho_r", "rho_star_r")):
        printed = case[key]
        assert abs(getattr(s, attr) - float(printed)) <= _tol(printed), (attr, getattr(s, attr), printed)


def _cons_flux(rho, u, p, gamma):
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return (rho, rho * u, E), (rho * u, rho * u * u + p, u * (E + p))


@pytest.mark.parametrize("gamma,case", _cases(), ids=lambda c: str(c["id"]) if isinstance(c, dict) else "")
def test_jump_conditions_of_sampled_solution(gamma, case):
    L, R = case["left"], case["right"]
    s = ER.star_state(*L, *R, gamma)
    speeds = ER.wave_speeds(*L, *R, gamma)
    for side, (rho, u, p), rho_star in (("l", L, s.rho_l), ("r", R, s.rho_r)):
        if side + "_shock" in speeds:
            S = speeds[side + "_shock"]
            Ua, Fa = _cons_flux(rho, u, p, gamma)
            Ub, Fb = _cons_flux(rho_star, s.u, s.p, gamma)
            for q in range(3):  # F_b - F_a = S (U_b - U_a)
                scale = max(abs(Fa[q]), abs(Fb[q]), abs(S * Ua[q]), 1.0)
                assert abs((Fb[q] - Fa[q]) - S * (Ub[q] - Ua[q])) <= 1e-9 * scale
        else:
            # isentropic: p / rho^gamma constant; Riemann invariant u -/+ 2c/(gamma-1) constant
            assert abs(s.p / rho_star**gamma - p / rho**gamma) <= 1e-9 * p / rho**gamma
            sign = 1.0 if side == "l" else -1.0
            c, cs = math.sqrt(gamma * p / rho), math.sqrt(gamma * s.p / rho_star)
            assert abs((u + sign * 2 * c / (gamma - 1)) - (s.u + sign * 2 * cs / (gamma - 1))) <= 1e-9 * (1 + abs(u) + c)
            # the sampled fan keeps both along the whole fan
            head, tail = speeds[side + "_head"], speeds[side + "_tail"]
            for a in (0.1, 0.5, 0.9):
                xi = head + a * (tail - head)
                rf, uf, pf = ER.sample(xi, *L, *R, gamma, star=s)
                cf = math.sqrt(gamma * pf / rf)
                assert abs(pf / rf**gamma - p / rho**gamma) <= 1e-9 * p / rho**gamma
                assert abs(uf + sign * 2 * cf / (gamma - 1) - (u + sign * 2 * c / (gamma - 1))) <= 1e-9 * (1 + abs(u) + c)
                # characteristic of the fan: xi = u -/+ c inside a left/right fan
                assert abs(xi - (uf - sign * cf)) <= 1e-9 * (1 + abs(xi))
    # contact: pressure and velocity continuous, density jumps rho*_L -> rho*_R
    eps = 1e-9 * (1 + abs(s.u))
    left_c = ER.sample(s.u - eps, *L, *R, gamma, star=s)
    right_c = ER.sample(s.u + eps, *L, *R, gamma, star=s)
    assert left_c[2] == pytest.approx(right_c[2], rel=1e-12) and left_c[1] == pytest.approx(right_c[1], rel=1e-12)
    assert left_c[0] == pytest.approx(s.rho_l, rel=1e-12) and right_c[0] == pytest.approx(s.rho_r, rel=1e-12)


def test_far_field_is_initial_data():
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    assert ER.sample(-10.0, *L, *R, 1.4) == pytest.approx(L)
    assert ER.sample(10.0, *L, *R, 1.4) == pytest.approx(R)
