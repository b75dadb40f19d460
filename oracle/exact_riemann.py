"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

TEST INFRASTRUCTURE: used only to pin the oracle (Sod shock tube), never by the
product path.

The paper's Sedov application uses the ideal-gas gamma-law equation of state
(Sec. 5.2).  The exact Riemann solution for that EOS is the textbook one
(Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", 3rd ed.,
ch. 4): the star pressure p* is the root of

    f(p) = f_L(p, W_L) + f_R(p, W_R) + (u_R - u_L) = 0,

with, for K in {L, R},

    shock (p > p_K):        f_K = (p - p_K) sqrt(A_K / (p + B_K)),
                            A_K = 2 / ((gamma+1) rho_K),  B_K = p_K (gamma-1)/(gamma+1)
    rarefaction (p <= p_K): f_K = 2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1),

and u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.  The solution is self-similar
in x/t; `sample` evaluates it at a given x/t.  Plain Python floats, Newton
iteration with a bisection safeguard.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class StarState:
    p: float
    u: float
    rho_l: float
    rho_r: float


def _f_k(p: float, rho: float, pk: float, gamma: float) -> tuple[float, float]:
    """Pressure function f_K and its derivative (shock or rarefaction branch)."""
    ck = math.sqrt(gamma * pk / rho)
    if p > pk:
        a = 2.0 / ((gamma + 1.0) * rho)
        b = pk * (gamma - 1.0) / (gamma + 1.0)
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (b + p))
    ratio = p / pk
    f = 2.0 * ck / (gamma - 1.0) * (ratio ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rho * ck) * ratio ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma) -> StarState:
    """Star-region pressure, velocity and the densities either side of the contact."""
    c_l = math.sqrt(gamma * p_l / rho_l)
    c_r = math.sqrt(gamma * p_r / rho_r)
    if 2.0 * (c_l + c_r) / (gamma - 1.0) <= u_r - u_l:
        raise ValueError("initial data generate vacuum")

    def g(p):
        fl, dfl = _f_k(p, rho_l, p_l, gamma)
        fr, dfr = _f_k(p, rho_r, p_r, gamma)
        return fl + fr + (u_r - u_l), dfl + dfr

    # bracket: g is monotone increasing in p
    lo, hi = 1e-300, max(p_l, p_r)
    while g(hi)[0] < 0.0:
        hi *= 2.0
    # two-rarefaction guess, clipped into the bracket
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((c_l + c_r - 0.5 * (gamma - 1.0) * (u_r - u_l)) / (c_l / p_l**z + c_r / p_r**z)) ** (1.0 / z)
    p = min(max(p, lo), hi)
    for _ in range(200):
        val, dval = g(p)
        if val > 0.0:
            hi = p
        else:
            lo = p
        p_new = p - val / dval
        if not (lo < p_new < hi):
            p_new = 0.5 * (lo + hi)
        if abs(p_new - p) <= 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _f_k(p, rho_l, p_l, gamma)
    fr, _ = _f_k(p, rho_r, p_r, gamma)
    u = 0.5 * (u_l + u_r) + 0.5 * (fr - fl)
    return StarState(p, u, _star_rho(p, rho_l, p_l, gamma), _star_rho(p, rho_r, p_r, gamma))


def _star_rho(p: float, rho: float, pk: float, gamma: float) -> float:
    if p > pk:  # shock: Rankine-Hugoniot density ratio
        r = p / pk
        g1 = (gamma - 1.0) / (gamma + 1.0)
        return rho * (r + g1) / (g1 * r + 1.0)
    return rho * (p / pk) ** (1.0 / gamma)  # rarefaction: isentropic


def wave_speeds(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma) -> dict:
    """Shock speeds or rarefaction head/tail speeds of the left and right waves."""
    s = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    out = {}
    for side, rho, u, pk, sign in (("l", rho_l, u_l, p_l, -1.0), ("r", rho_r, u_r, p_r, 1.0)):
        c = math.sqrt(gamma * pk / rho)
        if s.p > pk:
            out[side + "_shock"] = u + sign * c * math.sqrt(
                (gamma + 1.0) / (2.0 * gamma) * s.p / pk + (gamma - 1.0) / (2.0 * gamma)
            )
        else:
            rho_star = s.rho_l if side == "l" else s.rho_r
            c_star = math.sqrt(gamma * s.p / rho_star)
            out[side + "_head"] = u + sign * c
            out[side + "_tail"] = s.u + sign * c_star
    return out


def sample(xi: float, rho_l, u_l, p_l, rho_r, u_r, p_r, gamma, star: StarState | None = None):
    """(rho, u, p) of the exact solution at similarity coordinate xi = x/t."""
    s = star or star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    if xi <= s.u:  # left of the contact
        rho, u, pk, sign, rho_star = rho_l, u_l, p_l, -1.0, s.rho_l
    else:
        rho, u, pk, sign, rho_star = rho_r, u_r, p_r, 1.0, s.rho_r
    c = math.sqrt(gamma * pk / rho)
    # mirror the right-going wave onto the left-going formulas via sign
    if s.p > pk:  # shock
        shock = u + sign * c * math.sqrt((gamma + 1.0) / (2.0 * gamma) * s.p / pk + (gamma - 1.0) / (2.0 * gamma))
        if sign * (xi - shock) >= 0.0:
            return rho, u, pk
        return rho_star, s.u, s.p
    head = u + sign * c
    c_star = math.sqrt(gamma * s.p / rho_star)
    tail = s.u + sign * c_star
    if sign * (xi - head) >= 0.0:
        return rho, u, pk
    if sign * (xi - tail) <= 0.0:
        return rho_star, s.u, s.p
    # inside the fan
    g = gamma
    uf = 2.0 / (g + 1.0) * (-sign * c + 0.5 * (g - 1.0) * u + xi)
    cf = 2.0 / (g + 1.0) * (c - sign * 0.5 * (g - 1.0) * (u - xi))
    rhof = rho * (cf / c) ** (2.0 / (g - 1.0))
    pf = pk * (cf / c) ** (2.0 * g / (g - 1.0))
    return rhof, uf, pf
