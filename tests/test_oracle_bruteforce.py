"""Brute force on tiny meshes: one SSP-RK2 step recomputed here in 50-digit
arithmetic (mpmath), from the textbook statements of each step, and compared
with the FP64 oracle, which must agree to 1e-13 relative (floored per
variable at 1e-6 of its largest magnitude, as the GPU parity measure; the
FP64 rounding of the ~50 operations per value, amplified where the flux
differences cancel against a small momentum, reaches ~2e-14).  A variable
that is zero throughout (rho w in 2D) must stay exactly zero.

The high-precision step is written independently of the oracle: cell values
are fetched through the face rules directly (periodic wrap, outflow clamp,
neighbour's interior), primitives recovered per cell, minmod-limited PLM per
face, the four-branch HLLC of Toro (2009) sec. 10.4 with Davis bounds, the
flux differences summed over directions, and the SSP-RK2 combine.  Cases: a
4^3 self-periodic block (every guard a wrap), and two linked 2D blocks with
outflow faces (neighbour guards and edge copies).
"""
import numpy as np
from mpmath import mp, mpf, sqrt

from oracle import oracle as O
from paper_2507_09337_amd import inputs as I

mp.dps = 50


def mp_prim(U, g):
    r, mx, my, mz, E = U
    u, v, w = mx / r, my / r, mz / r
    return [r, u, v, w, (g - 1) * (E - (mx * u + my * v + mz * w) / 2)]


def mp_minmod(a, b):
    if a > 0 and b > 0:
        return min(a, b)
    if a < 0 and b < 0:
        return max(a, b)
    return mpf(0)


def mp_hllc(WL, WR, g):
    """Toro sec. 10.4 HLLC, Davis bounds; states (rho, u_n, u_t1, u_t2, p)."""
    def parts(W):
        r, u, v, w, p = W
        E = p / (g - 1) + r * (u * u + v * v + w * w) / 2
        return [r, r * u, r * v, r * w, E], [r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)]

    (rL, uL, vL, wL, pL), (rR, uR, vR, wR, pR) = WL, WR
    cL, cR = sqrt(g * pL / rL), sqrt(g * pR / rR)
    SL, SR = min(uL - cL, uR - cR), max(uL + cL, uR + cR)
    Sst = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))
    UL, FL = parts(WL)
    UR, FR = parts(WR)

    def star(W, U, S):
        r, u, v, w, p = W
        f = r * (S - u) / (S - Sst)
        return [f, f * Sst, f * v, f * w, f * (U[4] / r + (Sst - u) * (Sst + p / (r * (S - u))))]

    if SL >= 0:
        return FL
    if Sst >= 0:
        Us = star(WL, UL, SL)
        return [FL[k] + SL * (Us[k] - UL[k]) for k in range(5)]
    if SR > 0:
        Us = star(WR, UR, SR)
        return [FR[k] + SR * (Us[k] - UR[k]) for k in range(5)]
    return FR


class MPMesh:
    """Block values as mp numbers, fetched through the face rules."""

    def __init__(self, mesh, U):
        self.m = mesh
        self.vals = [[[[[mpf(float(x)) for x in row] for row in plane] for plane in var]
                      for var in mesh.block_view(U, b)] for b in range(mesh.nblocks)]

    def get(self, b, c):
        """Conserved values of cell c (i, j, k) of block b; at most one
        coordinate outside the block."""
        m = self.m
        n = [int(x) for x in m.n[b]]
        c = list(c)
        for d in range(3):
            if 0 <= c[d] < n[d]:
                continue
            f = 2 * d + (1 if c[d] >= n[d] else 0)
            kind = int(m.kind[b, f])
            if kind == I.PERIODIC_SELF:
                c[d] %= n[d]
            elif kind == I.OUTFLOW:
                c[d] = n[d] - 1 if c[d] >= n[d] else 0
            else:  # neighbour's interior
                s = int(m.nbr[b, f])
                c[d] = c[d] - n[d] if c[d] >= n[d] else int(m.n[s][d]) + c[d]
                return self.get(s, c)
        i, j, k = c
        return [self.vals[b][v][k][j][i] for v in range(5)]


def mp_L(mesh, mpm, g, dt):
    """dt * (flux differences) for every block, directions summed x, y, z."""
    out = []
    for b in range(mesh.nblocks):
        n = [int(x) for x in mesh.n[b]]
        dU = {}
        for d in range(mesh.ndim):
            dxd = mpf(float(mesh.dx[b, d]))
            flux = {}
            for k in range(n[2] + (d == 2)):
                for j in range(n[1] + (d == 1)):
                    for i in range(n[0] + (d == 0)):
                        cells = []
                        for s in (-2, -1, 0, 1):
                            c = [i, j, k]
                            c[d] += s
                            cells.append(mp_prim(mpm.get(b, c), g))
                        wl = [cells[1][v] + mp_minmod(cells[1][v] - cells[0][v], cells[2][v] - cells[1][v]) / 2
                              for v in range(5)]
                        wr = [cells[2][v] - mp_minmod(cells[2][v] - cells[1][v], cells[3][v] - cells[2][v]) / 2
                              for v in range(5)]
                        perm = [0, 1 + d] + [1 + t for t in range(3) if t != d] + [4]
                        F = mp_hllc([wl[p] for p in perm], [wr[p] for p in perm], g)
                        Fx = [None] * 5
                        for a, p in enumerate(perm):
                            Fx[p] = F[a]
                        flux[(i, j, k)] = Fx
            for k in range(n[2]):
                for j in range(n[1]):
                    for i in range(n[0]):
                        hi = [i, j, k]
                        hi[d] += 1
                        lo, up = flux[(i, j, k)], flux[tuple(hi)]
                        acc = dU.setdefault((i, j, k), [mpf(0)] * 5)
                        for v in range(5):
                            acc[v] += dt / dxd * (lo[v] - up[v])
        out.append(dU)
    return out


def mp_step(mesh, U, g, dt):
    dt = mpf(dt)
    mpn = MPMesh(mesh, U)
    L0 = mp_L(mesh, mpn, g, dt)
    mp1 = MPMesh(mesh, U)
    for b in range(mesh.nblocks):
        for (i, j, k), d in L0[b].items():
            for v in range(5):
                mp1.vals[b][v][k][j][i] = mpn.vals[b][v][k][j][i] + d[v]
    L1 = mp_L(mesh, mp1, g, dt)
    res = []
    for b in range(mesh.nblocks):
        n = [int(x) for x in mesh.n[b]]
        arr = np.zeros((5, n[2], n[1], n[0]))
        for (i, j, k), d in L1[b].items():
            for v in range(5):
                val = mpn.vals[b][v][k][j][i] / 2 + (mp1.vals[b][v][k][j][i] + d[v]) / 2
                arr[v, k, j, i] = float(val)
        res.append(arr)
    return res


def compare(mesh, U0, g, dt):
    ref = mp_step(mesh, U0, mpf(g), dt)
    U = U0.copy()
    O.step(mesh, U, dt, g)
    for v in range(5):
        scale = max(np.abs(r[v]).max() for r in ref)
        for b in range(mesh.nblocks):
            got = mesh.block_view(U, b)[v]
            if scale == 0.0:
                assert np.all(got == 0.0)
                continue
            err = np.abs(got - ref[b][v]) / np.maximum(np.abs(ref[b][v]), 1e-6 * scale)
            assert err.max() <= 1e-13, (b, v, err.max())


def mp_max_rate(mesh, U, g):
    """max over cells of sum_d (|u_d| + c)/dx_d."""
    mpm = MPMesh(mesh, U)
    lam = mpf(0)
    for b in range(mesh.nblocks):
        n = [int(x) for x in mesh.n[b]]
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    W = mp_prim(mpm.get(b, (i, j, k)), g)
                    c = sqrt(g * W[4] / W[0])
                    lam = max(lam, sum((abs(W[1 + d]) + c) / mpf(float(mesh.dx[b, d])) for d in range(mesh.ndim)))
    return lam


def test_periodic_4cube_one_step_in_50_digits():
    mesh = I.independent_blocks([4], 3)
    U0 = I.random_smooth_state(mesh, 61, 1.4)
    lam = O.max_lambda(mesh, U0, 1.4)
    assert abs(lam - float(mp_max_rate(mesh, U0, mpf(1.4)))) <= 1e-14 * lam
    compare(mesh, U0, 1.4, 0.4 / lam)


def test_linked_2d_blocks_with_outflow_in_50_digits():
    mesh = I.block_grid((2, 1, 1), (4, 4, 1), (0, 0, 0), (1, 0.5, 1), "outflow", 2)
    # link the two blocks along x (the outer x faces stay outflow)
    mesh.kind[0, 1] = mesh.kind[1, 0] = I.NBR
    mesh.nbr[0, 1], mesh.nbr[1, 0] = 1, 0
    prims = I.grid_field(mesh, lambda x, y, z: (1 + 0.3 * np.sin(5 * x + 2 * y), 0.5 * np.cos(3 * x), 0.2 * np.sin(4 * y),
                                                0 * x, 1 + 0.4 * np.cos(2 * x - 3 * y)))
    U0 = I.conserved_arena(mesh, prims, 1.4)
    dt = 0.4 / O.max_lambda(mesh, U0, 1.4)
    compare(mesh, U0, 1.4, dt)
