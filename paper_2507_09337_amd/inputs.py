"""Seeded synthetic inputs: block meshes, initial conserved states and packets.

This module is the only code that both the HIP path's tests/benchmark and the
FP64 oracle consume.  It holds no arithmetic of the solver (no primitive
recovery, reconstruction, Riemann solver, update or time-step rule); it only
lays out blocks and writes initial conditions.  Initial conditions are point
values at cell centres; the conserved total energy of an initial state is
written from its specified density, velocity and pressure with the ideal-gas
definition E = p/(gamma-1) + rho |v|^2 / 2, which is part of the problem
statement, not of the method.

Mesh model (Sec. 5.1 of the paper: the domain is decomposed into blocks that
all have the same number of equally sized cells; Sec. 4.3: a data packet
concatenates n blocks, n chosen at run time):

* ``BlockMesh``: per block the interior extent n[3] (n[2] == 1 in 2D), the
  cell widths dx[3], the kind of each of the six faces (-x,+x,-y,+y,-z,+z) and
  the linked neighbour block of ``NBR`` faces, and the element offset of the
  block in the state arena.
* Arena layout: block b, variable v (rho, rho*u, rho*v, rho*w, E), interior
  cell (i, j, k) lives at ``offset[b] + v*nx*ny*nz + (k*ny + j)*nx + i``.

Workloads (sizes from the benchmark configurations; readings of unstated
details are listed in the design notes):

* ``sod2d``         -- 2D Sod tube, 4x2 blocks of 16^2 on [0,1]x[0,0.5], outflow.
* ``sedov3d``       -- 3D Sedov-like blast, 8^3 blocks of 16^3, periodic.
* ``smooth3d``      -- 3D smooth random flow, 16^3 blocks of 16^3, periodic.
* ``uneven``        -- 6000 self-periodic blocks of 8^3/16^3/32^3.
* ``sedov_noise``   -- 32^3 blocks of 16^3, Sedov deposit + 1 % density noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NVAR = 5
NBR, OUTFLOW, PERIODIC_SELF = 0, 1, 2


@dataclass
class BlockMesh:
    ndim: int
    n: np.ndarray  # (nb, 3) int32
    dx: np.ndarray  # (nb, 3) float64
    kind: np.ndarray  # (nb, 6) int32
    nbr: np.ndarray  # (nb, 6) int32
    offset: np.ndarray  # (nb,) int64
    origin: np.ndarray  # (nb, 3) float64, lower corner of each block
    grid: tuple | None = None  # (nbx, nby, nbz) for uniform block grids
    meta: dict = field(default_factory=dict)

    @property
    def nblocks(self) -> int:
        return int(self.n.shape[0])

    @property
    def ncells(self) -> np.ndarray:
        return self.n.prod(axis=1).astype(np.int64)

    @property
    def total_cells(self) -> int:
        return int(self.ncells.sum())

    @property
    def arena_len(self) -> int:
        return int((self.offset + NVAR * self.ncells).max()) if self.nblocks else 0

    def block_view(self, U: np.ndarray, b: int) -> np.ndarray:
        """(5, nz, ny, nx) view of block b inside an arena array."""
        nx, ny, nz = (int(v) for v in self.n[b])
        o = int(self.offset[b])
        return U[o : o + NVAR * nx * ny * nz].reshape(NVAR, nz, ny, nx)

    def cell_centres(self, b: int):
        """(x, y, z) arrays of shape (nz, ny, nx) for block b."""
        nx, ny, nz = (int(v) for v in self.n[b])
        x0 = self.origin[b]
        d = self.dx[b]
        z, y, x = np.meshgrid(
            x0[2] + (np.arange(nz) + 0.5) * d[2],
            x0[1] + (np.arange(ny) + 0.5) * d[1],
            x0[0] + (np.arange(nx) + 0.5) * d[0],
            indexing="ij",
        )
        return x, y, z

    def subset(self, ids) -> "BlockMesh":
        """Mesh of the listed blocks only (links to blocks outside the list
        become self-periodic); arena offsets are repacked contiguously."""
        ids = np.asarray(ids, dtype=np.int64)
        remap = -np.ones(self.nblocks, dtype=np.int64)
        remap[ids] = np.arange(ids.size)
        kind = self.kind[ids].copy()
        nbr = self.nbr[ids].copy()
        for f in range(6):
            linked = kind[:, f] == NBR
            tgt = remap[np.where(linked, nbr[:, f], 0)]
            lost = linked & (tgt < 0)
            kind[lost, f] = PERIODIC_SELF
            nbr[:, f] = np.where(linked & ~lost, tgt, -1)
        n = self.n[ids].copy()
        sizes = NVAR * n.prod(axis=1).astype(np.int64)
        offset = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        return BlockMesh(self.ndim, n, self.dx[ids].copy(), kind.astype(np.int32), nbr.astype(np.int32), offset,
                         self.origin[ids].copy(), None, dict(self.meta))

    def gather(self, U: np.ndarray, ids) -> np.ndarray:
        """Arena of the listed blocks (layout of ``subset(ids)``)."""
        return np.concatenate([self.block_view(U, int(b)).ravel() for b in ids]) if len(ids) else np.zeros(0)


def _contiguous_offsets(n: np.ndarray) -> np.ndarray:
    sizes = NVAR * n.prod(axis=1).astype(np.int64)
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)


def block_grid(nblk, ncell, lo, hi, bc: str, ndim: int) -> BlockMesh:
    """Uniform grid of nblk = (nbx, nby, nbz) blocks, each ncell = (nx, ny, nz)
    interior cells, covering the box [lo, hi].  bc: 'periodic' links the
    outer faces around the domain; 'outflow' marks them zero-gradient.
    Blocks are numbered lexicographically, x fastest."""
    nbx, nby, nbz = nblk
    if ndim == 2:
        assert nbz == 1 and ncell[2] == 1
    nb = nbx * nby * nbz
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    dx = (hi - lo) / (np.asarray(nblk) * np.asarray(ncell))
    n = np.tile(np.asarray(ncell, dtype=np.int32), (nb, 1))
    kind = np.full((nb, 6), NBR, dtype=np.int32)
    nbr = np.full((nb, 6), -1, dtype=np.int32)
    origin = np.zeros((nb, 3))
    dims = (nbx, nby, nbz)
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                b = (bz * nby + by) * nbx + bx
                c = [bx, by, bz]
                origin[b] = lo + np.asarray(c) * np.asarray(ncell) * dx
                for axis in range(3):
                    for side in range(2):
                        f = 2 * axis + side
                        if axis >= ndim:
                            kind[b, f], nbr[b, f] = OUTFLOW, -1
                            continue
                        cc = list(c)
                        cc[axis] += 1 if side else -1
                        inside = 0 <= cc[axis] < dims[axis]
                        if not inside and bc == "outflow":
                            kind[b, f], nbr[b, f] = OUTFLOW, -1
                            continue
                        cc[axis] %= dims[axis]
                        kind[b, f] = NBR
                        nbr[b, f] = (cc[2] * nby + cc[1]) * nbx + cc[0]
    dxs = np.tile(np.where(np.arange(3) < ndim, dx, 1.0), (nb, 1))
    if ndim == 2:
        dxs[:, 2] = 1.0
    return BlockMesh(ndim, n, dxs, kind, nbr, _contiguous_offsets(n), origin, (nbx, nby, nbz))


def independent_blocks(sizes, ndim: int = 3) -> BlockMesh:
    """One self-periodic block per entry of `sizes` (edge length), each on its
    own unit cube (dx = 1/n)."""
    sizes = np.asarray(sizes, dtype=np.int32)
    nb = sizes.size
    n = np.stack([sizes, sizes, sizes if ndim == 3 else np.ones_like(sizes)], axis=1).astype(np.int32)
    dx = 1.0 / n.astype(np.float64)
    if ndim == 2:
        dx[:, 2] = 1.0
    kind = np.full((nb, 6), PERIODIC_SELF, dtype=np.int32)
    if ndim == 2:
        kind[:, 4:] = OUTFLOW
    nbr = np.full((nb, 6), -1, dtype=np.int32)
    return BlockMesh(ndim, n, dx, kind, nbr, _contiguous_offsets(n), np.zeros((nb, 3)), None)


def grid_field(mesh: BlockMesh, f) -> np.ndarray:
    """Evaluate f(x, y, z) -> (rho, u, v, w, p) per block and return the
    primitive fields block by block as a list of (5, nz, ny, nx) arrays."""
    out = []
    for b in range(mesh.nblocks):
        x, y, z = mesh.cell_centres(b)
        out.append(np.stack([np.broadcast_to(a, x.shape) for a in f(x, y, z)]).astype(np.float64))
    return out


def conserved_arena(mesh: BlockMesh, prims, gamma: float) -> np.ndarray:
    """Arena of conserved variables from per-block primitive fields (rho, u, v,
    w, p): rho, rho*u, rho*v, rho*w, E = p/(gamma-1) + rho|v|^2/2."""
    U = np.empty(mesh.arena_len, dtype=np.float64)
    for b, w in enumerate(prims):
        blk = mesh.block_view(U, b)
        rho, u, v, ww, p = w
        blk[0] = rho
        blk[1] = rho * u
        blk[2] = rho * v
        blk[3] = rho * ww
        blk[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + ww * ww)
    return U


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    mesh: BlockMesh
    U0: np.ndarray
    gamma: float
    cfl: float
    nsteps: int
    packets: list  # list of int arrays of block ids
    meta: dict = field(default_factory=dict)


def sod2d(nblk=(4, 2, 1), n=16, nsteps=20) -> Problem:
    """2D Sod shock tube on [0,1]x[0,0.5]: rho,p = 1,1 for x < 0.5 else
    0.125,0.1, at rest; outflow on every outer face; gamma 1.4; CFL 0.4."""
    gamma = 1.4
    mesh = block_grid(nblk, (n, n, 1), (0.0, 0.0, 0.0), (1.0, 0.5, 1.0), "outflow", 2)

    def f(x, y, z):
        left = x < 0.5
        return np.where(left, 1.0, 0.125), 0.0, 0.0, 0.0, np.where(left, 1.0, 0.1)

    U0 = conserved_arena(mesh, grid_field(mesh, f), gamma)
    return Problem("sod2d", mesh, U0, gamma, 0.4, nsteps, [np.arange(mesh.nblocks)])


def sedov_deposit(mesh: BlockMesh, prims, energy: float, radius_cells: float, centre, gamma: float):
    """Add `energy` of thermal energy uniformly to the cells whose centres lie
    within radius_cells * dx of `centre` (pressure raised by (gamma-1) * e)."""
    sel = []
    for b in range(mesh.nblocks):
        x, y, z = mesh.cell_centres(b)
        r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
        sel.append(r2 <= (radius_cells * mesh.dx[b, 0]) ** 2 * (1 + 1e-12))
    count = sum(int(s.sum()) for s in sel)
    vol = float(np.prod(mesh.dx[0]))
    e_density = energy / (count * vol)
    for b in range(mesh.nblocks):
        prims[b][4] = np.where(sel[b], prims[b][4] + (gamma - 1.0) * e_density, prims[b][4])
    return count


def sedov3d(nblk=(8, 8, 8), n=16, packet=64, nsteps=50) -> Problem:
    """3D Sedov-like blast on the periodic unit cube: rho = 1, p = 1e-5,
    energy 1.0 deposited uniformly in the cells within 2 cells of the centre;
    gamma 1.4; packets are the z-layers of the block grid (64 blocks each)."""
    gamma = 1.4
    mesh = block_grid(nblk, (n, n, n), (0, 0, 0), (1, 1, 1), "periodic", 3)
    prims = grid_field(mesh, lambda x, y, z: (1.0, 0.0, 0.0, 0.0, 1e-5))
    count = sedov_deposit(mesh, prims, 1.0, 2.0, (0.5, 0.5, 0.5), gamma)
    U0 = conserved_arena(mesh, prims, gamma)
    return Problem("sedov3d", mesh, U0, gamma, 0.4, nsteps, contiguous_packets(mesh.nblocks, packet),
                   {"deposit_cells": count})


def _smooth_modes(rng):
    ks = np.array([(a, b, c) for a in range(-4, 5) for b in range(-4, 5) for c in range(-4, 5)
                   if 1 <= a * a + b * b + c * c <= 16], dtype=np.float64)
    return ks


_KS = None


def smooth_fields(rng, x, y, z):
    """rho = 1 + 0.1 * mean of 8 cosines, v_d = 0.1/sqrt(8) * sum of 8 Gaussian-
    weighted cosines; wave vectors uniform over integer k with 1 <= |k| <= 4
    (so the fields are periodic on the unit cube); p = 1."""
    global _KS
    if _KS is None:
        _KS = _smooth_modes(rng)
    ks = _KS

    def series(weights):
        idx = rng.integers(0, len(ks), size=8)
        phase = rng.uniform(0.0, 2.0 * math.pi, size=8)
        acc = np.zeros_like(x)
        for m in range(8):
            k = ks[idx[m]]
            acc += weights[m] * np.cos(2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + phase[m])
        return acc

    rho = 1.0 + 0.1 * series(np.full(8, 1.0 / 8.0))
    vel = [0.1 / math.sqrt(8.0) * series(rng.standard_normal(8)) for _ in range(3)]
    return rho, vel[0], vel[1], vel[2], np.ones_like(x)


def smooth3d(nblk=(16, 16, 16), n=16, packet=64, nsteps=100, seed=1) -> Problem:
    """3D smooth random flow on the periodic unit cube, gamma 5/3."""
    gamma = 5.0 / 3.0
    mesh = block_grid(nblk, (n, n, n), (0, 0, 0), (1, 1, 1), "periodic", 3)
    rng = np.random.default_rng(seed)
    # one global draw of the modes, evaluated block by block
    state = rng.bit_generator.state
    prims = []
    for b in range(mesh.nblocks):
        r = np.random.default_rng()
        r.bit_generator.state = state
        x, y, z = mesh.cell_centres(b)
        prims.append(np.stack(smooth_fields(r, x, y, z)))
    U0 = conserved_arena(mesh, prims, gamma)
    return Problem("smooth3d", mesh, U0, gamma, 0.4, nsteps, contiguous_packets(mesh.nblocks, packet))


def loguniform_packets(nblocks: int, seed: int, lo: int = 1, hi: int = 256) -> list:
    """Cut 0..nblocks-1 sequentially into packets whose sizes are
    round(exp(U(ln lo, ln hi))) (the last one takes the remainder)."""
    rng = np.random.default_rng(seed)
    out, start = [], 0
    while start < nblocks:
        s = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        s = max(lo, min(hi, s))
        out.append(np.arange(start, min(nblocks, start + s)))
        start += s
    return out


def uneven(nblocks=6000, nsteps=20, seed=2, packet_seed=3, sizes=(8, 16, 32), probs=(0.5, 0.35, 0.15)) -> Problem:
    """Self-periodic blocks of edge 8/16/32 (probabilities 0.5/0.35/0.15), each
    on its own unit cube with smooth random fields seeded seed + block id;
    gamma 5/3; packets of log-uniform size in [1, 256]."""
    gamma = 5.0 / 3.0
    rng = np.random.default_rng(seed)
    edge = rng.choice(np.asarray(sizes), size=nblocks, p=np.asarray(probs))
    mesh = independent_blocks(edge, 3)
    prims = []
    for b in range(nblocks):
        x, y, z = mesh.cell_centres(b)
        prims.append(np.stack(smooth_fields(np.random.default_rng(seed + b), x, y, z)))
    U0 = conserved_arena(mesh, prims, gamma)
    return Problem("uneven", mesh, U0, gamma, 0.4, nsteps, loguniform_packets(nblocks, packet_seed))


def sedov_noise(nblk=(32, 32, 32), n=16, packet=64, nsteps=20, seed=4) -> Problem:
    """Large run: 32^3 blocks of 16^3 on the periodic unit cube, Sedov deposit
    as in ``sedov3d`` plus density noise rho *= 1 + 0.01 xi, xi ~ U(-1, 1)
    i.i.d. per cell; gamma 1.4.  Fields are written straight into the arena
    (the per-block loop of ``grid_field`` would be slow at this size)."""
    gamma = 1.4
    nbx, nby, nbz = nblk
    mesh = block_grid(nblk, (n, n, n), (0, 0, 0), (1, 1, 1), "periodic", 3)
    U0 = np.empty(mesh.arena_len, dtype=np.float64)
    blocks = U0.reshape(nbz, nby, nbx, NVAR, n, n, n)
    rng = np.random.default_rng(seed)
    h = 1.0 / (nbx * n)
    centre_cells = []
    # global cell index of the deposit: centres within 2h of (1/2,1/2,1/2)
    gi = np.arange(nbx * n)
    off = (gi + 0.5) * h - 0.5
    near = np.nonzero(np.abs(off) <= 2.0 * h)[0]
    for a in near:
        for bb in near:
            for c in near:
                if off[a] ** 2 + off[bb] ** 2 + off[c] ** 2 <= (2.0 * h) ** 2 * (1 + 1e-12):
                    centre_cells.append((c, bb, a))  # (z, y, x) global indices
    count = len(centre_cells)
    e_dep = 1.0 / (count * h ** 3)
    p0 = 1e-5
    for bz in range(nbz):
        # density noise drawn layer by layer in (z, y, x) global order
        noise = rng.uniform(-1.0, 1.0, size=(n, nby * n, nbx * n))
        rho = 1.0 + 0.01 * noise
        rho_b = rho.reshape(n, nby, n, nbx, n).transpose(1, 3, 0, 2, 4)
        layer = blocks[bz]
        layer[:, :, 0] = rho_b
        layer[:, :, 1:4] = 0.0
        layer[:, :, 4] = p0 / (gamma - 1.0)
    for (z, y, x) in centre_cells:
        blocks[z // n, y // n, x // n, 4, z % n, y % n, x % n] += e_dep
    return Problem("sedov_noise", mesh, U0, gamma, 0.4, nsteps, contiguous_packets(mesh.nblocks, packet),
                   {"deposit_cells": count, "subset": centred_subset(nblk, 8)})


def centred_subset(nblk, width: int) -> np.ndarray:
    """Ids of the width^3 cube of blocks centred in the block grid."""
    nbx, nby, nbz = nblk
    lo = [(d - width) // 2 for d in nblk]
    ids = [((z * nby + y) * nbx + x)
           for z in range(lo[2], lo[2] + width)
           for y in range(lo[1], lo[1] + width)
           for x in range(lo[0], lo[0] + width)]
    return np.asarray(ids, dtype=np.int64)


def contiguous_packets(nblocks: int, size: int) -> list:
    return [np.arange(s, min(nblocks, s + size)) for s in range(0, nblocks, size)]


def uniform_state(mesh: BlockMesh, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, gamma=1.4) -> np.ndarray:
    prims = grid_field(mesh, lambda x, y, z: (rho, vel[0], vel[1] if mesh.ndim >= 2 else 0.0,
                                              vel[2] if mesh.ndim == 3 else 0.0, p))
    return conserved_arena(mesh, prims, gamma)


def random_smooth_state(mesh: BlockMesh, seed: int, gamma: float) -> np.ndarray:
    """Smooth random state evaluated on an arbitrary mesh (per-block seeds)."""
    prims = []
    for b in range(mesh.nblocks):
        x, y, z = mesh.cell_centres(b)
        r, u, v, w, p = smooth_fields(np.random.default_rng(seed + b), x, y, z)
        if mesh.ndim == 2:
            w = np.zeros_like(w)
        prims.append(np.stack([r, u, v, w, p]))
    return conserved_arena(mesh, prims, gamma)
