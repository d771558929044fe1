"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module only draws inputs (cells, grid sizes, atom positions, charges,
widths, random grids); it holds none of the solver's arithmetic, so both the
GPU path and the CPU oracle can consume what it returns.

The workloads stand in for the paper's diamond benchmark system (Sec. 5.1.3,
"Benchmark system"): OpenMX densities of C atoms on a regular grid.  Here the
density is a sum of normalized Gaussians (Z = 4 for carbon's valence charge)
placed on diamond lattice sites, so no basis sets or pseudopotentials are
needed.

Five named configurations (seed = 1209 + index):

0. ``cubic32``       cubic cell a = 10 Bohr, 32^3 grid, 8 uniform atoms.
1. ``diamond180``    4x4x4 conventional diamond cell (512 atoms), a = 26.96 Bohr, 180^3.
2. ``diamond360``    8x8x8 diamond (4096 atoms), a = 53.93 Bohr, 360^3 (headline size).
3. ``batched24``     24 orthorhombic cells, edges U[8, 40] Bohr, each grid dim drawn
                     from {48, 60, 72, 90, 120, 150, 180, 240}, 16..512 atoms with
                     Z in {1, 4, 6} and sigma in U[0.6, 1.0]; per-problem seed 120900 + p.
4. ``cubic1024``     cubic a = 150 Bohr, 1024^3 grid, 32768 uniform atoms.

and, on grids with a factor 7 at the paper's own grid spacing (0.2568 Bohr,
Sec. 5.2.6: 420 x 420 x 210 points for 16,384 diamond atoms):

5. ``diamond16384``  16x16x8 conventional diamond cells (16,384 atoms),
                     107.85 x 107.85 x 53.93 Bohr, 420 x 420 x 210 grid.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1209
BATCH_DIMS = (48, 60, 72, 90, 120, 150, 180, 240)

# fractional coordinates of the 8 atoms of the conventional diamond cell
_DIAMOND_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
     [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25]])


@dataclass
class Problem:
    """One periodic cell with its grid and Gaussian atoms (Bohr, electron charges)."""

    name: str
    cell: np.ndarray          # (3, 3) rows a, b, c
    dims: tuple               # (Na, Nb, Nc)
    pos: np.ndarray           # (n, 3) Cartesian positions
    Z: np.ndarray             # (n,)
    sigma: np.ndarray         # (n,)
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def natoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def npoints(self) -> int:
        return int(np.prod(self.dims))


def diamond_sites(reps: int, a_conv: float) -> np.ndarray:
    """Cartesian sites of a reps^3 supercell of the conventional diamond cell."""
    cells = np.array([[i, j, k] for i in range(reps) for j in range(reps) for k in range(reps)], float)
    frac = (cells[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3) / reps
    return frac * (a_conv * reps)


def _cubic(L: float) -> np.ndarray:
    return np.diag([L, L, L]).astype(np.float64)


def cubic32(seed: int = SEED_BASE + 0) -> Problem:
    rng = np.random.default_rng(seed)
    L = 10.0
    frac = rng.random((8, 3))
    return Problem("cubic32", _cubic(L), (32, 32, 32), frac * L, np.full(8, 4.0), np.full(8, 0.8), seed)


def _diamond(reps: int, L: float, n: int, name: str, seed: int) -> Problem:
    rng = np.random.default_rng(seed)
    sites = diamond_sites(reps, L / reps)
    pos = sites + rng.normal(0.0, 0.05, sites.shape)
    na = sites.shape[0]
    p = Problem(name, _cubic(L), (n, n, n), pos, np.full(na, 4.0), np.full(na, 0.8), seed)
    return p


def diamond180(seed: int = SEED_BASE + 1) -> Problem:
    return _diamond(4, 26.96, 180, "diamond180", seed)


def diamond360(seed: int = SEED_BASE + 2) -> Problem:
    p = _diamond(8, 53.93, 360, "diamond360", seed)
    # the 16 atoms whose forces are checked by finite differences
    p.extra["fd_atoms"] = np.random.default_rng(seed + 7).choice(p.natoms, 16, replace=False)
    return p


def diamond16384(seed: int = SEED_BASE + 5) -> Problem:
    """16x16x8 conventional diamond cells (a = 6.7406 Bohr) on the paper's
    420 x 420 x 210 grid; 16 atoms chosen for the force checks."""
    rng = np.random.default_rng(seed)
    a_conv = 53.93 / 8
    reps = (16, 16, 8)
    cells = np.array([[i, j, k] for i in range(reps[0]) for j in range(reps[1]) for k in range(reps[2])], float)
    sites = (cells[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3) * a_conv
    pos = sites + rng.normal(0.0, 0.05, sites.shape)
    n = pos.shape[0]
    cell = np.diag([a_conv * reps[0], a_conv * reps[1], a_conv * reps[2]])
    p = Problem("diamond16384", cell, (420, 420, 210), pos, np.full(n, 4.0), np.full(n, 0.8), seed)
    p.extra["fd_atoms"] = np.random.default_rng(seed + 7).choice(n, 16, replace=False)
    return p


def batched24(seed: int = SEED_BASE + 3, nprob: int = 24) -> list:
    out = []
    for p in range(nprob):
        rng = np.random.default_rng(SEED_BASE * 100 + p)
        edges = rng.uniform(8.0, 40.0, 3)
        dims = tuple(int(v) for v in rng.choice(BATCH_DIMS, 3))
        n = int(rng.integers(16, 513))
        Z = rng.choice(np.array([1.0, 4.0, 6.0]), n)
        sigma = rng.uniform(0.6, 1.0, n)
        pos = rng.random((n, 3)) * edges
        out.append(Problem("batched24[%d]" % p, np.diag(edges), dims, pos, Z, sigma, SEED_BASE * 100 + p))
    return out


def cubic1024(seed: int = SEED_BASE + 4) -> Problem:
    rng = np.random.default_rng(seed)
    L = 150.0
    n = 32768
    p = Problem("cubic1024", _cubic(L), (1024, 1024, 1024), rng.random((n, 3)) * L,
                np.full(n, 4.0), np.full(n, 0.8), seed)
    # the 16 atoms whose forces are checked against the oracle adjoint
    p.extra["fd_atoms"] = np.random.default_rng(seed + 7).choice(n, 16, replace=False)
    return p


CONFIGS = {0: cubic32, 1: diamond180, 2: diamond360, 3: batched24, 4: cubic1024, 5: diamond16384}


def config(i: int):
    return CONFIGS[i]()


def random_grid(dims, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded N(0, 1) grid of shape dims (the loss weights c and test fields)."""
    return np.random.default_rng(seed).standard_normal(tuple(int(v) for v in dims)).astype(dtype)


def random_cell(seed: int, triclinic: bool = True) -> np.ndarray:
    """A seeded well-conditioned cell: a scaled identity plus a shear."""
    rng = np.random.default_rng(seed)
    A = np.diag(rng.uniform(6.0, 12.0, 3))
    if triclinic:
        A = A + np.triu(rng.uniform(-2.0, 2.0, (3, 3)), 1)
    return A


def small_problem(dims, natoms: int, seed: int, L=(9.0, 10.0, 11.0), zs=(1.0, 4.0, 6.0),
                  sig=(0.6, 1.0)) -> Problem:
    """A small orthorhombic test problem with mixed charges and widths."""
    rng = np.random.default_rng(seed)
    edges = np.asarray(L, dtype=np.float64)
    pos = rng.random((natoms, 3)) * edges
    Z = rng.choice(np.asarray(zs), natoms)
    sigma = rng.uniform(sig[0], sig[1], natoms)
    return Problem("small", np.diag(edges), tuple(int(v) for v in dims), pos, Z, sigma, seed)


def small_cell_problem(cell, dims, natoms: int, seed: int, zs=(1.0, 4.0, 6.0), sig=(0.6, 1.0)) -> Problem:
    """Atoms at uniform fractional positions of any (e.g. triclinic) cell; some
    positions are pushed outside the cell to exercise the wrapping."""
    rng = np.random.default_rng(seed)
    cell = np.asarray(cell, dtype=np.float64)
    frac = rng.random((natoms, 3)) + rng.integers(-1, 2, (natoms, 3))
    pos = frac @ cell
    Z = rng.choice(np.asarray(zs), natoms)
    sigma = rng.uniform(sig[0], sig[1], natoms)
    return Problem("small_cell", cell, tuple(int(v) for v in dims), pos, Z, sigma, seed)


def diamond_fcc1024(seed: int = SEED_BASE + 6) -> Problem:
    """Diamond in its primitive (FCC, rhombohedral) cell, 8 x 8 x 8 primitive
    cells of 2 atoms (1,024 atoms), on a 160^3 grid: a non-orthogonal cell for
    the general-cell splat."""
    rng = np.random.default_rng(seed)
    a_conv = 53.93 / 8
    prim = 0.5 * a_conv * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    reps = 8
    cell = reps * prim
    idx = np.array([[i, j, k] for i in range(reps) for j in range(reps) for k in range(reps)], float)
    # two atoms per primitive cell, at fractional (0, 0, 0) and (1/4, 1/4, 1/4)
    basis = np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]]) @ prim
    sites = ((idx @ prim)[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = sites + rng.normal(0.0, 0.05, sites.shape)
    n = pos.shape[0]
    p = Problem("diamond_fcc1024", cell, (160, 160, 160), pos, np.full(n, 4.0), np.full(n, 0.8), seed)
    p.extra["fd_atoms"] = np.random.default_rng(seed + 7).choice(n, 16, replace=False)
    return p
