"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws densities and evaluation points.  It holds none of the
gravity arithmetic, so both the GPU library's callers and the oracle can use
it without sharing any of the method.

Recipes (stand-ins for the paper's setups: a brick voxel mesh with a smooth or
prismatic density and stations on a plane above it, Secs. 2.1 and 3):

* Grid: ``n`` cells per axis on the unit cube, ``h = 1/n``, origin 0; cell
  (i, j, k) has centre ``((i, j, k) + 1/2) h``; arrays are ``[nz][ny][nx]``.
* Gaussian blobs: centres U[0,1]^3, widths U[0.05, 0.2], amplitudes N(0, 1),
  drawn in that order from ``numpy.random.default_rng(seed)``; the density of a
  cell is the blob sum sampled at its centre (constant per cell); optional
  additive noise U[-a, a] drawn after the blobs.
* Stations: an ``ns x ns`` regular array at height ``z`` (default 1.1) over
  the grid's horizontal extent, points at ``((i + 1/2)/ns, (j + 1/2)/ns)``,
  x fastest.
* Voxel centres: every cell centre, x fastest (the order of ``rho``).
* The paper's model (Sec. 3): domain [0,600]^2 x [-450,150] m, a cube
  [250,350]^2 x [-200,-100] m of density 2000 kg/m^3 in void.
* Seeded subsets: ``default_rng(7).choice(M, k, replace=False)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    origin: tuple = (0.0, 0.0, 0.0)
    h: float = 1.0

    @staticmethod
    def unit(n: int) -> "Grid":
        return Grid(n, n, n, (0.0, 0.0, 0.0), 1.0 / n)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def axis_centres(self, axis: int) -> np.ndarray:
        n = (self.nx, self.ny, self.nz)[axis]
        return self.origin[axis] + (np.arange(n) + 0.5) * self.h

    def centres(self) -> np.ndarray:
        """All cell centres ``[ncell, 3]``, x fastest."""
        x, y, z = (self.axis_centres(a) for a in range(3))
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def gaussian_blobs(grid: Grid, n_blobs: int, seed: int, noise: float = 0.0,
                   width=(0.05, 0.2), lo=0.0, hi=1.0) -> np.ndarray:
    """Sum of seeded Gaussian blobs sampled at cell centres: ``[nz, ny, nx]`` f64."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(n_blobs, 3))
    widths = rng.uniform(width[0], width[1], size=n_blobs)
    amps = rng.normal(0.0, 1.0, size=n_blobs)
    x, y, z = (grid.axis_centres(a) for a in range(3))
    rho = np.zeros(grid.shape, dtype=np.float64)
    for b in range(n_blobs):
        s = 1.0 / (2.0 * widths[b] ** 2)
        ex = np.exp(-s * (x - centres[b, 0]) ** 2)
        ey = np.exp(-s * (y - centres[b, 1]) ** 2)
        ez = np.exp(-s * (z - centres[b, 2]) ** 2)
        rho += amps[b] * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    if noise:
        rho += rng.uniform(-noise, noise, size=grid.shape)
    return rho


def stations(ns: int, z: float = 1.1, xr=(0.0, 1.0), yr=(0.0, 1.0)) -> np.ndarray:
    """``ns x ns`` regular stations at height z, x fastest: ``[ns*ns, 3]``."""
    x = xr[0] + (np.arange(ns) + 0.5) * (xr[1] - xr[0]) / ns
    y = yr[0] + (np.arange(ns) + 0.5) * (yr[1] - yr[0]) / ns
    Y, X = np.meshgrid(y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)


def box_density(grid: Grid, box, value: float = 1.0) -> np.ndarray:
    """``value`` in every cell whose centre lies inside ``box``, else 0."""
    x, y, z = (grid.axis_centres(a) for a in range(3))
    mx = (x > box[0][0]) & (x < box[0][1])
    my = (y > box[1][0]) & (y < box[1][1])
    mz = (z > box[2][0]) & (z < box[2][1])
    m = mz[:, None, None] & my[None, :, None] & mx[None, None, :]
    return np.where(m, float(value), 0.0)


def snapped_box(grid: Grid, box):
    """The union of cells selected by :func:`box_density`, as an explicit box."""
    out = []
    for a in range(3):
        c = grid.axis_centres(a)
        sel = np.nonzero((c > box[a][0]) & (c < box[a][1]))[0]
        if sel.size == 0:
            return None
        out.append((grid.origin[a] + sel[0] * grid.h, grid.origin[a] + (sel[-1] + 1) * grid.h))
    return tuple(out)


# The paper's synthetic model (Sec. 3).
PAPER_DOMAIN = ((0.0, 600.0), (0.0, 600.0), (-450.0, 150.0))
PAPER_CUBE = ((250.0, 350.0), (250.0, 350.0), (-200.0, -100.0))
PAPER_RHO = 2000.0
G_SI = 6.67428e-11


def paper_model(nbar: int):
    """(grid, rho) of the paper's model on an nbar^3 mesh."""
    h = 600.0 / nbar
    grid = Grid(nbar, nbar, nbar, (0.0, 0.0, -450.0), h)
    return grid, box_density(grid, PAPER_CUBE, PAPER_RHO)


def sample_indices(m: int, k: int = 4096, seed: int = 7) -> np.ndarray:
    """Seeded subset of k distinct target indices (all of them if m <= k)."""
    if m <= k:
        return np.arange(m)
    return np.sort(np.random.default_rng(seed).choice(m, k, replace=False))


def sphere_density(grid: Grid, centre, radius: float, value: float = 1.0) -> np.ndarray:
    """Voxelised ball: ``value`` in cells whose centre lies within ``radius``."""
    x, y, z = (grid.axis_centres(a) for a in range(3))
    d2 = ((z - centre[2]) ** 2)[:, None, None] + ((y - centre[1]) ** 2)[None, :, None] \
        + ((x - centre[0]) ** 2)[None, None, :]
    return np.where(d2 <= radius * radius, float(value), 0.0)
