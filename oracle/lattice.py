"""Lattice geometry (Sec. 4) and the hierarchy of nested grids (Sec. 7.2).

Part of the FP64 CPU oracle -- test infrastructure only.

Readings taken where the paper is silent:
* Node (a, b, c) rests at t_hat = o + h (a, b, c); nodes are numbered
  a + nx (b + ny c).
* A point's cell is floor((x - o) / h) clamped per axis to [0, n - 2]; its
  fractional coordinate f = (x - o)/h - cell.  A point on the last plane
  therefore uses cell n - 2 with f = 1.  Outside the lattice f leaves [0, 1],
  which is linear extrapolation (used only by prolongation).
* Corner k = dx + 2 dy + 4 dz of a cell has weight prod_axis (f if d else 1-f).
* The one-ring of Sec. 6 is the 6-neighbourhood; boundary nodes have 3-5.
* Levels are vertex-nested: n_coarse = ceil(n_fine / 2), h_coarse = 2 h_fine,
  a shared origin, and coarse node j coincides with fine node 2 j.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


@dataclass(frozen=True)
class Grid:
    dims: Tuple[int, int, int]
    h: float
    origin: Tuple[float, float, float]

    @property
    def n(self) -> int:
        nx, ny, nz = self.dims
        return nx * ny * nz

    def node_id(self, a, b, c):
        nx, ny, _ = self.dims
        return np.asarray(a) + nx * (np.asarray(b) + ny * np.asarray(c))

    def coords(self) -> np.ndarray:
        """Integer lattice coordinates (N,3) in node order."""
        nx, ny, nz = self.dims
        c, b, a = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        return np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)

    def rest_positions(self) -> np.ndarray:
        """t_hat_i = o + h (a, b, c), Sec. 4: positions start as a regular grid."""
        return np.asarray(self.origin, np.float64)[None, :] + self.h * self.coords().astype(np.float64)


def level_grids(dims: Sequence[int], h: float, origin: Sequence[float],
                num_levels: int) -> List[Grid]:
    """The nested hierarchy of Sec. 7.2, listed coarse -> fine."""
    grids = []
    d = tuple(int(x) for x in dims)
    hh = float(h)
    for _ in range(num_levels):
        if min(d) < 2:
            raise ValueError("every level needs at least 2 nodes per axis")
        grids.append(Grid(d, hh, tuple(float(x) for x in origin)))
        d = tuple((x + 1) // 2 for x in d)
        hh *= 2.0
    return grids[::-1]


def cell_and_frac(grid: Grid, x: np.ndarray):
    """Cell index (K,3) and fractional coordinates (K,3) of points x (K,3)."""
    u = (np.asarray(x, np.float64) - np.asarray(grid.origin)[None, :]) / grid.h
    hi = np.asarray(grid.dims) - 2
    cell = np.clip(np.floor(u), 0, hi[None, :]).astype(np.int64)
    return cell, u - cell


CORNERS = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], np.int64)


def trilinear(grid: Grid, x: np.ndarray):
    """Trilinear interpolation weights of Sec. 4: for each point the 8 corner
    node ids (K,8) and weights alpha (K,8), so that S(x) = sum_k alpha_k t_k."""
    cell, f = cell_and_frac(grid, x)
    ids = np.empty((cell.shape[0], 8), np.int64)
    w = np.empty((cell.shape[0], 8), np.float64)
    for k, (dx, dy, dz) in enumerate(CORNERS):
        ids[:, k] = grid.node_id(cell[:, 0] + dx, cell[:, 1] + dy, cell[:, 2] + dz)
        wx = f[:, 0] if dx else 1.0 - f[:, 0]
        wy = f[:, 1] if dy else 1.0 - f[:, 1]
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        w[:, k] = wx * wy * wz
    return ids, w


def inside(grid: Grid, x: np.ndarray) -> np.ndarray:
    """True where x lies in the closed box spanned by the grid's nodes."""
    u = (np.asarray(x, np.float64) - np.asarray(grid.origin)[None, :]) / grid.h
    hi = np.asarray(grid.dims, np.float64) - 1.0
    return np.all((u >= 0.0) & (u <= hi[None, :]), axis=1)


def arap_edges(grid: Grid):
    """Directed edges (i, j) with j in the 6-neighbourhood of i (eq. (4))."""
    coords = grid.coords()
    ids = grid.node_id(coords[:, 0], coords[:, 1], coords[:, 2])
    src, dst = [], []
    for axis in range(3):
        for step in (-1, 1):
            nb = coords.copy()
            nb[:, axis] += step
            ok = (nb[:, axis] >= 0) & (nb[:, axis] < grid.dims[axis])
            src.append(ids[ok])
            dst.append(grid.node_id(nb[ok, 0], nb[ok, 1], nb[ok, 2]))
    return np.concatenate(src), np.concatenate(dst)
