"""Non-rigid TSDF fusion (Sec. 8) and the data-parallel marching cubes that
extracts the canonical surface (Sec. 4), with the extracted vertices deformed
by the current field S(x) = R sum_k alpha_k(x) t_k + t.

Part of the FP64 CPU oracle -- test infrastructure only.

The TSDF shares the finest lattice's grid (Sec. 4): grid point i stores a
truncated signed distance D_i and a confidence W_i, both 0 initially (W = 0:
never observed), as float32.  Readings where the paper is silent:

  * F1 grid point i sits, deformed, at x_i = R t_i + t (its lattice position
    after deformation, then the global pose);
  * F2 its projective signed distance is eta = D(u) - x_i.z, with u the pixel
    x_i falls on (the camera model of ``assoc``) and D(u) > 0 required;
  * F3 with truncation tau: no update if eta < -tau, else the sample is
    min(1, eta / tau);
  * F4 weighted floating average with unit sample weight:
    D_i <- (W_i D_i + s) / (W_i + 1), W_i <- min(W_i + 1, W_max), computed in
    float64 from the stored float32 values and stored as float32;
  * F5 only grid points allowed by a mask are updated: those of M that have
    been in the optimisation for at least K_min = 3 frames in a row (Sec. 8);
    the first frame of a sequence, before any surface exists, integrates into
    every grid point;
  * F6 marching cubes on the lattice's cells whose 8 corners all have W > 0:
    a corner is inside when D < 0; the vertex on an edge (a, b) whose corners
    differ is x_a + (D_a / (D_a - D_b)) (x_b - x_a), in float64 from the
    float32 D and rounded to float32;
  * F7 the polygon of a cell is built face by face: walking each face's four
    corners counter-clockwise as seen from outside the cube, every maximal
    run of inside corners gives a segment from the edge where the run is
    entered to the edge where it is left (so a face whose inside corners are
    diagonal cuts each of them off separately); the segments chain into
    closed loops, each loop starts at its lowest edge index and is split into
    a fan of triangles from that vertex.  Corners are k = dx + 2 dy + 4 dz;
    the 12 edges are numbered 4 q + j along axis q, j = b1 + 2 b2 from the
    bits of the two other axes in increasing order;
  * F8 output: triangles in increasing cell order (x fastest), then in loop
    and fan order, each as three edge numbers and three canonical vertices.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from . import assoc
from .lattice import Grid, cell_and_frac, CORNERS


# ---------------------------------------------------------------------------
# TSDF fusion
# ---------------------------------------------------------------------------

def deformed_points(grid: Grid, disp: np.ndarray, pose: np.ndarray) -> np.ndarray:
    """Reading F1: x_i = R (t_hat_i + d_i) + t, each component summed left to
    right."""
    rest = np.asarray(grid.origin, np.float64)[None, :] + grid.h * grid.coords().astype(np.float64)
    p = rest + np.asarray(disp, np.float64).reshape(-1, 3)
    P = np.asarray(pose, np.float64).reshape(12)
    x = np.empty_like(p)
    for r in range(3):
        x[:, r] = P[3 * r] * p[:, 0] + P[3 * r + 1] * p[:, 1] + P[3 * r + 2] * p[:, 2] + P[9 + r]
    return x


def integrate(grid: Grid, D: np.ndarray, W: np.ndarray, disp: np.ndarray, pose: np.ndarray,
              cam: assoc.Camera, depth: np.ndarray, allowed: np.ndarray, tau: float,
              w_max: float) -> Tuple[np.ndarray, np.ndarray, int]:
    """One fusion step (readings F1-F5).  Returns (D, W, points updated)."""
    D = np.asarray(D, np.float32).copy()
    W = np.asarray(W, np.float32).copy()
    x = deformed_points(grid, disp, pose)
    n = 0
    for i in np.flatnonzero(np.asarray(allowed, bool)):
        pix = assoc.pixel_of(cam, x[i])
        if pix is None:
            continue
        u, v = pix
        z = float(depth[v, u])
        if not z > 0.0:
            continue
        eta = z - x[i, 2]
        if eta < -tau:
            continue
        s = min(1.0, eta / tau)
        w = float(W[i])
        D[i] = np.float32((w * float(D[i]) + s) / (w + 1.0))
        W[i] = np.float32(min(w + 1.0, w_max))
        n += 1
    return D, W, n


def allowed_points(act: np.ndarray, frames_in_set: np.ndarray, k_min: int = 3) -> np.ndarray:
    """Reading F5: points of M that have been optimised for k_min frames."""
    return np.asarray(act, bool) & (np.asarray(frames_in_set) >= k_min)


# ---------------------------------------------------------------------------
# marching cubes
# ---------------------------------------------------------------------------

def _edge_of(a: int, b: int) -> int:
    """Edge number of the corners a, b (differing in one bit), reading F7."""
    q = (a ^ b).bit_length() - 1
    o1, o2 = [k for k in range(3) if k != q]
    j = ((a >> o1) & 1) + 2 * ((a >> o2) & 1)
    return 4 * q + j


EDGE_CORNERS = []
for _q in range(3):
    _o1, _o2 = [k for k in range(3) if k != _q]
    for _j in range(4):
        _a = (((_j >> 0) & 1) << _o1) | (((_j >> 1) & 1) << _o2)
        EDGE_CORNERS.append((_a, _a | (1 << _q)))


def _faces():
    """Every face's corners counter-clockwise as seen from outside the cube."""
    faces = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3      # e_b x e_c = e_a
        for s in (0, 1):
            ring = [(0, 0), (1, 0), (1, 1), (0, 1)]   # counter-clockwise about +e_a
            if s == 0:
                ring = ring[::-1]                       # outward normal -e_a
            faces.append([(s << a) | (u << b) | (w << c) for (u, w) in ring])
    return faces


FACES = _faces()


def cell_loops(inside: int) -> List[List[int]]:
    """Reading F7: the closed loops (lists of edge numbers) of a cube whose
    corners k with bit k of `inside` set are inside."""
    nxt = {}
    for face in FACES:
        neg = [(inside >> k) & 1 for k in face]
        if all(neg) or not any(neg):
            continue
        for m in range(4):
            # a run of inside corners starts at face[m] (its predecessor outside)
            if neg[m] and not neg[m - 1]:
                enter = _edge_of(face[m - 1], face[m])
                e = m
                while neg[(e + 1) % 4]:
                    e = (e + 1) % 4
                leave = _edge_of(face[e], face[(e + 1) % 4])
                nxt[enter] = leave
    loops = []
    seen = set()
    for start in sorted(nxt):
        if start in seen:
            continue
        loop = [start]
        seen.add(start)
        e = nxt[start]
        while e != start:
            loop.append(e)
            seen.add(e)
            e = nxt[e]
        loops.append(loop)
    return loops


def cell_triangles(inside: int) -> List[Tuple[int, int, int]]:
    """Fan triangles of every loop (reading F7)."""
    tris = []
    for loop in cell_loops(inside):
        for k in range(1, len(loop) - 1):
            tris.append((loop[0], loop[k], loop[k + 1]))
    return tris


def marching_cubes(grid: Grid, D: np.ndarray, W: np.ndarray):
    """Readings F6-F8.  Returns (cell ids (T,), edge numbers (T,3), canonical
    vertices (T,3,3) float32)."""
    D = np.asarray(D, np.float32)
    W = np.asarray(W, np.float32)
    nx, ny, nz = grid.dims
    o = np.asarray(grid.origin, np.float64)
    cells, edges, verts = [], [], []
    for cz in range(nz - 1):
        for cy in range(ny - 1):
            for cx in range(nx - 1):
                ids = [grid.node_id(cx + dx, cy + dy, cz + dz) for (dx, dy, dz) in CORNERS]
                if not all(W[i] > 0 for i in ids):
                    continue
                val = [float(D[i]) for i in ids]
                inside = sum(1 << k for k in range(8) if val[k] < 0.0)
                if inside == 0 or inside == 255:
                    continue
                for tri in cell_triangles(inside):
                    vv = []
                    for e in tri:
                        a, b = EDGE_CORNERS[e]
                        xa = o + grid.h * np.array([cx + (a & 1), cy + ((a >> 1) & 1),
                                                    cz + (a >> 2)], np.float64)
                        xb = o + grid.h * np.array([cx + (b & 1), cy + ((b >> 1) & 1),
                                                    cz + (b >> 2)], np.float64)
                        t = val[a] / (val[a] - val[b])
                        vv.append((xa + t * (xb - xa)).astype(np.float32))
                    cells.append(cx + (nx - 1) * (cy + (ny - 1) * cz))
                    edges.append(tri)
                    verts.append(vv)
    return (np.array(cells, np.int64), np.array(edges, np.int64).reshape(-1, 3),
            np.array(verts, np.float32).reshape(-1, 3, 3))


def deform_vertices(grid: Grid, disp: np.ndarray, pose: np.ndarray, x: np.ndarray) -> np.ndarray:
    """S(x) = R (x + sum_k alpha_k(x) d_k) + t for canonical points x (the
    extracted vertices, Sec. 4), summed over the corners k in order."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    d = np.asarray(disp, np.float64).reshape(-1, 3)
    cell, f = cell_and_frac(grid, x)
    s = np.zeros_like(x)
    for (dx, dy, dz) in CORNERS:
        wx = f[:, 0] if dx else 1.0 - f[:, 0]
        wy = f[:, 1] if dy else 1.0 - f[:, 1]
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        a = wx * wy * wz
        ids = grid.node_id(cell[:, 0] + dx, cell[:, 1] + dy, cell[:, 2] + dz)
        for r in range(3):
            s[:, r] += a * d[ids, r]
    p = x + s
    P = np.asarray(pose, np.float64).reshape(12)
    out = np.empty_like(p)
    for r in range(3):
        out[:, r] = P[3 * r] * p[:, 0] + P[3 * r + 1] * p[:, 1] + P[3 * r + 2] * p[:, 2] + P[9 + r]
    return out

