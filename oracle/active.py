"""The sparse set M of optimised grid points (Sec. 6, Sec. 7) and the lattice
solve restricted to it, with grid growth by extrapolation (Sec. 8).

Part of the FP64 CPU oracle -- test infrastructure only.

Sec. 6 sums the regulariser over i in M and j in the one-ring N_i of i, with
M the grid points of the isosurface plus their one-ring; Sec. 7 optimises
only the positions and rotations of M (6|M| unknowns); Sec. 8 initialises
grid points that join M for the first time by extrapolating the deformation
field.  Readings where the paper is silent:

  * M1 the isosurface's grid points are the corners of every cell that holds
    a constraint sample (dense or sparse; the samples are the isosurface's
    samples, whatever their association weight), per level;
  * M2 M = those points plus their 6-neighbourhood (the one-ring, as N_i);
  * M3 eq. (4) sums over the points used in the optimisation: i runs over M
    and j over the one-ring points of i that are in M (a point outside M is
    not used at all, so no term anchors M to its stale position; every
    isosurface point keeps its whole one-ring, which is why M adds it);
  * M4 points outside M keep their position and rotation through the frame;
    on every level the prolongated increment and the rotation steps act on
    M only;
  * M5 grid growth on the finest level: the points of M that were not in the
    previous frame's M are filled layer by layer from the points already
    known (the previous M, then earlier layers): a point with at least one
    known 6-neighbour takes the mean of their displacements (summed in the
    order -x, +x, -y, +y, -z, +z) and the rotation of the first of them in
    that order.  Points no layer reaches keep their state.  Without a
    previous M (the first frame) nothing is extrapolated.

Solved as in ``solver.solve_frame``: per level the residual vector of
eqs. (2)-(4) with the ARAP rows of the directed edges inside M; the
position step is Jacobi-PCG (or a direct solve) on the normal equations
restricted to the coordinates of M.
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .energy import Constraints, prepare_constraints
from .lattice import Grid, arap_edges, level_grids, trilinear
from .procrustes import fit_rotations
from .solver import inject, pcg, prolong, rest_state

# neighbour order of reading M5
_STEPS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


def surface_points(grid: Grid, cons: Constraints) -> np.ndarray:
    """Reading M1: corners of the cells holding a dense or sparse sample."""
    flag = np.zeros(grid.n, bool)
    for x in (cons.canon, cons.sparse_canon):
        if x.shape[0]:
            ids, _ = trilinear(grid, x)
            flag[ids.ravel()] = True
    return flag


def one_ring(grid: Grid, flag: np.ndarray) -> np.ndarray:
    """flag plus the 6-neighbours of every flagged point."""
    out = flag.copy()
    src, dst = arap_edges(grid)
    out[dst[flag[src]]] = True
    return out


def active_set(grid: Grid, cons: Constraints) -> np.ndarray:
    """Reading M2: M = isosurface points plus their one-ring."""
    return one_ring(grid, surface_points(grid, cons))


class ActiveSystem:
    """J of eqs. (2)-(4) with the ARAP rows of the edges (i, j) inside M, and
    the normal equations restricted to the coordinates of M."""

    def __init__(self, grid: Grid, cons: Constraints, act: np.ndarray):
        self.grid, self.act = grid, act
        C = cons.canon.shape[0]
        S = cons.sparse_canon.shape[0]
        rows, cols, vals = [], [], []
        ids, alpha = trilinear(grid, cons.canon)
        s = np.sqrt(cons.w_dense * cons.weight)
        for k in range(8):
            for a in range(3):
                rows.append(np.arange(C))
                cols.append(3 * ids[:, k] + a)
                vals.append(s * alpha[:, k] * cons.normal[:, a])
        self.c_dense = s * np.einsum("ca,ca->c", cons.normal, cons.target)
        ids_s, beta = trilinear(grid, cons.sparse_canon)
        ss = np.sqrt(cons.w_sparse)
        for k in range(8):
            for a in range(3):
                rows.append(C + 3 * np.arange(S) + a)
                cols.append(3 * ids_s[:, k] + a)
                vals.append(np.full(S, ss) * beta[:, k])
        self.c_sparse = ss * cons.sparse_target.reshape(-1)
        src, dst = arap_edges(grid)
        keep = act[src] & act[dst]
        src, dst = src[keep], dst[keep]
        E = src.size
        base = C + 3 * S
        sr = np.sqrt(cons.w_arap)
        for a in range(3):
            r = base + 3 * np.arange(E) + a
            rows += [r, r]
            cols += [3 * src + a, 3 * dst + a]
            vals += [np.full(E, sr), np.full(E, -sr)]
        self.J = sp.csr_matrix(
            (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
            shape=(base + 3 * E, 3 * grid.n))
        self.src, self.dst = src, dst
        rest = grid.rest_positions()
        self.e = rest[src] - rest[dst]
        self.sqrt_wr = sr
        self.cols = np.flatnonzero(np.repeat(act, 3))   # coordinates of M
        Ja = self.J[:, self.cols]
        self.A = (Ja.T @ Ja).tocsr()
        d = self.A.diagonal()
        self.dinv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
        self._lu = None

    def residual(self, t: np.ndarray, R: np.ndarray) -> np.ndarray:
        rot_e = np.einsum("eab,eb->ea", R[self.src], self.e)
        c = np.concatenate([self.c_dense, self.c_sparse, self.sqrt_wr * rot_e.reshape(-1)])
        return self.J @ t.reshape(-1) - c

    def gradient(self, t: np.ndarray, R: np.ndarray) -> np.ndarray:
        """g = (J^T r) on the coordinates of M (E(t + d) = E + 2 g^T d + d^T A d
        for displacements d of M)."""
        return (self.J.T @ self.residual(t, R))[self.cols]

    def position_step(self, t: np.ndarray, R: np.ndarray, mode: str, iters: int) -> np.ndarray:
        g = self.gradient(t, R)
        if mode == "direct":
            if self._lu is None:
                self._lu = spla.splu(self.A.tocsc(), permc_spec="COLAMD")
            delta = self._lu.solve(-g)
        else:
            delta = pcg(self.A, -g, self.dinv, iters)
        out = t.reshape(-1).copy()
        out[self.cols] += delta
        return out.reshape(-1, 3)


def energy_terms_active(grid: Grid, t: np.ndarray, R: np.ndarray, cons: Constraints,
                        act: np.ndarray):
    """(E_total, w_d E_dense, w_s E_sparse, w_r E_reg) with E_reg summed over
    the directed edges inside M (reading M3), from the definitions."""
    ids, alpha = trilinear(grid, cons.canon)
    S_p = np.einsum("ck,cka->ca", alpha, t[ids])
    e_dense = float(np.sum(cons.weight * np.einsum("ca,ca->c", S_p - cons.target,
                                                   cons.normal) ** 2))
    ids_s, beta = trilinear(grid, cons.sparse_canon)
    S_f = np.einsum("sk,ska->sa", beta, t[ids_s])
    e_sparse = float(np.sum((S_f - cons.sparse_target) ** 2))
    src, dst = arap_edges(grid)
    keep = act[src] & act[dst]
    src, dst = src[keep], dst[keep]
    rest = grid.rest_positions()
    rot_e = np.einsum("eab,eb->ea", R[src], rest[src] - rest[dst])
    e_reg = float(np.sum(((t[src] - t[dst]) - rot_e) ** 2))
    wd, ws, wr = cons.w_dense * e_dense, cons.w_sparse * e_sparse, cons.w_arap * e_reg
    return (wd + ws + wr, wd, ws, wr)


def rotation_step_active(grid: Grid, t: np.ndarray, R: np.ndarray, act: np.ndarray):
    """Procrustes fit (Sec. 7.1) of every point of M over its one-ring points
    in M (the terms of eq. (4) that depend on R_i); points outside M keep
    their rotation."""
    src, dst = arap_edges(grid)
    rest = grid.rest_positions()
    keep = act[src] & act[dst]
    src, dst = src[keep], dst[keep]
    M = np.zeros((grid.n, 3, 3))
    np.add.at(M, src, np.einsum("ea,eb->eab", t[src] - t[dst], rest[src] - rest[dst]))
    out = R.copy()
    idx = np.flatnonzero(act)
    if idx.size:
        out[idx], _ = fit_rotations(M[idx], R[idx])
    return out


def grow(grid: Grid, t: np.ndarray, R: np.ndarray, act: np.ndarray, prev: np.ndarray):
    """Reading M5: extrapolate the points of `act` missing from `prev`, layer
    by layer.  Returns (t, R, layers)."""
    t = t.copy()
    R = R.copy()
    rest = grid.rest_positions()
    d = t - rest
    known = prev.copy()
    todo = act & ~prev
    nx, ny, nz = grid.dims
    coords = grid.coords()
    layers = 0
    while True:
        cand = np.flatnonzero(todo & ~known)
        fill = []
        for i in cand:
            a, b, c = coords[i]
            acc = np.zeros(3)
            cnt = 0
            rot = None
            for (dx, dy, dz) in _STEPS:
                x, y, z = a + dx, b + dy, c + dz
                if 0 <= x < nx and 0 <= y < ny and 0 <= z < nz:
                    j = x + nx * (y + ny * z)
                    if known[j]:
                        acc = acc + d[j]
                        cnt += 1
                        if rot is None:
                            rot = R[j]
            if cnt:
                fill.append((i, acc / cnt, rot))
        if not fill:
            break
        for i, di, Ri in fill:
            d[i] = di
            R[i] = Ri
            known[i] = True
        layers += 1
    return rest + d, R, layers


def solve_frame_active(scene, state=None, prev_active: Optional[np.ndarray] = None,
                       mode: str = "replica", trace: Optional[List] = None,
                       gn_iters=None, pcg_iters=None) -> Dict:
    """One frame of the solve restricted to M (readings M1-M5), from `state`
    ((t, R) of the finest level; None: rest).  `prev_active` is the finest
    level's M of the previous frame (None: no grid growth).  Returns the new
    finest state, its energy (over M), the finest M and the number of growth
    layers."""
    spec = scene.spec
    grids = level_grids(spec.dims, spec.spacing, spec.origin, spec.num_levels)
    L = len(grids)
    cons = prepare_constraints(scene, grids[0])
    finest = grids[-1]
    if state is None:
        tF, RF = rest_state(finest)
    else:
        tF = np.asarray(state[0], np.float64).reshape(-1, 3)
        RF = np.asarray(state[1], np.float64).reshape(-1, 3, 3)
    acts = [active_set(g, cons) for g in grids]
    layers = 0
    if prev_active is not None:
        tF, RF, layers = grow(finest, tF, RF, acts[-1], np.asarray(prev_active, bool))
    gn = gn_iters if gn_iters is not None else spec.gn_iters
    pc = pcg_iters if pcg_iters is not None else spec.pcg_iters
    prev = None
    t = R = None
    for lvl, grid in enumerate(grids):
        act = acts[lvl]
        stride = 2 ** (L - 1 - lvl)
        base = inject(finest, tF, grid, stride)
        t = base.copy()
        R = inject(finest, RF, grid, stride)
        if prev is not None:
            pg, p_base, p_final = prev
            inc = prolong(pg, p_final - p_base, grid)
            t[act] = t[act] + inc[act]
            R = rotation_step_active(grid, t, R, act)
        system = ActiveSystem(grid, cons, act)
        for _ in range(gn[lvl]):
            t = system.position_step(t, R, mode, pc[lvl])
            if trace is not None:
                trace.append(("pos", lvl, energy_terms_active(grid, t, R, cons, act)[0]))
            R = rotation_step_active(grid, t, R, act)
            if trace is not None:
                trace.append(("rot", lvl, energy_terms_active(grid, t, R, cons, act)[0]))
        prev = (grid, base, t)
    # points of the finest level outside M keep the state the frame started from
    E = energy_terms_active(finest, t, R, cons, acts[-1])
    return {"t": t, "R": R, "energy": E, "grid": finest, "active": acts[-1], "layers": layers}
