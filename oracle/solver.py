"""The flip-flop solve of Sec. 7: position steps by the normal equations,
rotation steps by Procrustes, over the nested hierarchy of Sec. 7.2.

Part of the FP64 CPU oracle -- test infrastructure only.

Position step (Sec. 7.1).  With rotations fixed, E = ||J t - c(R)||^2 is
quadratic in t.  Setting its gradient to zero gives the normal equations
A t = J^T c with A = J^T J (the paper's L + B^T B; its L is the ARAP block
2 w_r (graph Laplacian x I_3) and B the weighted constraint rows).  Written as
an increment from the current t: A delta = -g with g = J^T (J t - c).
  * mode "direct": A is factorised (SuperLU) and the step is exact.
  * mode "replica": the data-parallel solver the paper runs, preconditioned
    CG, here with the Jacobi preconditioner D = diag(A), delta_0 = 0 and a fixed
    iteration count.  Readings: the preconditioner is not named in the paper;
    a zero denominator gives a zero step size (alpha = 0 if p^T A p <= 0,
    beta = 0 if r^T z of the previous iterate is <= 0).

Rotation step: ``procrustes.rotation_step``.

Flip-flop order (Sec. 7.1): positions first, then rotations, repeated for a
fixed number of iterations per level (the paper iterates to convergence; the
counts come from the workload's schedule).

Hierarchy (Sec. 7.2), coarse -> fine.  Readings: levels are vertex-nested
(coarse node j = fine node 2 j); each level starts from the finest state
injected to it; from the second level on, the increment of the previous
level's result over the finest state injected there is prolongated (trilinear
evaluation at the finer rest positions, linear extrapolation past the last
coarse node) and added, and the rotations are then refitted by one Procrustes
step.  Constraints are re-expressed on every level by trilinear weights of the
coarser grid.
"""

from __future__ import annotations

from typing import Dict, List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .energy import Assembled, assemble, energy_terms, prepare_constraints
from .lattice import Grid, level_grids, trilinear
from .procrustes import rotation_step


def jacobi_diag(J: sp.csr_matrix) -> np.ndarray:
    """diag(J^T J): the squared column norms of J."""
    return np.asarray(J.multiply(J).sum(axis=0)).ravel()


def pcg(A, b: np.ndarray, dinv: np.ndarray, iters: int, trace=None) -> np.ndarray:
    """Jacobi-preconditioned conjugate gradient on A x = b from x = 0, a fixed
    number of iterations, with the zero-denominator guards described above."""
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    for _ in range(iters):
        q = A @ p
        pq = float(p @ q)
        alpha = rz / pq if pq > 0 else 0.0
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = float(r @ z)
        beta = rz_new / rz if rz > 0 else 0.0
        p = z + beta * p
        rz = rz_new
        if trace is not None:
            trace.append(x.copy())
    return x


class LevelSystem:
    """J, A = J^T J and D^-1 of one level; A does not depend on R."""

    def __init__(self, grid: Grid, cons):
        self.grid = grid
        self.asm: Assembled = assemble(grid, cons)
        self.A = (self.asm.J.T @ self.asm.J).tocsr()
        d = jacobi_diag(self.asm.J)
        self.dinv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
        self._lu = None

    def gradient(self, t: np.ndarray, R: np.ndarray) -> np.ndarray:
        """g = J^T r, so that E(t + delta) = E + 2 g^T delta + delta^T A delta."""
        return self.asm.J.T @ self.asm.residual(t, R)

    def solve(self, b: np.ndarray, mode: str, iters: int) -> np.ndarray:
        if mode == "direct":
            if self._lu is None:
                self._lu = spla.splu(self.A.tocsc(), permc_spec="COLAMD")
            return self._lu.solve(b)
        if mode == "replica":
            return pcg(self.A, b, self.dinv, iters)
        raise ValueError(mode)


def position_step(system: LevelSystem, t: np.ndarray, R: np.ndarray,
                  mode: str = "replica", iters: int = 10) -> np.ndarray:
    g = system.gradient(t, R)
    delta = system.solve(-g, mode, iters)
    return t + delta.reshape(-1, 3)


def inject(fine: Grid, values: np.ndarray, coarse: Grid, stride: int) -> np.ndarray:
    """Sample a per-node field of the fine grid at the coarse nodes, coarse
    node (a,b,c) = fine node stride * (a,b,c)."""
    cc = coarse.coords() * stride
    return values[fine.node_id(cc[:, 0], cc[:, 1], cc[:, 2])]


def prolong(coarse: Grid, values: np.ndarray, fine: Grid) -> np.ndarray:
    """Trilinear evaluation of a coarse per-node field at the fine rest
    positions (linear extrapolation beyond the last coarse node)."""
    ids, w = trilinear(coarse, fine.rest_positions())
    return np.einsum("nk,nka->na", w, values[ids])


def rest_state(grid: Grid):
    return grid.rest_positions(), np.broadcast_to(np.eye(3), (grid.n, 3, 3)).copy()


def solve_frame(scene, state=None, mode: str = "replica", trace: List | None = None,
                gn_iters=None, pcg_iters=None) -> Dict:
    """One frame of the solve.  ``state`` = (t, R) at the finest level (the
    previous frame's result); None starts at rest.  Returns the new finest
    state and the energy terms at it."""
    spec = scene.spec
    grids = level_grids(spec.dims, spec.spacing, spec.origin, spec.num_levels)
    L = len(grids)
    cons = prepare_constraints(scene, grids[0])
    finest = grids[-1]
    if state is None:
        tF, RF = rest_state(finest)
    else:
        tF, RF = (np.asarray(state[0], np.float64).reshape(-1, 3),
                  np.asarray(state[1], np.float64).reshape(-1, 3, 3))
    gn = gn_iters if gn_iters is not None else spec.gn_iters
    pc = pcg_iters if pcg_iters is not None else spec.pcg_iters
    prev = None  # (grid, injected finest state, final state) of the previous level
    for lvl, grid in enumerate(grids):
        stride = 2 ** (L - 1 - lvl)
        base = inject(finest, tF, grid, stride)
        t = base.copy()
        R = inject(finest, RF, grid, stride)
        if prev is not None:
            pg, p_base, p_final = prev
            t = t + prolong(pg, p_final - p_base, grid)
            R = rotation_step(grid, t, R)
        system = LevelSystem(grid, cons)
        for _ in range(gn[lvl]):
            t = position_step(system, t, R, mode, pc[lvl])
            if trace is not None:
                trace.append(("pos", lvl, energy_terms(grid, t, R, cons)[0]))
            R = rotation_step(grid, t, R)
            if trace is not None:
                trace.append(("rot", lvl, energy_terms(grid, t, R, cons)[0]))
        prev = (grid, base, t)
    E = energy_terms(finest, t, R, cons)
    return {"t": t, "R": R, "energy": E, "grid": finest}
