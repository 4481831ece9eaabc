"""The deformation energy of Sec. 6, eqs. (1)-(4), and its Jacobian.

Part of the FP64 CPU oracle -- test infrastructure only.

E_total = w_s E_sparse + w_d E_dense + w_r E_reg                     (eq. 1)
E_dense = sum_c w_c [ (S(p_hat_c) - p_c)^T n_c ]^2                   (eq. 2)
E_sparse = sum_s || S(f_hat_s) - f_s ||^2                            (eq. 3)
E_reg = sum_i sum_{j in N_i} || (t_i - t_j) - R_i (t_hat_i - t_hat_j) ||^2   (eq. 4)

with S(x) = sum_k alpha_k(x) t_k (Sec. 4; the global rigid motion is the
identity on this path).  The energy is a plain sum with no factor 1/2, and
every undirected lattice edge enters E_reg twice (once from each end).

Stacking the square roots of the weighted terms into a residual vector r gives
E = r^T r with r = J t - c(R): J is constant (it does not depend on R) and the
rotations enter only the constant c.  The unknown vector is t flattened as
(N,3) -> 3 i + axis.  Residual rows are ordered: dense (C), sparse (3 S, one
per axis), ARAP (3 per directed edge).

Readings: the set M of optimised points is the whole lattice; N_i is the
6-neighbourhood; w_c is an input weight (1 for the synthetic workloads).
Normals are renormalised on input and a zero normal gets weight 0.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .lattice import Grid, arap_edges, inside, trilinear


@dataclass
class Constraints:
    canon: np.ndarray          # (C,3) p_hat
    target: np.ndarray         # (C,3) p^a
    normal: np.ndarray         # (C,3) n^a, unit length
    weight: np.ndarray         # (C,)  w_c
    sparse_canon: np.ndarray   # (S,3) f_hat
    sparse_target: np.ndarray  # (S,3) f
    w_dense: float
    w_sparse: float
    w_arap: float


def prepare_constraints(scene, coarsest: Grid | None = None) -> Constraints:
    """Promote a scene's inputs to float64, renormalise normals (zero normal ->
    weight 0) and validate them.  Raises ValueError for non-finite values,
    negative weights, or samples outside the coarsest lattice."""
    spec = scene.spec
    canon = np.asarray(scene.canon, np.float64).reshape(-1, 3)
    target = np.asarray(scene.target, np.float64).reshape(-1, 3)
    normal = np.asarray(scene.normal, np.float64).reshape(-1, 3)
    weight = (np.ones(canon.shape[0]) if scene.weight is None
              else np.asarray(scene.weight, np.float64).reshape(-1))
    sc = np.asarray(scene.sparse_canon, np.float64).reshape(-1, 3)
    st = np.asarray(scene.sparse_target, np.float64).reshape(-1, 3)
    for a in (canon, target, normal, weight, sc, st):
        if not np.all(np.isfinite(a)):
            raise ValueError("non-finite constraint value")
    if np.any(weight < 0):
        raise ValueError("negative weight")
    for wv in (spec.w_dense, spec.w_sparse, spec.w_arap):
        if not (np.isfinite(wv) and wv >= 0):
            raise ValueError("bad energy weight")
    ln = np.linalg.norm(normal, axis=1)
    weight = np.where(ln > 0, weight, 0.0)
    normal = normal / np.where(ln > 0, ln, 1.0)[:, None]
    if coarsest is not None:
        if not (np.all(inside(coarsest, canon)) and np.all(inside(coarsest, sc))):
            raise ValueError("sample outside the coarsest lattice")
    return Constraints(canon, target, normal, weight, sc, st,
                       float(spec.w_dense), float(spec.w_sparse), float(spec.w_arap))


class Assembled:
    """J (csr), the R-independent constants and the edge list of one level."""

    def __init__(self, grid: Grid, cons: Constraints):
        self.grid = grid
        n3 = 3 * grid.n
        C = cons.canon.shape[0]
        S = cons.sparse_canon.shape[0]
        rows, cols, vals = [], [], []
        # dense point-to-plane rows, eq. (2): sqrt(w_d w_c) n^T sum_k alpha_k t_k
        ids, alpha = trilinear(grid, cons.canon)
        s = np.sqrt(cons.w_dense * cons.weight)
        for k in range(8):
            for a in range(3):
                rows.append(np.arange(C))
                cols.append(3 * ids[:, k] + a)
                vals.append(s * alpha[:, k] * cons.normal[:, a])
        self.c_dense = s * np.einsum("ca,ca->c", cons.normal, cons.target)
        # sparse point-to-point rows, eq. (3): sqrt(w_s) (sum_k beta_k t_k)_a
        ids_s, beta = trilinear(grid, cons.sparse_canon)
        ss = np.sqrt(cons.w_sparse)
        for k in range(8):
            for a in range(3):
                rows.append(C + 3 * np.arange(S) + a)
                cols.append(3 * ids_s[:, k] + a)
                vals.append(np.full(S, ss) * beta[:, k])
        self.c_sparse = ss * cons.sparse_target.reshape(-1)
        # ARAP rows, eq. (4): sqrt(w_r) (t_i - t_j)_a for every directed edge
        src, dst = arap_edges(grid)
        E = src.size
        base = C + 3 * S
        sr = np.sqrt(cons.w_arap)
        for a in range(3):
            r = base + 3 * np.arange(E) + a
            rows += [r, r]
            cols += [3 * src + a, 3 * dst + a]
            vals += [np.full(E, sr), np.full(E, -sr)]
        nrows = base + 3 * E
        self.J = sp.csr_matrix(
            (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
            shape=(nrows, n3))
        self.src, self.dst = src, dst
        rest = grid.rest_positions()
        self.e = rest[src] - rest[dst]          # t_hat_i - t_hat_j per edge
        self.sqrt_wr = sr
        self.rows = (C, 3 * S, 3 * E)

    def constant(self, R: np.ndarray) -> np.ndarray:
        """c(R): the targets and the rotated rest edges sqrt(w_r) R_i e_ij."""
        rot_e = np.einsum("eab,eb->ea", R[self.src], self.e)
        return np.concatenate([self.c_dense, self.c_sparse,
                               self.sqrt_wr * rot_e.reshape(-1)])

    def residual(self, t: np.ndarray, R: np.ndarray) -> np.ndarray:
        return self.J @ t.reshape(-1) - self.constant(R)


def assemble(grid: Grid, cons: Constraints) -> Assembled:
    return Assembled(grid, cons)


def residual_direct(grid: Grid, t: np.ndarray, R: np.ndarray, cons: Constraints) -> np.ndarray:
    """The residual vector evaluated straight from eqs. (2)-(4) by gathering
    node positions (no matrix), in the same row order as Assembled."""
    ids, alpha = trilinear(grid, cons.canon)
    S_p = np.einsum("ck,cka->ca", alpha, t[ids])
    r_dense = np.sqrt(cons.w_dense * cons.weight) * np.einsum(
        "ca,ca->c", S_p - cons.target, cons.normal)
    ids_s, beta = trilinear(grid, cons.sparse_canon)
    S_f = np.einsum("sk,ska->sa", beta, t[ids_s])
    r_sparse = np.sqrt(cons.w_sparse) * (S_f - cons.sparse_target).reshape(-1)
    src, dst = arap_edges(grid)
    rest = grid.rest_positions()
    rot_e = np.einsum("eab,eb->ea", R[src], rest[src] - rest[dst])
    r_arap = np.sqrt(cons.w_arap) * ((t[src] - t[dst]) - rot_e).reshape(-1)
    return np.concatenate([r_dense, r_sparse, r_arap])


def energy_terms(grid: Grid, t: np.ndarray, R: np.ndarray, cons: Constraints):
    """(E_total, w_d E_dense, w_s E_sparse, w_r E_reg), eq. (1), evaluated from
    the definitions eqs. (2)-(4)."""
    ids, alpha = trilinear(grid, cons.canon)
    S_p = np.einsum("ck,cka->ca", alpha, t[ids])
    e_dense = float(np.sum(cons.weight * np.einsum("ca,ca->c", S_p - cons.target, cons.normal) ** 2))
    ids_s, beta = trilinear(grid, cons.sparse_canon)
    S_f = np.einsum("sk,ska->sa", beta, t[ids_s])
    e_sparse = float(np.sum((S_f - cons.sparse_target) ** 2))
    src, dst = arap_edges(grid)
    rest = grid.rest_positions()
    rot_e = np.einsum("eab,eb->ea", R[src], rest[src] - rest[dst])
    e_reg = float(np.sum(((t[src] - t[dst]) - rot_e) ** 2))
    wd, ws, wr = cons.w_dense * e_dense, cons.w_sparse * e_sparse, cons.w_arap * e_reg
    return (wd + ws + wr, wd, ws, wr)
