"""The rotation half of the flip-flop, Sec. 7.1 (Procrustes / shape matching).

Part of the FP64 CPU oracle -- test infrastructure only.

With positions fixed, R_i appears only in the eq. (4) terms whose first index
is i: sum_{j in N_i} ||(t_i - t_j) - R_i e_ij||^2 with e_ij = t_hat_i - t_hat_j.
Minimising it over rotations is the orthogonal Procrustes problem: maximise
trace(R^T M_i) for the cross-covariance M_i = sum_j (t_i - t_j) e_ij^T.  With
M_i = U Sigma V^T (singular values descending) the minimiser in SO(3) is
R_i = U diag(1, 1, d) V^T, d = sign(det(U V^T)).

Reading: the paper does not say how reflections are handled; the determinant
correction above is the standard one.  When rank(M_i) <= 1 (sigma_2 <= 1e-12
sigma_1) the minimiser is not unique and the previous R_i is kept.
"""

from __future__ import annotations

import numpy as np

from .lattice import Grid, arap_edges

DEGENERATE_RATIO = 1e-12


def cross_covariance(grid: Grid, t: np.ndarray) -> np.ndarray:
    """M_i = sum_{j in N_i} (t_i - t_j)(t_hat_i - t_hat_j)^T, shape (N,3,3)."""
    src, dst = arap_edges(grid)
    rest = grid.rest_positions()
    outer = np.einsum("ea,eb->eab", t[src] - t[dst], rest[src] - rest[dst])
    M = np.zeros((grid.n, 3, 3))
    np.add.at(M, src, outer)
    return M


def fit_rotations(M: np.ndarray, R_prev: np.ndarray | None = None):
    """Best rotations for a batch of cross-covariances (K,3,3).  Returns
    (R, degenerate mask); degenerate entries take R_prev (or I)."""
    U, s, Vt = np.linalg.svd(M)
    d = np.sign(np.linalg.det(U @ Vt))
    d = np.where(d == 0, 1.0, d)
    D = np.zeros_like(M)
    D[:, 0, 0] = 1.0
    D[:, 1, 1] = 1.0
    D[:, 2, 2] = d
    R = U @ D @ Vt
    degenerate = ~(s[:, 1] > DEGENERATE_RATIO * s[:, 0])
    if np.any(degenerate):
        fallback = (np.broadcast_to(np.eye(3), M.shape) if R_prev is None else R_prev)
        R = np.where(degenerate[:, None, None], fallback, R)
    return R, degenerate


def rotation_step(grid: Grid, t: np.ndarray, R_prev: np.ndarray) -> np.ndarray:
    R, _ = fit_rotations(cross_covariance(grid, t), R_prev)
    return R
