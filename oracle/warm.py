"""FP64 reference of the warm-start input features (not part of the paper).

Part of the CPU oracle -- test infrastructure only.

For the coming frame k, each node i of the finest lattice gets 8 channels,
all lengths divided by the node spacing h:
  0-2  t_i^{k-1} - t_hat_i   (the previous frame's solved displacement)
  3-5  t_i^{k-1} - t_i^{k-2}  (its change from the frame before: the same
       information as that frame's displacement, encoded as a difference so
       that a small motion survives rounding to bfloat16)
  6    sum_c alpha_ci w_c r_c / sum_c alpha_ci w_c, with the point-to-plane
       residual r_c = n_c . (S(p_hat_c) - p_c) of eq. (2) evaluated at the
       plain initialisation t^{k-1}, the trilinear weights alpha of Sec. 4 and
       w_c = w_d times the sample weight (0 where the denominator is 0)
  7    1 where that denominator is > 0, else 0
"""

from __future__ import annotations

import numpy as np

from .energy import Assembled, Constraints
from .lattice import Grid, trilinear


def features(grid: Grid, cons: Constraints, t_prev: np.ndarray, t_prev2=None) -> np.ndarray:
    """(N, 8) features; t_prev, t_prev2 are (N, 3) node positions (t_prev2
    None: the same as t_prev)."""
    rest = grid.rest_positions()
    t_prev = np.asarray(t_prev, np.float64).reshape(-1, 3)
    t_prev2 = t_prev if t_prev2 is None else np.asarray(t_prev2, np.float64).reshape(-1, 3)
    out = np.zeros((grid.n, 8))
    out[:, 0:3] = (t_prev - rest) / grid.h
    out[:, 3:6] = (t_prev - t_prev2) / grid.h
    ids, alpha = trilinear(grid, cons.canon)
    warped = np.einsum("ck,cka->ca", alpha, t_prev[ids])          # S(p_hat_c)
    res = np.einsum("ca,ca->c", cons.normal, warped - cons.target)  # eq. (2) residual
    w = cons.w_dense * cons.weight
    num = np.zeros(grid.n)
    den = np.zeros(grid.n)
    for k in range(8):
        np.add.at(num, ids[:, k], alpha[:, k] * w * res)
        np.add.at(den, ids[:, k], alpha[:, k] * w)
    valid = den > 0
    out[valid, 6] = num[valid] / den[valid] / grid.h
    out[:, 7] = valid.astype(np.float64)
    return out


def exact_step(asm: Assembled, t: np.ndarray, R: np.ndarray, delta: np.ndarray):
    """Minimiser along a direction of the energy at fixed rotations.  With R
    fixed, E(t) = |J t - c(R)|^2 is quadratic in the positions (Sec. 7.1), so
    E(t + s v) = E(t) + 2 s g.v + s^2 |J v|^2 with g = J^T r(t), and its
    minimiser along v is s* = -g.v / |J v|^2 (0 when |J v| = 0).  t, delta:
    (N, 3); returns (s*, t + s* delta)."""
    t = np.asarray(t, np.float64).reshape(-1, 3)
    v = np.asarray(delta, np.float64).reshape(-1)
    g = asm.J.T @ asm.residual(t, R)
    Jv = asm.J @ v
    den = float(Jv @ Jv)
    s = -float(g @ v) / den if den > 0.0 else 0.0
    return s, t + s * v.reshape(-1, 3)
