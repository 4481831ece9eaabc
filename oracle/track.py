"""Association of a lattice's model samples (Sec. 5.1 on the deformation of
Sec. 4) and the lattice solve with the association repeated ICP-style
(Sec. 3).

Part of the FP64 CPU oracle -- test infrastructure only.

Model samples are canonical positions p_hat_c with canonical normals n_hat_c
(the rasterised isosurface of Sec. 5.1).  From a lattice state with node
displacements d_i = t_i - t_hat_i and rotations R_i, and the global pose
(R, t):
  p_c = R (p_hat_c + sum_k alpha_k d_k) + t      (S(p_hat_c) = sum_k alpha_k t_k,
                                                   with sum_k alpha_k t_hat_k = p_hat_c)
  n_c = R sum_k alpha_k R_k n_hat_c               (reading A4 of ``assoc``)
are associated as in ``assoc.associate``; targets and normals are brought
back to the lattice frame (R^T (p^a - t), R^T n^a), where the lattice solve
works (the energy is invariant under the rigid pose).  The sums run over the
corners k = dx + 2 dy + 4 dz in that order, as written here.

One tracked frame (Sec. 3): repeat `icp_iters` times -- associate from the
current state, replace the dense constraints by the associated pairs (weights
w_c, pruned pairs weight 0) and the frame's sparse pairs (targets
R^T (f - t)), and run the flip-flop schedule of Sec. 7 from the current
state.  The association outputs enter the solve as float32, the precision of
the constraint interface.
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from . import assoc
from .lattice import Grid, cell_and_frac, CORNERS
from .solver import level_grids, rest_state, solve_frame


class _Constraints:
    """A scene-like record of constraints for ``solver.solve_frame``."""

    def __init__(self, spec, canon, target, normal, weight, sparse_canon, sparse_target):
        self.spec = spec
        self.canon = canon
        self.target = target
        self.normal = normal
        self.weight = weight
        self.sparse_canon = sparse_canon
        self.sparse_target = sparse_target


def deform_samples(grid: Grid, disp: np.ndarray, rot: np.ndarray, canon: np.ndarray,
                   cnormal: np.ndarray, pose: np.ndarray):
    """Camera-frame positions and normals of the model samples (see above).
    disp (N,3), rot (N,3,3), canon / cnormal (M,3), pose (12,)."""
    x = np.asarray(canon, np.float64).reshape(-1, 3)
    nh = np.asarray(cnormal, np.float64).reshape(-1, 3)
    d = np.asarray(disp, np.float64).reshape(-1, 3)
    Rn = np.asarray(rot, np.float64).reshape(-1, 3, 3)
    cell, f = cell_and_frac(grid, x)
    s = np.zeros_like(x)
    nc = np.zeros_like(x)
    for (dx, dy, dz) in CORNERS:
        wx = f[:, 0] if dx else 1.0 - f[:, 0]
        wy = f[:, 1] if dy else 1.0 - f[:, 1]
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        a = wx * wy * wz
        ids = grid.node_id(cell[:, 0] + dx, cell[:, 1] + dy, cell[:, 2] + dz)
        for r in range(3):
            s[:, r] += a * d[ids, r]
            Rr = Rn[ids, r]
            nc[:, r] += a * (Rr[:, 0] * nh[:, 0] + Rr[:, 1] * nh[:, 1] + Rr[:, 2] * nh[:, 2])
    p = x + s
    P = np.asarray(pose, np.float64).reshape(12)
    q = np.empty_like(p)
    nq = np.empty_like(p)
    for r in range(3):
        q[:, r] = P[3 * r] * p[:, 0] + P[3 * r + 1] * p[:, 1] + P[3 * r + 2] * p[:, 2] + P[9 + r]
        nq[:, r] = P[3 * r] * nc[:, 0] + P[3 * r + 1] * nc[:, 1] + P[3 * r + 2] * nc[:, 2]
    return q, nq


def to_model_frame(x: np.ndarray, pose: np.ndarray) -> np.ndarray:
    """R^T (x - t) for camera-frame points x (M,3)."""
    P = np.asarray(pose, np.float64).reshape(12)
    x = np.asarray(x, np.float64).reshape(-1, 3)
    dx = x - P[9:12][None, :]
    out = np.empty_like(dx)
    for r in range(3):
        out[:, r] = P[r] * dx[:, 0] + P[3 + r] * dx[:, 1] + P[6 + r] * dx[:, 2]
    return out


def lattice_associate(grid: Grid, disp, rot, frame: Dict, prm: assoc.AssocParams):
    """(target, normal) in the lattice frame, weights and pixels of the
    frame's model samples at the lattice state (disp, rot)."""
    cam = assoc.Camera(**frame["camera"])
    pose = np.asarray(frame.get("pose", _identity_pose()), np.float64)
    q, nq = deform_samples(grid, disp, rot, frame["model_canon"], frame["model_normal"], pose)
    pa, na, w, px = assoc.associate(cam, frame["depth"], q, nq, prm)
    keep = w > 0.0
    tl = np.zeros_like(pa)
    nl = np.zeros_like(na)
    tl[keep] = to_model_frame(pa[keep], pose)
    nl[keep] = to_model_frame(na[keep], np.concatenate([pose[:9], np.zeros(3)]))
    return tl, nl, w, px


def _identity_pose():
    return np.concatenate([np.eye(3).ravel(), np.zeros(3)])


def solve_frame_icp(spec, frame: Dict, prm: assoc.AssocParams, icp_iters: int,
                    state=None, history: Optional[List] = None):
    """One tracked frame (see above) from `state` ((t, R) of the finest level,
    None: rest).  Returns the ``solver.solve_frame`` result of the last solve."""
    grids = level_grids(spec.dims, spec.spacing, spec.origin, spec.num_levels)
    finest = grids[-1]
    if state is None:
        t, R = rest_state(finest)
    else:
        t = np.asarray(state[0], np.float64).reshape(-1, 3)
        R = np.asarray(state[1], np.float64).reshape(-1, 3, 3)
    pose = np.asarray(frame.get("pose", _identity_pose()), np.float64)
    sc = frame.get("sparse_canon")
    if sc is None:
        sc = np.zeros((0, 3), np.float32)
        st = np.zeros((0, 3), np.float32)
    else:
        st = to_model_frame(frame["sparse_target"], pose).astype(np.float32)
    out = None
    for _ in range(icp_iters):
        tl, nl, w, _ = lattice_associate(finest, t - finest.rest_positions(), R, frame, prm)
        cons = _Constraints(spec, np.asarray(frame["model_canon"], np.float32),
                            tl.astype(np.float32), nl.astype(np.float32), w.astype(np.float32),
                            np.asarray(sc, np.float32), st)
        out = solve_frame(cons, state=(t, R))
        t, R = out["t"], out["R"]
        if history is not None:
            history.append((np.array(out["energy"], np.float64), int(np.count_nonzero(w))))
    return out


def track_frame(spec, frame: Dict, prm: assoc.AssocParams, rigid_iters: int, icp_iters: int,
                state=None, pose=None, history: Optional[List] = None):
    """One tracked frame with the global pose found first (Sec. 6): the
    model samples deformed by the lattice state (in the lattice frame) run
    `rigid_iters` projective ICP iterations from `pose` (12 floats, R
    row-major then t; None: identity), then ``solve_frame_icp`` runs with
    that pose.  Returns (solve result, pose, rigid-ICP history)."""
    grids = level_grids(spec.dims, spec.spacing, spec.origin, spec.num_levels)
    finest = grids[-1]
    if state is None:
        t, R = rest_state(finest)
    else:
        t = np.asarray(state[0], np.float64).reshape(-1, 3)
        R = np.asarray(state[1], np.float64).reshape(-1, 3, 3)
    P = _identity_pose() if pose is None else np.asarray(pose, np.float64).reshape(12)
    cam = assoc.Camera(**frame["camera"])
    q, nq = deform_samples(finest, t - finest.rest_positions(), R, frame["model_canon"],
                           frame["model_normal"], _identity_pose())
    Rg, tg, hist = assoc.rigid_pose(cam, frame["depth"], q, nq, prm, rigid_iters,
                                    P[:9].reshape(3, 3), P[9:])
    P = np.concatenate([Rg.ravel(), tg])
    out = solve_frame_icp(spec, dict(frame, pose=P), prm, icp_iters, state=(t, R),
                          history=history)
    return out, P, hist
