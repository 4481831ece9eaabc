"""Shared helpers of the test suite: run the oracle and the GPU library on the
same seeded scene and compare."""

from __future__ import annotations

import numpy as np

import oracle
from oracle.energy import prepare_constraints
from oracle.lattice import level_grids


def grids_of(scene):
    s = scene.spec
    return level_grids(s.dims, s.spacing, s.origin, s.num_levels)


def oracle_cons(scene):
    return prepare_constraints(scene, grids_of(scene)[0])


def random_state(grid, rng, amp=0.3, rot_amp=0.3):
    """Positions rest + amp*h*N(0,1) and rotations exp(rot_amp * N(0,1) axis)."""
    pos = grid.rest_positions() + amp * grid.h * rng.normal(size=(grid.n, 3))
    w = rot_amp * rng.normal(size=(grid.n, 3))
    th = np.linalg.norm(w, axis=1, keepdims=True)
    k = w / np.maximum(th, 1e-30)
    K = np.zeros((grid.n, 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -k[:, 2], k[:, 1]
    K[:, 1, 0], K[:, 1, 2] = k[:, 2], -k[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -k[:, 1], k[:, 0]
    s, c = np.sin(th)[..., None], np.cos(th)[..., None]
    R = np.eye(3)[None] + s * K + (1 - c) * (K @ K)
    return pos.astype(np.float32), R.astype(np.float32)


def rel_err(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rotation_angle(Ra, Rb):
    """Angle (rad) of Ra^T Rb per node, as atan2(|skew part|, (trace-1)/2):
    unlike arccos((trace-1)/2) it stays accurate for tiny angles."""
    Ra = np.asarray(Ra, np.float64)
    Rb = np.asarray(Rb, np.float64)
    M = np.einsum("nba,nbc->nac", Ra, Rb)
    w = 0.5 * np.stack([M[:, 2, 1] - M[:, 1, 2], M[:, 0, 2] - M[:, 2, 0],
                        M[:, 1, 0] - M[:, 0, 1]], axis=1)
    c = 0.5 * (np.trace(M, axis1=1, axis2=2) - 1.0)
    return np.arctan2(np.linalg.norm(w, axis=1), c)


def make_lattice(scene, **kw):
    from paper_1603_08161_amd import Lattice
    lat = Lattice.from_spec(scene.spec, **kw)
    lat.set_scene(scene)
    return lat


def oracle_solve(scene, **kw):
    return oracle.solve_frame(scene, **kw)


def edge_fit_cases(seed, n=600):
    """Cross-covariances (float32-representable, as float64) that drive the
    rotation fit's Jacobi sweeps to their edge branches, with previous
    rotations: a third nearly diagonal (distinct diagonal magnitudes about
    3, 2, 1 with random signs, off-diagonal entries 1e-6 down to 1e-33 of the
    diagonal: tiny rotation angles, |theta| far beyond 1e15, entries too small
    to rotate), a third random scaled by 1e-15 and a third by 1e15.  The
    previous rotation is the identity for even cases and a half turn about z
    for odd ones (a different basis of the warm start)."""
    rng = np.random.default_rng(seed)
    k = n // 3
    M = np.empty((n, 3, 3))
    mag = np.array([3.0, 2.0, 1.0]) * (1.0 + 0.1 * rng.uniform(-1, 1, size=(k, 3)))
    mag = np.take_along_axis(mag, np.argsort(rng.uniform(size=(k, 3)), axis=1), axis=1)
    diag = mag * rng.choice([-1.0, 1.0], size=(k, 3))
    rel = 10.0 ** rng.uniform(-33, -6, size=(k, 1, 1))
    M[:k] = rng.normal(size=(k, 3, 3)) * rel + diag[:, :, None] * np.eye(3)
    M[k:2 * k] = rng.normal(size=(k, 3, 3)) * 1e-15
    M[2 * k:] = rng.normal(size=(n - 2 * k, 3, 3)) * 1e15
    Rp = np.broadcast_to(np.eye(3), (n, 3, 3)).copy()
    Rp[1::2] = np.diag([-1.0, -1.0, 1.0])
    return M.astype(np.float32).astype(np.float64), Rp
