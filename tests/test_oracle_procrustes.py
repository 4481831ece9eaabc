"""Pins of the oracle's rotation step (Sec. 7.1, Procrustes via SVD):

* no rotation from a dense random sample of SO(3), refined by local search,
  beats the SVD answer on trace(R^T M);
* Horn's closed-form unit-quaternion method (an independent algorithm: the
  dominant eigenvector of a 4x4 symmetric matrix) gives the same rotation;
* rest pose gives the identity, a rigid motion gives its rotation, the ARAP
  objective never increases, a rank-1 covariance keeps the previous rotation."""

import numpy as np
import pytest

from oracle.lattice import Grid
from oracle.procrustes import cross_covariance, fit_rotations, rotation_step
from oracle.energy import prepare_constraints, energy_terms
from synth import make_tiny, random_rotation


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def _horn(M):
    """Rotation maximising trace(R^T M), M = sum target source^T (Horn 1987)."""
    S = M.T  # sum source target^T
    Sxx, Sxy, Sxz = S[0]
    Syx, Syy, Syz = S[1]
    Szx, Szy, Szz = S[2]
    N = np.array([
        [Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx],
        [Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz],
        [Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy],
        [Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz]])
    wv, V = np.linalg.eigh(N)
    return _quat_to_rot(V[:, -1])


def _random_rotations(rng, k):
    q = rng.normal(size=(k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = w * w + x * x - y * y - z * z
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = w * w - x * x + y * y - z * z
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = w * w - x * x - y * y + z * z
    return R


def _expm_so3(w):
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-15:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_never_beats_svd(seed):
    rng = np.random.default_rng(100 + seed)
    M = rng.normal(size=(3, 3))
    if seed % 2:
        M[:, 0] = -M[:, 0]  # also cover det(M) < 0
    R, deg = fit_rotations(M[None])
    best_svd = np.trace(R[0].T @ M)
    Rs = _random_rotations(rng, 200_000)
    obj = np.einsum("kab,ab->k", Rs, M)
    Rb = Rs[np.argmax(obj)]
    fb = obj.max()
    step = 0.05
    for _ in range(3000):
        cand = _expm_so3(step * rng.normal(size=3)) @ Rb
        fc = np.trace(cand.T @ M)
        if fc > fb:
            Rb, fb = cand, fc
        else:
            step *= 0.998
    assert not deg[0]
    assert fb <= best_svd + 1e-9
    assert best_svd - fb < 1e-4  # the search did get close: the check is meaningful
    np.testing.assert_allclose(R[0] @ R[0].T, np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(R[0]) - 1.0) < 1e-12


def test_matches_horn_quaternion_method():
    rng = np.random.default_rng(7)
    Ms = rng.normal(size=(200, 3, 3))
    Ms[::3, :, 1] *= -1.0
    R, _ = fit_rotations(Ms)
    for k in range(Ms.shape[0]):
        np.testing.assert_allclose(R[k], _horn(Ms[k]), atol=1e-9)


def test_rest_pose_and_rigid_motion():
    g = Grid((4, 5, 3), 0.5, (1.0, 0.0, -1.0))
    rest = g.rest_positions()
    M = cross_covariance(g, rest)
    co = g.coords()
    interior = np.all((co > 0) & (co < np.asarray(g.dims) - 1), axis=1)
    np.testing.assert_allclose(M[interior], np.broadcast_to(2 * 0.25 * np.eye(3), M[interior].shape), atol=1e-14)
    R = rotation_step(g, rest, np.broadcast_to(np.eye(3), (g.n, 3, 3)))
    np.testing.assert_allclose(R, np.broadcast_to(np.eye(3), R.shape), atol=1e-13)
    rng = np.random.default_rng(8)
    Q = random_rotation(rng)
    t = rest @ Q.T + rng.normal(size=3)
    R = rotation_step(g, t, np.broadcast_to(np.eye(3), (g.n, 3, 3)))
    np.testing.assert_allclose(R, np.broadcast_to(Q, R.shape), atol=1e-12)


def test_objective_never_increases():
    rng = np.random.default_rng(9)
    scene = make_tiny(seed=9, dims=(4, 4, 4))
    g = Grid(scene.spec.dims, scene.spec.spacing, scene.spec.origin)
    cons = prepare_constraints(scene, g)
    t = g.rest_positions() + 0.3 * rng.normal(size=(g.n, 3))
    R0 = np.stack([random_rotation(rng) for _ in range(g.n)])
    E0 = energy_terms(g, t, R0, cons)
    R1 = rotation_step(g, t, R0)
    E1 = energy_terms(g, t, R1, cons)
    assert E1[3] <= E0[3]
    # and every node's own terms are individually minimal (block minimiser)
    for _ in range(20):
        R2 = R1.copy()
        i = rng.integers(g.n)
        R2[i] = _expm_so3(0.05 * rng.normal(size=3)) @ R1[i]
        assert energy_terms(g, t, R2, cons)[3] >= E1[3] - 1e-12


def test_rank_one_keeps_previous():
    rng = np.random.default_rng(10)
    a, b = rng.normal(size=3), rng.normal(size=3)
    M = np.stack([np.outer(a, b), np.zeros((3, 3))])
    prev = np.stack([random_rotation(rng), random_rotation(rng)])
    R, deg = fit_rotations(M, prev)
    assert deg.all()
    np.testing.assert_array_equal(R, prev)
