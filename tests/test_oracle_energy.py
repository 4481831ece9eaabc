"""Pins of the oracle's energy (Sec. 6, eqs. (1)-(4)) and Jacobian.

* hand-computed worked examples (tests/golden/hand_examples.json);
* zero energy under the identity warp and under any rigid motion;
* the assembled J equals central finite differences of the residual evaluated
  straight from the definitions, and 2 J^T r equals the finite-difference
  gradient of the energy;
* A = J^T J is symmetric positive semi-definite, p^T A p = ||J p||^2, and its
  ARAP block annihilates affine fields at interior nodes;
* the Jacobi diagonal matches its closed form;
* input validation."""

import json
import os

import numpy as np
import pytest

import oracle
from oracle.energy import assemble, prepare_constraints, residual_direct, energy_terms
from oracle.lattice import Grid, level_grids, trilinear
from oracle.solver import LevelSystem, jacobi_diag
from synth import LatticeSpec, Scene, make_tiny, random_rotation
from synth.scenes import make_identity_scene, make_rigid_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _rot_z(deg):
    a = np.deg2rad(deg)
    return np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1.0]])


def _scene_from_example(ex):
    spec = LatticeSpec(dims=(2, 2, 2), spacing=1.0, origin=(0, 0, 0), num_levels=1,
                       gn_iters=(1,), pcg_iters=(1,), w_dense=1.0, w_sparse=10.0, w_arap=5.0)
    d, s = ex["dense"], ex["sparse"]
    return Scene(spec=spec, canon=np.array([d["canon"]]), target=np.array([d["target"]]),
                 normal=np.array([d["normal"]]), weight=np.array([d["weight"]]),
                 sparse_canon=np.array([s["canon"]]), sparse_target=np.array([s["target"]]))


@pytest.mark.parametrize("name", ["translate_node0", "rotate_node0"])
def test_hand_examples(name):
    ex = json.load(open(GOLDEN))[name]
    scene = _scene_from_example(ex)
    g = Grid((2, 2, 2), 1.0, (0.0, 0.0, 0.0))
    cons = prepare_constraints(scene, g)
    t = g.rest_positions()
    t[0] += ex["node0_offset"]
    R = np.broadcast_to(np.eye(3), (8, 3, 3)).copy()
    R[0] = _rot_z(ex["rot_node0_z_deg"])
    E = energy_terms(g, t, R, cons)
    exp = ex["expected"]
    np.testing.assert_allclose(E, [exp["E_total"], exp["wd_E_dense"], exp["ws_E_sparse"],
                                   exp["wr_E_reg"]], rtol=1e-12, atol=1e-15)
    # the assembled residual gives the same energy
    r = assemble(g, cons).residual(t, R)
    assert abs(r @ r - exp["E_total"]) < 1e-12


def test_identity_warp_has_zero_energy():
    base = make_tiny(seed=4, dims=(5, 4, 3))
    scene = make_identity_scene(base)
    g = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, 1)[0]
    cons = prepare_constraints(scene, g)
    t, R = oracle.rest_state(g)
    E = energy_terms(g, t, R, cons)
    assert E[0] < 1e-24


def test_rigid_motion_has_zero_energy():
    rng = np.random.default_rng(5)
    base = make_tiny(seed=5, dims=(4, 5, 4))
    Q = random_rotation(rng)
    c = rng.normal(size=3)
    scene = make_rigid_scene(base, Q, c)
    g = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, 1)[0]
    # the targets were rounded to float32: compare against the exact rigid map
    cons = prepare_constraints(scene, g)
    cons.target = cons.canon @ Q.T + c
    cons.sparse_target = cons.sparse_canon @ Q.T + c
    cons.normal = (base.normal.astype(np.float64) @ Q.T)
    cons.normal /= np.linalg.norm(cons.normal, axis=1, keepdims=True)
    t = g.rest_positions() @ Q.T + c
    R = np.broadcast_to(Q, (g.n, 3, 3)).copy()
    E = energy_terms(g, t, R, cons)
    assert E[0] < 1e-20


def _tiny_state(seed, dims=(3, 4, 3)):
    rng = np.random.default_rng(seed)
    scene = make_tiny(seed=seed, dims=dims, n_dense=25, n_sparse=4)
    g = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, 1)[0]
    cons = prepare_constraints(scene, g)
    t = g.rest_positions() + 0.2 * rng.normal(size=(g.n, 3))
    R = np.stack([random_rotation(rng) for _ in range(g.n)])
    return g, cons, t, R


def test_assembled_matches_direct_residual_and_fd_jacobian():
    g, cons, t, R = _tiny_state(6)
    asm = assemble(g, cons)
    r_direct = residual_direct(g, t, R, cons)
    np.testing.assert_allclose(asm.residual(t, R), r_direct, atol=1e-12)
    J = asm.J.toarray()
    eps = 1e-6
    tf = t.reshape(-1)
    for col in range(tf.size):
        tp = tf.copy(); tp[col] += eps
        tm = tf.copy(); tm[col] -= eps
        fd = (residual_direct(g, tp.reshape(-1, 3), R, cons)
              - residual_direct(g, tm.reshape(-1, 3), R, cons)) / (2 * eps)
        np.testing.assert_allclose(J[:, col], fd, atol=1e-8)


def test_gradient_matches_fd_energy():
    g, cons, t, R = _tiny_state(7)
    system = LevelSystem(g, cons)
    grad = 2.0 * system.gradient(t, R)
    eps = 1e-6
    tf = t.reshape(-1)
    fd = np.empty_like(tf)
    for col in range(tf.size):
        tp = tf.copy(); tp[col] += eps
        tm = tf.copy(); tm[col] -= eps
        fd[col] = (energy_terms(g, tp.reshape(-1, 3), R, cons)[0]
                   - energy_terms(g, tm.reshape(-1, 3), R, cons)[0]) / (2 * eps)
    np.testing.assert_allclose(grad, fd, rtol=1e-6, atol=1e-6)
    # exact quadratic expansion E(t + d) = E + 2 g^T d + d^T A d
    rng = np.random.default_rng(8)
    d = 0.3 * rng.normal(size=tf.size)
    E0 = energy_terms(g, t, R, cons)[0]
    E1 = energy_terms(g, (tf + d).reshape(-1, 3), R, cons)[0]
    np.testing.assert_allclose(E1, E0 + grad @ d + d @ (system.A @ d), rtol=1e-10)


def test_normal_matrix_properties():
    g, cons, t, R = _tiny_state(9)
    system = LevelSystem(g, cons)
    A = system.A.toarray()
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() > -1e-10
    rng = np.random.default_rng(10)
    p = rng.normal(size=A.shape[0])
    Jp = system.asm.J @ p
    np.testing.assert_allclose(p @ A @ p, Jp @ Jp, rtol=1e-12)
    # A does not depend on R: the same J serves every rotation
    R2 = np.stack([random_rotation(rng) for _ in range(g.n)])
    np.testing.assert_allclose(system.asm.residual(t, R) - system.asm.residual(t, R2),
                               system.asm.constant(R2) - system.asm.constant(R), atol=1e-12)


def test_arap_block_annihilates_affine_fields_at_interior_nodes():
    rng = np.random.default_rng(11)
    base = make_tiny(seed=11, dims=(5, 5, 5), weights=(0.0, 0.0, 5.0))
    g = level_grids(base.spec.dims, base.spec.spacing, base.spec.origin, 1)[0]
    cons = prepare_constraints(base, g)
    system = LevelSystem(g, cons)
    G = rng.normal(size=(3, 3))
    p = (g.rest_positions() @ G.T + rng.normal(size=3)).reshape(-1)
    Ap = (system.A @ p).reshape(-1, 3)
    co = g.coords()
    interior = np.all((co > 0) & (co < np.asarray(g.dims) - 1), axis=1)
    assert interior.sum() == 27
    np.testing.assert_allclose(Ap[interior], 0.0, atol=1e-11)
    assert np.abs(Ap[~interior]).max() > 1e-3


def test_jacobi_diagonal_closed_form():
    scene = make_tiny(seed=12, dims=(4, 3, 5), n_dense=30, n_sparse=5)
    g = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, 1)[0]
    cons = prepare_constraints(scene, g)
    d = jacobi_diag(assemble(g, cons).J).reshape(-1, 3)
    expect = np.zeros((g.n, 3))
    ids, alpha = trilinear(g, cons.canon)
    for c in range(cons.canon.shape[0]):
        for k in range(8):
            expect[ids[c, k]] += cons.w_dense * cons.weight[c] * alpha[c, k] ** 2 * cons.normal[c] ** 2
    ids, beta = trilinear(g, cons.sparse_canon)
    for s in range(cons.sparse_canon.shape[0]):
        for k in range(8):
            expect[ids[s, k]] += cons.w_sparse * beta[s, k] ** 2
    co = g.coords()
    nb = np.zeros(g.n)
    for axis in range(3):
        nb += (co[:, axis] > 0).astype(float) + (co[:, axis] < g.dims[axis] - 1)
    expect += 2.0 * cons.w_arap * nb[:, None]
    np.testing.assert_allclose(d, expect, rtol=1e-12)


def test_validation():
    base = make_tiny(seed=13, dims=(4, 4, 4))
    g = level_grids(base.spec.dims, base.spec.spacing, base.spec.origin, 1)[0]
    bad = make_tiny(seed=13, dims=(4, 4, 4))
    bad.canon = bad.canon.copy()
    bad.canon[0] = [10.0, 0.0, 0.0]
    with pytest.raises(ValueError):
        prepare_constraints(bad, g)
    bad = make_tiny(seed=13, dims=(4, 4, 4))
    bad.target = bad.target.copy()
    bad.target[1, 2] = np.nan
    with pytest.raises(ValueError):
        prepare_constraints(bad, g)
    bad = make_tiny(seed=13, dims=(4, 4, 4))
    bad.weight = bad.weight.copy()
    bad.weight[2] = -1.0
    with pytest.raises(ValueError):
        prepare_constraints(bad, g)
    zero = make_tiny(seed=13, dims=(4, 4, 4))
    zero.normal = zero.normal.copy()
    zero.normal[3] = 0.0
    cons = prepare_constraints(zero, g)
    assert cons.weight[3] == 0.0 and np.all(np.isfinite(cons.normal))
