"""Pins of the oracle's position step and flip-flop (Sec. 7.1) and hierarchy
(Sec. 7.2):

* Jacobi-PCG terminates: on 24 unknowns, 24 iterations equal the exact solve;
* PCG decreases the quadratic model at every iterate;
* the exact position step zeroes the gradient and equals dense least squares
  (numpy lstsq, an independent routine) on J t ~ c(R);
* every half-step of the flip-flop is non-increasing in energy;
* a rigid state that explains its targets is a fixed point on every level;
* the identity warp stays at rest with no NaN (0/0 guards);
* with exact steps and enough iterations the flip-flop reaches a stationary
  point: zero position gradient and Procrustes-optimal rotations."""

import numpy as np
import pytest

import oracle
from oracle.energy import prepare_constraints, energy_terms, assemble
from oracle.lattice import Grid, level_grids
from oracle.procrustes import rotation_step
from oracle.solver import LevelSystem, pcg, position_step
from synth import make_tiny, make_config0, random_rotation
from synth.scenes import make_identity_scene, make_rigid_scene


def _system(seed, dims, **kw):
    scene = make_tiny(seed=seed, dims=dims, **kw)
    g = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, 1)[0]
    cons = prepare_constraints(scene, g)
    return scene, g, cons, LevelSystem(g, cons)


def test_pcg_finite_termination():
    _, g, cons, system = _system(20, (2, 2, 2), n_dense=12, n_sparse=2)
    assert system.A.shape[0] == 24
    rng = np.random.default_rng(20)
    t = g.rest_positions() + 0.2 * rng.normal(size=(8, 3))
    R = np.stack([random_rotation(rng) for _ in range(8)])
    b = -system.gradient(t, R)
    exact = np.linalg.solve(system.A.toarray(), b)
    x = pcg(system.A, b, system.dinv, 24)
    np.testing.assert_allclose(x, exact, rtol=0, atol=1e-9 * np.abs(exact).max())


def test_pcg_monotone_model_decrease():
    _, g, cons, system = _system(21, (5, 4, 4), n_dense=60, n_sparse=5)
    rng = np.random.default_rng(21)
    t = g.rest_positions() + 0.2 * rng.normal(size=(g.n, 3))
    R = np.broadcast_to(np.eye(3), (g.n, 3, 3)).copy()
    gvec = system.gradient(t, R)
    trace = []
    pcg(system.A, -gvec, system.dinv, 30, trace=trace)
    model = [2 * gvec @ x + x @ (system.A @ x) for x in trace]
    assert model[0] < 0
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(model, model[1:]))


def test_exact_step_zero_gradient_and_lstsq():
    _, g, cons, system = _system(22, (3, 3, 4), n_dense=30, n_sparse=3)
    rng = np.random.default_rng(22)
    t = g.rest_positions() + 0.1 * rng.normal(size=(g.n, 3))
    R = np.stack([random_rotation(rng) for _ in range(g.n)])
    t1 = position_step(system, t, R, mode="direct")
    gnew = system.gradient(t1, R)
    assert np.abs(gnew).max() < 1e-9
    J = system.asm.J.toarray()
    ls, *_ = np.linalg.lstsq(J, system.asm.constant(R), rcond=None)
    np.testing.assert_allclose(t1.reshape(-1), ls, atol=1e-9)


def test_flip_flop_half_steps_monotone():
    scene = make_config0(0)
    trace = []
    out = oracle.solve_frame(scene, trace=trace)
    E = [e for (_, _, e) in trace]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(E, E[1:]))
    assert out["energy"][0] < 0.5 * energy_terms(out["grid"], *oracle.rest_state(out["grid"]),
                                                 prepare_constraints(scene))[0]


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_rigid_fixed_point(levels):
    rng = np.random.default_rng(30 + levels)
    base = make_tiny(seed=30 + levels, dims=(9, 8, 9), num_levels=levels, gn=2, pcg=6,
                     n_dense=80, n_sparse=6)
    Q = random_rotation(rng)
    c = rng.normal(size=3)
    scene = make_rigid_scene(base, Q, c)
    # exact (float64) rigid targets
    scene.target = scene.canon.astype(np.float64) @ Q.T + c
    scene.sparse_target = scene.sparse_canon.astype(np.float64) @ Q.T + c
    scene.normal = base.normal.astype(np.float64) @ Q.T
    grids = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, levels)
    fin = grids[-1]
    t0 = fin.rest_positions() @ Q.T + c
    R0 = np.broadcast_to(Q, (fin.n, 3, 3)).copy()
    out = oracle.solve_frame(scene, state=(t0, R0))
    np.testing.assert_allclose(out["t"], t0, atol=1e-9)
    np.testing.assert_allclose(out["R"], R0, atol=1e-9)
    assert out["energy"][0] < 1e-16


@pytest.mark.parametrize("levels", [1, 3])
def test_identity_warp_stays_at_rest(levels):
    base = make_tiny(seed=40, dims=(9, 9, 9), num_levels=levels, n_dense=50)
    scene = make_identity_scene(base)
    out = oracle.solve_frame(scene)
    fin = out["grid"]
    assert np.all(np.isfinite(out["t"])) and np.all(np.isfinite(out["R"]))
    np.testing.assert_allclose(out["t"], fin.rest_positions(), atol=1e-6)
    np.testing.assert_allclose(out["R"], np.broadcast_to(np.eye(3), out["R"].shape), atol=1e-6)


def test_flip_flop_converges_to_stationary_point():
    scene = make_tiny(seed=50, dims=(4, 4, 4), n_dense=60, n_sparse=4, gn=600, amp=0.2)
    out = oracle.solve_frame(scene, mode="direct")
    g = out["grid"]
    cons = prepare_constraints(scene, g)
    system = LevelSystem(g, cons)
    grad = system.gradient(out["t"], out["R"])
    assert np.abs(grad).max() < 1e-9
    R_fit = rotation_step(g, out["t"], out["R"])
    np.testing.assert_allclose(R_fit, out["R"], atol=1e-9)


def test_coarse_increment_reaches_finest():
    """Only the coarsest level iterates; the translation it finds must arrive
    unchanged at the finest level through two prolongations (Sec. 7.2)."""
    base = make_tiny(seed=60, dims=(9, 9, 9), num_levels=3, n_dense=80, n_sparse=6)
    v = np.array([0.3, -0.2, 0.1])
    scene = make_identity_scene(base)
    scene.target = scene.canon.astype(np.float64) + v
    scene.sparse_target = scene.sparse_canon.astype(np.float64) + v
    out = oracle.solve_frame(scene, mode="direct", gn_iters=(3, 0, 0), pcg_iters=(0, 0, 0))
    fin = out["grid"]
    np.testing.assert_allclose(out["t"], fin.rest_positions() + v, atol=1e-9)
    np.testing.assert_allclose(out["R"], np.broadcast_to(np.eye(3), out["R"].shape), atol=1e-9)
