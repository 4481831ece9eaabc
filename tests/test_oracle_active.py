"""Pins of the oracle's solve restricted to the optimised set M (Sec. 6,
Sec. 7) with grid growth (Sec. 8): a hand-counted M, the reduction to the
dense solve when M covers the lattice, points outside M staying put, the
gradient against finite differences of the restricted energy, monotone
energy, the rigid fixed point, and the extrapolation of new points."""

import numpy as np
import pytest

from oracle import active, solver
from oracle.energy import prepare_constraints
from oracle.lattice import level_grids
from synth import LatticeSpec
from synth.scenes import Scene, make_patch, make_rigid_scene, make_tiny, random_rotation


def _grid_cons(scene):
    s = scene.spec
    grids = level_grids(s.dims, s.spacing, s.origin, s.num_levels)
    return grids, prepare_constraints(scene, grids[0])


def _one_sample_scene(n=4, x=(0.3, 0.4, 0.5)):
    spec = LatticeSpec(dims=(n, n, n), spacing=1.0, origin=(0.0, 0.0, 0.0), num_levels=1,
                       gn_iters=(2,), pcg_iters=(6,))
    c = np.array([x], np.float32)
    z = np.zeros((0, 3), np.float32)
    return Scene(spec=spec, canon=c, target=c + 0.1, normal=np.array([[0, 0, 1]], np.float32),
                 weight=np.ones(1, np.float32), sparse_canon=z, sparse_target=z)


def test_hand_counted_active_set():
    """One sample in cell (0,0,0) of a 4^3 lattice: the isosurface points are
    the cell's 8 corners; their one-ring adds the 12 points with exactly one
    coordinate 2 and the others in {0, 1}: |M| = 20."""
    grids, cons = _grid_cons(_one_sample_scene())
    g = grids[-1]
    surf = active.surface_points(g, cons)
    act = active.active_set(g, cons)
    co = g.coords()
    np.testing.assert_array_equal(surf, np.all(co <= 1, axis=1))
    expect = np.all(co <= 1, axis=1) | ((np.sum(co == 2, axis=1) == 1) & np.all(co <= 2, axis=1))
    np.testing.assert_array_equal(act, expect)
    assert act.sum() == 20


def test_full_set_reduces_to_the_dense_solve():
    """Samples in every cell: M is the whole lattice and the restricted solve
    is the dense solve (same J, same normal equations) on 1 and 2 levels."""
    for levels, dims in ((1, (5, 4, 4)), (2, (7, 7, 7))):
        sc = make_tiny(seed=3, dims=dims, n_dense=1500, n_sparse=8, num_levels=levels, gn=2,
                       pcg=6)
        grids, cons = _grid_cons(sc)
        assert all(active.active_set(g, cons).all() for g in grids)
        a = active.solve_frame_active(sc)
        d = solver.solve_frame(sc)
        np.testing.assert_allclose(a["t"], d["t"], rtol=0, atol=1e-11)
        np.testing.assert_allclose(a["energy"], d["energy"], rtol=1e-11)


def test_points_outside_the_set_keep_their_state():
    sc = make_patch(seed=1, dims=(12, 12, 12), num_levels=2, gn=2, pcg=8)
    grids, cons = _grid_cons(sc)
    g = grids[-1]
    rng = np.random.default_rng(2)
    t0 = g.rest_positions() + 0.05 * rng.normal(size=(g.n, 3))
    R0 = np.stack([random_rotation(rng) for _ in range(g.n)])
    out = active.solve_frame_active(sc, state=(t0, R0))
    act = out["active"]
    assert 0.05 < act.mean() < 0.5
    np.testing.assert_array_equal(out["t"][~act], t0[~act])
    np.testing.assert_array_equal(out["R"][~act], R0[~act])
    assert np.abs(out["t"][act] - t0[act]).max() > 1e-3


def test_gradient_is_half_the_finite_difference_of_the_restricted_energy():
    """E restricted to M is quadratic in the positions of M (R fixed), so
    central differences are exact up to rounding: dE/dt_M = 2 g."""
    sc = make_patch(seed=4, dims=(8, 8, 8), n_dense=150, n_sparse=4)
    grids, cons = _grid_cons(sc)
    g = grids[-1]
    act = active.active_set(g, cons)
    rng = np.random.default_rng(5)
    t = g.rest_positions() + 0.1 * rng.normal(size=(g.n, 3))
    R = np.stack([random_rotation(rng) for _ in range(g.n)])
    system = active.ActiveSystem(g, cons, act)
    grad = system.gradient(t, R)
    cols = system.cols
    pick = rng.choice(cols.size, size=25, replace=False)
    h = 1e-4
    for k in pick:
        tp = t.reshape(-1).copy()
        tm = tp.copy()
        tp[cols[k]] += h
        tm[cols[k]] -= h
        ep = active.energy_terms_active(g, tp.reshape(-1, 3), R, cons, act)[0]
        em = active.energy_terms_active(g, tm.reshape(-1, 3), R, cons, act)[0]
        assert abs((ep - em) / (2 * h) - 2 * grad[k]) <= 1e-6 * max(1.0, abs(grad[k]))
    # a point outside M does not appear in the energy's dependence on M's rows
    out = np.flatnonzero(~np.repeat(act, 3))
    assert out.size > 0


def test_energy_never_increases():
    sc = make_patch(seed=6, dims=(10, 10, 10), num_levels=2, gn=3, pcg=10)
    tr = []
    active.solve_frame_active(sc, trace=tr)
    for lvl in (0, 1):
        e = [x[2] for x in tr if x[1] == lvl]
        assert all(b <= a * (1 + 1e-12) + 1e-15 for a, b in zip(e, e[1:]))


def test_rigid_state_is_a_fixed_point():
    """The whole lattice moved rigidly with exactly moved targets: zero energy
    over M, and the solve stays there."""
    base = make_patch(seed=7, dims=(8, 8, 8), n_dense=200, gn=2, pcg=8)
    rng = np.random.default_rng(8)
    Q = random_rotation(rng)
    c = np.array([0.3, -0.2, 0.5])
    sc = make_rigid_scene(base, Q, c)
    grids, cons = _grid_cons(sc)
    g = grids[-1]
    t0 = g.rest_positions() @ Q.T + c
    R0 = np.broadcast_to(Q, (g.n, 3, 3)).copy()
    out = active.solve_frame_active(sc, state=(t0, R0))
    assert out["energy"][0] < 1e-10
    assert np.abs(out["t"] - t0).max() < 1e-6


def test_growth_extrapolates_layer_by_layer():
    """Known points with a constant displacement c: every new point reached
    by the layers gets c; a point with two known neighbours takes their mean
    and the rotation of the first neighbour in the order -x, +x, -y, +y, -z,
    +z; two layers reach distance 2."""
    spec_grid = level_grids((6, 5, 4), 1.0, (0.0, 0.0, 0.0), 1)[-1]
    g = spec_grid
    n = g.n
    rest = g.rest_positions()
    co = g.coords()
    prev = co[:, 0] <= 1                          # slab x <= 1 known
    act = co[:, 0] <= 3                           # M grows to x <= 3
    c = np.array([0.1, -0.2, 0.3])
    t = rest + c
    R = np.broadcast_to(np.eye(3), (n, 3, 3)).copy()
    Rk = random_rotation(np.random.default_rng(9))
    R[prev] = Rk
    t2, R2, layers = active.grow(g, t + 7.0 * (~prev)[:, None], R, act, prev)
    assert layers == 2
    np.testing.assert_allclose(t2[act] - rest[act], np.broadcast_to(c, (act.sum(), 3)),
                               atol=1e-15)
    np.testing.assert_array_equal(R2[act], np.broadcast_to(Rk, (act.sum(), 3, 3)))
    np.testing.assert_array_equal(t2[~act], (t + 7.0)[~act])
    # mean of two known neighbours; rotation of the first in order (-x before +x)
    prev2 = np.zeros(n, bool)
    i = g.node_id(2, 2, 1)
    lo, hi = g.node_id(1, 2, 1), g.node_id(3, 2, 1)
    prev2[[lo, hi]] = True
    act2 = prev2.copy()
    act2[i] = True
    tt = rest.copy()
    tt[lo] += [1.0, 0.0, 0.0]
    tt[hi] += [0.0, 2.0, 0.0]
    RR = np.broadcast_to(np.eye(3), (n, 3, 3)).copy()
    Ra, Rb = random_rotation(np.random.default_rng(10)), random_rotation(np.random.default_rng(11))
    RR[lo], RR[hi] = Ra, Rb
    t3, R3, layers = active.grow(g, tt, RR, act2, prev2)
    assert layers == 1
    np.testing.assert_allclose(t3[i] - rest[i], [0.5, 1.0, 0.0], atol=1e-15)
    np.testing.assert_array_equal(R3[i], Ra)


def test_growth_enters_the_frame():
    """With the previous frame's M smaller than this frame's, the new points
    start from the extrapolated field; without a previous M nothing moves
    before the solve."""
    sc = make_patch(seed=12, dims=(10, 10, 10), gn=1, pcg=0)
    grids, cons = _grid_cons(sc)
    g = grids[-1]
    act = active.active_set(g, cons)
    prev = active.surface_points(g, cons)         # a smaller previous M
    rest = g.rest_positions()
    t0 = rest + np.array([0.2, 0.0, -0.1])
    R0 = np.broadcast_to(np.eye(3), (g.n, 3, 3)).copy()
    out = active.solve_frame_active(sc, state=(t0, R0), prev_active=prev, gn_iters=(0,))
    assert out["layers"] == 1
    np.testing.assert_allclose(out["t"], t0, atol=1e-15)
