"""Pins of the warm-start feature reference (oracle/warm.py)."""

import numpy as np

from oracle import net
from oracle.energy import Constraints
from oracle.lattice import Grid
from oracle.warm import features


def _cons(canon, target, normal, weight, w_dense=1.0):
    z = np.zeros((0, 3))
    return Constraints(np.asarray(canon, float), np.asarray(target, float),
                       np.asarray(normal, float), np.asarray(weight, float), z, z,
                       w_dense, 10.0, 5.0)


def test_constant_offset_along_normals():
    """Targets displaced by delta along each unit normal from the warped
    sample give r_c = -delta for every sample, so channel 6 is -delta / h at
    every touched node whatever the weights."""
    rng = np.random.default_rng(0)
    g = Grid((5, 4, 6), 0.5, (0.1, -0.2, 0.3))
    rest = g.rest_positions()
    t = rest + 0.05 * rng.normal(size=rest.shape)
    canon = g.origin + rng.uniform(0, 1, size=(40, 3)) * (np.array(g.dims) - 1) * g.h
    n = rng.normal(size=(40, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    from oracle.lattice import trilinear
    ids, al = trilinear(g, canon)
    warped = np.einsum("ck,cka->ca", al, t[ids])
    delta = 0.037
    target = warped + delta * n
    f = features(g, _cons(canon, target, n, rng.uniform(0.5, 2, 40), w_dense=3.0), t)
    v = f[:, 7] > 0
    assert v.sum() > 10
    np.testing.assert_allclose(f[v, 6], -delta / g.h, rtol=1e-12, atol=1e-12)
    assert np.all(f[~v, 6] == 0)
    np.testing.assert_allclose(f[:, 0:3], (t - rest) / g.h, rtol=1e-12, atol=1e-15)
    assert np.all(f[:, 3:6] == 0.0)  # no second frame given: no change


def test_brute_force_per_node():
    """Channel 6 and 7 against a direct per-node loop over samples."""
    rng = np.random.default_rng(1)
    g = Grid((3, 4, 3), 1.0, (0.0, 0.0, 0.0))
    rest = g.rest_positions()
    t = rest + 0.1 * rng.normal(size=rest.shape)
    t2 = rest + 0.1 * rng.normal(size=rest.shape)
    canon = rng.uniform(0, 1, size=(7, 3)) * (np.array(g.dims) - 1)
    canon[0] = [2.0, 3.0, 2.0]  # on the last node of every axis
    target = canon + 0.2 * rng.normal(size=canon.shape)
    n = rng.normal(size=(7, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    w = rng.uniform(0, 2, 7)
    w[3] = 0.0
    f = features(g, _cons(canon, target, n, w, w_dense=2.0), t, t2)
    for i in range(g.n):
        a, b, c = i % 3, (i // 3) % 4, i // 12
        num = den = 0.0
        for s in range(7):
            u = canon[s]
            cell = [min(int(np.floor(u[k])), g.dims[k] - 2) for k in range(3)]
            fr = [u[k] - cell[k] for k in range(3)]
            corner = (a - cell[0], b - cell[1], c - cell[2])
            if not all(x in (0, 1) for x in corner):
                continue
            alpha = np.prod([fr[k] if corner[k] else 1 - fr[k] for k in range(3)])
            # warp of the sample: sum over its 8 corners
            S = np.zeros(3)
            for k in range(8):
                dx, dy, dz = k & 1, (k >> 1) & 1, k >> 2
                wk = np.prod([fr[0] if dx else 1 - fr[0], fr[1] if dy else 1 - fr[1],
                              fr[2] if dz else 1 - fr[2]])
                S += wk * t[(cell[0] + dx) + 3 * ((cell[1] + dy) + 4 * (cell[2] + dz))]
            r = n[s] @ (S - target[s])
            num += alpha * 2.0 * w[s] * r
            den += alpha * 2.0 * w[s]
        assert f[i, 7] == (1.0 if den > 0 else 0.0)
        assert abs(f[i, 6] - (num / den if den > 0 else 0.0)) <= 1e-12
        np.testing.assert_allclose(f[i, 3:6], t[i] - t2[i], atol=1e-14)


def test_param_count_and_flatten_roundtrip():
    p = net.init_params(np.random.default_rng(2))
    v = net.flatten(p)
    assert v.size == 357587
    q = net.unflatten(v)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])


def _tiny_system(seed):
    from oracle.energy import prepare_constraints
    from oracle.lattice import level_grids
    from oracle.procrustes import rotation_step
    from oracle.solver import LevelSystem, rest_state
    from synth import make_tiny
    scene = make_tiny(seed=seed, dims=(5, 4, 4), num_levels=1, gn=1, pcg=4, n_dense=120,
                      n_sparse=6, spacing=0.5, origin=(0.1, -0.2, 0.3))
    g = level_grids(scene.spec.dims, scene.spec.spacing, scene.spec.origin, 1)[0]
    cons = prepare_constraints(scene, g)
    t, R = rest_state(g)
    rng = np.random.default_rng(seed)
    t = t + 0.05 * rng.standard_normal(t.shape)
    R = rotation_step(g, t, R)
    return g, cons, LevelSystem(g, cons), t, R, rng


def test_exact_step_recovers_the_position_minimiser():
    """Along the direction to the exact minimiser of E at fixed R (a direct
    sparse solve of A d = -g, another path than the step's formula) the step
    is 1 and lands on that minimiser."""
    from oracle.warm import exact_step
    for seed in (1, 2):
        g, cons, sysm, t, R, _ = _tiny_system(seed)
        d = sysm.solve(-sysm.gradient(t, R), "direct", 0).reshape(-1, 3)
        s, t_new = exact_step(sysm.asm, t, R, d)
        assert abs(s - 1.0) < 1e-9, s
        assert np.abs(t_new - (t + d)).max() < 1e-9


def test_exact_step_is_the_minimum_along_the_line():
    """E(t + s v), evaluated from the definitions eqs. (1)-(4), is smallest at
    the returned s among a fine grid of steps, for random directions (the
    exact minimum of a parabola through three of those values agrees)."""
    from oracle.energy import energy_terms
    from oracle.warm import exact_step
    g, cons, sysm, t, R, rng = _tiny_system(3)
    for _ in range(3):
        v = rng.standard_normal(t.shape) * 0.1
        s, _ = exact_step(sysm.asm, t, R, v)
        E = lambda x: energy_terms(g, t + x * v, R, cons)[0]
        e0 = E(s)
        for x in s + np.linspace(-1.0, 1.0, 41) * max(abs(s), 0.1):
            assert e0 <= E(x) + 1e-12
        # vertex of the parabola through s - 1, s, s + 1
        a, b, c = E(s - 1.0), e0, E(s + 1.0)
        vertex = s - 0.5 * (c - a) / (a - 2 * b + c)
        assert abs(vertex - s) < 1e-9 * max(1.0, abs(s))


def test_exact_step_zero_direction():
    """A zero direction (|J v| = 0) keeps the state: s = 0."""
    from oracle.warm import exact_step
    g, cons, sysm, t, R, _ = _tiny_system(4)
    s, t_new = exact_step(sysm.asm, t, R, np.zeros_like(t))
    assert s == 0.0 and np.array_equal(t_new, t)
