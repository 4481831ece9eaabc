"""Kernel parity on the GPU: each test calls the HIP path through the C-ABI
and compares with the FP64 oracle on the same seeded inputs.

Tolerances (float32 path): A p and J^T r to 1e-5 norm-relative, energy at a
fixed state to 1e-6 relative, rotations to 1e-5 rad.  The float64 path returns
its vectors through the float32 interface, so they are held to the float32
rounding bound (1.5e-7); its energies come back as doubles and are held to
1e-11."""

import numpy as np
import pytest

import oracle
from oracle.energy import energy_terms
from oracle.procrustes import fit_rotations as oracle_fit, rotation_step
from oracle.solver import LevelSystem
from synth import make_config0, make_config1, make_tiny

from helpers import (edge_fit_cases, grids_of, make_lattice, oracle_cons, random_state, rel_err,
                     rotation_angle)

pytestmark = pytest.mark.gpu

SCENES = {
    "cfg0": lambda: make_config0(0),
    # ragged multi-tile lattice, three levels, random weights
    "ragged": lambda: make_tiny(seed=3, dims=(21, 13, 11), n_dense=900, n_sparse=40,
                                num_levels=3, spacing=0.5, origin=(-1.0, 2.0, 0.25)),
    # a lattice smaller than one tile
    "small": lambda: make_tiny(seed=4, dims=(3, 5, 2), n_dense=30, n_sparse=3),
}


@pytest.fixture(scope="module")
def cfg1():
    return make_config1(0)


def _levels(scene):
    return range(scene.spec.num_levels)


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_apply_matches_oracle(name, precision):
    scene = SCENES[name]()
    lat = make_lattice(scene, precision=precision)
    cons = oracle_cons(scene)
    rng = np.random.default_rng(1)
    tol = 1e-5 if precision == "fp32" else 1.5e-7
    for lvl, grid in zip(_levels(scene), grids_of(scene)):
        system = LevelSystem(grid, cons)
        for p in (rng.normal(size=(grid.n, 3)),
                  np.sin(grid.rest_positions() / (3 * grid.h))):
            p32 = p.astype(np.float32)
            ref = (system.A @ p32.astype(np.float64).reshape(-1)).reshape(-1, 3)
            got = lat.debug_apply(lvl, p32)
            assert rel_err(got, ref) < tol, (name, lvl)


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_diag_gradient_energy_match_oracle(name, precision):
    scene = SCENES[name]()
    lat = make_lattice(scene, precision=precision)
    vec_tol, e_tol = (1e-5, 1e-6) if precision == "fp32" else (1.5e-7, 1e-11)
    cons = oracle_cons(scene)
    rng = np.random.default_rng(2)
    for lvl, grid in zip(_levels(scene), grids_of(scene)):
        system = LevelSystem(grid, cons)
        d_ref = 1.0 / np.where(system.dinv > 0, system.dinv, np.inf)
        assert rel_err(lat.debug_diag(lvl), d_ref.reshape(-1, 3)) < max(vec_tol, 1e-6)
        pos, rot = random_state(grid, rng)
        t, R = pos.astype(np.float64), rot.astype(np.float64)
        g_ref = system.gradient(t, R).reshape(-1, 3)
        assert rel_err(lat.debug_gradient(lvl, pos, rot), g_ref) < vec_tol
        e_ref = energy_terms(grid, t, R, cons)
        e_gpu = lat.debug_energy(lvl, pos, rot)
        np.testing.assert_allclose(e_gpu, e_ref, rtol=e_tol, atol=1e-13 * e_ref[0])


def test_cfg1_levels_match_oracle(cfg1):
    """The paper-scale 64^3 lattice: every level's operator, gradient and
    energy at a perturbed state."""
    lat = make_lattice(cfg1)
    cons = oracle_cons(cfg1)
    rng = np.random.default_rng(3)
    for lvl, grid in zip(_levels(cfg1), grids_of(cfg1)):
        system = LevelSystem(grid, cons)
        p = rng.normal(size=(grid.n, 3)).astype(np.float32)
        ref = (system.A @ p.astype(np.float64).reshape(-1)).reshape(-1, 3)
        assert rel_err(lat.debug_apply(lvl, p), ref) < 1e-5
        pos, rot = random_state(grid, rng, amp=0.5, rot_amp=0.1)
        t, R = pos.astype(np.float64), rot.astype(np.float64)
        assert rel_err(lat.debug_gradient(lvl, pos, rot),
                       system.gradient(t, R).reshape(-1, 3)) < 1e-5
        np.testing.assert_allclose(lat.debug_energy(lvl, pos, rot),
                                   energy_terms(grid, t, R, cons), rtol=1e-6)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 3e-7)])
def test_rotation_step_matches_oracle(precision, tol):
    scene = SCENES["ragged"]()
    lat = make_lattice(scene, precision=precision)
    rng = np.random.default_rng(5)
    for lvl, grid in zip(_levels(scene), grids_of(scene)):
        pos, rot = random_state(grid, rng, amp=0.4)
        ref = rotation_step(grid, pos.astype(np.float64), rot.astype(np.float64))
        got = lat.debug_rotations(lvl, pos, rot)
        ang = rotation_angle(got, ref)
        assert ang.max() < tol, (lvl, ang.max())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batched_fit_matches_oracle(precision):
    from paper_1603_08161_amd import fit_rotations
    rng = np.random.default_rng(6)
    M = rng.normal(size=(4096, 3, 3)).astype(np.float32)
    M[::3, :, 0] *= -1.0                              # det < 0 cases
    M[1::7] = np.eye(3) + 1e-4 * rng.normal(size=(M[1::7].shape))  # near identity
    # exactly rank 1 in float32 (small integers): degenerate
    a = rng.integers(1, 4, size=(64, 3)) * rng.choice([-1, 1], size=(64, 3))
    b = rng.integers(1, 4, size=(64, 3)) * rng.choice([-1, 1], size=(64, 3))
    M[5::64] = np.einsum("ka,kb->kab", a, b)[: M[5::64].shape[0]]
    M[9::64] = 0.0                                                 # zero: degenerate
    prev = np.stack([np.eye(3)] * M.shape[0]).astype(np.float32)
    prev[:, 0, 0] = -1.0
    prev[:, 1, 1] = -1.0  # a rotation by pi about z, distinguishable from I
    R_ref, deg = oracle_fit(M.astype(np.float64), prev.astype(np.float64))
    R, code = fit_rotations(M, prev, precision=precision)
    np.testing.assert_array_equal(code == 2, deg)
    ang = rotation_angle(R[~deg], R_ref[~deg])
    assert ang.max() < (1e-5 if precision == "fp32" else 3e-7)
    np.testing.assert_array_equal(R[deg], prev[deg])
    # objective trace(R^T M) matches (the unique quantity)
    obj = np.einsum("nab,nab->n", R.astype(np.float64), M.astype(np.float64))
    obj_ref = np.einsum("nab,nab->n", R_ref, M.astype(np.float64))
    np.testing.assert_allclose(obj[~deg], obj_ref[~deg], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batched_fit_edge_cases(precision):
    """Nearly diagonal cross-covariances (rotation angles down to 1e-33, where
    the float32 sweeps take their large-theta and too-small-to-rotate
    branches) and covariances scaled by 1e-15 and 1e15 fit the same rotation
    as the oracle's SVD."""
    from paper_1603_08161_amd import fit_rotations
    M, prev = edge_fit_cases(11)
    R_ref, deg = oracle_fit(M, prev)
    assert not deg.any()
    R, code = fit_rotations(M.astype(np.float32), prev.astype(np.float32), precision=precision)
    assert np.isfinite(R).all()
    assert not (code == 2).any()
    ang = rotation_angle(R, R_ref)
    assert ang.max() < (1e-5 if precision == "fp32" else 3e-7), ang.max()


def test_prolong_matches_oracle():
    scene = SCENES["ragged"]()
    lat = make_lattice(scene)
    grids = grids_of(scene)
    rng = np.random.default_rng(7)
    for lvl in range(1, len(grids)):
        coarse = rng.normal(size=(grids[lvl - 1].n, 3)).astype(np.float32)
        ref = oracle.prolong(grids[lvl - 1], coarse.astype(np.float64), grids[lvl])
        got = lat.debug_prolong(lvl, coarse)
        np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6 * np.abs(ref).max())
