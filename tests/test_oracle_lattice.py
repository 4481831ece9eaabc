"""Pins of the oracle's lattice geometry (Sec. 4) and hierarchy (Sec. 7.2)
against closed forms: trilinear interpolation reproduces affine maps exactly,
the weights of a hand-computed point, the boundary convention, level sizes and
the 6-neighbourhood edge count."""

import json
import os

import numpy as np
import pytest

import oracle
from oracle.lattice import Grid, cell_and_frac, level_grids, trilinear, arap_edges

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def test_trilinear_reproduces_affine_maps():
    rng = np.random.default_rng(1)
    g = Grid((5, 4, 6), 0.7, (0.3, -1.0, 2.0))
    G = rng.normal(size=(3, 3))
    c = rng.normal(size=3)
    t = g.rest_positions() @ G.T + c
    # points inside, on faces, and outside (extrapolation)
    span = (np.asarray(g.dims) - 1) * g.h
    x = np.asarray(g.origin) + rng.uniform(-0.3, 1.3, size=(500, 3)) * span
    ids, w = trilinear(g, x)
    S = np.einsum("ck,cka->ca", w, t[ids])
    np.testing.assert_allclose(S, x @ G.T + c, rtol=0, atol=1e-12)


def test_weights_hand_example_and_partition_of_unity():
    ex = json.load(open(GOLDEN))["trilinear_point"]
    g = Grid((2, 2, 2), 1.0, (0.0, 0.0, 0.0))
    ids, w = trilinear(g, np.array([ex["point"]]))
    np.testing.assert_array_equal(ids[0], np.arange(8))
    np.testing.assert_allclose(w[0], ex["weights"], atol=1e-15)
    rng = np.random.default_rng(2)
    g = Grid((7, 7, 7), 1.0, (0.0, 0.0, 0.0))
    x = rng.uniform(0, 6, size=(1000, 3))
    _, w = trilinear(g, x)
    assert np.all(w >= 0)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-14)


def test_boundary_convention():
    g = Grid((4, 4, 4), 1.0, (0.0, 0.0, 0.0))
    cell, f = cell_and_frac(g, np.array([[3.0, 2.0, 0.0]]))
    # last plane: clamped to cell n-2 with f = 1; interior plane: the upper cell
    np.testing.assert_array_equal(cell[0], [2, 2, 0])
    np.testing.assert_allclose(f[0], [1.0, 0.0, 0.0])


@pytest.mark.parametrize("n,expect", [(64, [16, 32, 64]), (96, [24, 48, 96]), (5, [2, 3, 5])])
def test_level_sizes(n, expect):
    grids = level_grids((n, n, n), 1.0, (0, 0, 0), 3)
    assert [gr.dims[0] for gr in grids] == expect
    assert [gr.h for gr in grids] == [4.0, 2.0, 1.0]
    # vertex nesting: the coarse extent never exceeds the fine one
    for coarse, fine in zip(grids[:-1], grids[1:]):
        assert (coarse.dims[0] - 1) * coarse.h <= (fine.dims[0] - 1) * fine.h


def test_too_coarse_rejected():
    with pytest.raises(ValueError):
        level_grids((3, 3, 3), 1.0, (0, 0, 0), 3)


@pytest.mark.parametrize("n", [2, 3, 16])
def test_six_neighbourhood(n):
    g = Grid((n, n, n), 1.0, (0, 0, 0))
    src, dst = arap_edges(g)
    assert src.size == 6 * (n - 1) * n * n
    deg = np.bincount(src, minlength=g.n)
    assert deg.min() == 3 and deg.max() == (6 if n > 2 else 3)
    rest = g.rest_positions()
    np.testing.assert_allclose(np.linalg.norm(rest[src] - rest[dst], axis=1), 1.0)


def test_transfer_exact_on_affine_fields():
    rng = np.random.default_rng(3)
    grids = level_grids((8, 7, 6), 0.5, (1.0, 2.0, 3.0), 2)
    coarse, fine = grids
    G = rng.normal(size=(3, 3))
    c = rng.normal(size=3)
    fc = coarse.rest_positions() @ G.T + c
    ff = fine.rest_positions() @ G.T + c
    # prolongation reproduces the affine field at every fine node, including
    # the extrapolated last plane of the even-sized axes
    np.testing.assert_allclose(oracle.prolong(coarse, fc, fine), ff, atol=1e-12)
    np.testing.assert_allclose(oracle.inject(fine, ff, coarse, 2), fc, atol=1e-12)
