"""Pins of the oracle's TSDF fusion (Sec. 8) and marching cubes (Sec. 4)
against what geometry fixes: every sign-change edge of every one of the 256
corner cases is used exactly once; a single inside corner gives one triangle
facing away from it; diagonal inside corners of a face are cut off
separately; a linear distance field's vertices lie exactly on its plane; a
sphere's mesh is closed, consistently oriented (Euler characteristic 2) with
outward normals and the sphere's area; a fronto-parallel depth map fuses to
the closed-form truncated distances; vertices follow a rigid deformation."""

import numpy as np
import pytest

from oracle import assoc, fusion
from oracle.lattice import level_grids
from synth.scenes import random_rotation, render_planes

SMALL = dict(width=64, height=48, fx=60.0, fy=60.0, cx=32.0, cy=24.0)


def _grid(n, h=1.0, origin=(0.0, 0.0, 0.0)):
    return level_grids((n, n, n), h, origin, 1)[-1]


def test_every_case_uses_each_sign_change_edge_once():
    for inside in range(256):
        loops = fusion.cell_loops(inside)
        used = sorted(e for loop in loops for e in loop)
        change = sorted(e for e, (a, b) in enumerate(fusion.EDGE_CORNERS)
                        if ((inside >> a) & 1) != ((inside >> b) & 1))
        assert used == change, inside
        assert all(len(loop) >= 3 for loop in loops)
        tris = fusion.cell_triangles(inside)
        assert len(tris) == sum(len(loop) - 2 for loop in loops)


def test_edge_numbering():
    """Edge 4 q + j joins the corners that differ in bit q; j = b1 + 2 b2 from
    the two other axes' bits in increasing axis order."""
    assert fusion.EDGE_CORNERS[0] == (0, 1) and fusion.EDGE_CORNERS[3] == (6, 7)
    assert fusion.EDGE_CORNERS[4] == (0, 2) and fusion.EDGE_CORNERS[5] == (1, 3)
    assert fusion.EDGE_CORNERS[8] == (0, 4) and fusion.EDGE_CORNERS[11] == (3, 7)


def test_one_inside_corner_gives_one_outward_triangle():
    g = _grid(2)
    D = np.array([-0.25, 0.75, 0.75, 0.75, 0.75, 0.75, 0.75, 0.75], np.float32)
    W = np.ones(8, np.float32)
    cells, edges, verts = fusion.marching_cubes(g, D, W)
    assert cells.tolist() == [0]
    assert sorted(edges[0].tolist()) == [0, 4, 8]
    t = 0.25 / (0.25 + 0.75)
    np.testing.assert_allclose(sorted(map(tuple, verts[0].astype(np.float64))),
                               sorted([(0, 0, t), (0, t, 0), (t, 0, 0)]), atol=1e-7)
    v = verts[0].astype(np.float64)
    nrm = np.cross(v[1] - v[0], v[2] - v[0])
    assert np.all(nrm > 0)   # away from the inside corner 0, toward larger D


def test_ambiguous_face_separates_the_inside_corners():
    """Corners 0 and 3 (diagonal on the face z = 0) inside: two loops of 3."""
    loops = fusion.cell_loops((1 << 0) | (1 << 3))
    assert sorted(map(sorted, loops)) == [[0, 4, 8], [1, 5, 11]]


def test_linear_field_vertices_lie_on_the_plane():
    rng = np.random.default_rng(1)
    n = 9
    g = _grid(n, h=0.5, origin=(-1.0, -2.0, 0.5))
    m = rng.normal(size=3)
    m /= np.linalg.norm(m)
    x = g.rest_positions()
    c = x.mean(axis=0) + 0.1
    D = ((x - c) @ m).astype(np.float32)
    cells, edges, verts = fusion.marching_cubes(g, D, np.ones(g.n, np.float32))
    assert cells.size > 50
    v = verts.reshape(-1, 3).astype(np.float64)
    assert np.abs((v - c) @ m).max() < 2e-6
    tri = verts.astype(np.float64)
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    area = np.linalg.norm(nrm, axis=1)
    ok = area > 1e-9
    assert np.all(nrm[ok] @ m > 0)


def test_sphere_mesh_is_closed_oriented_and_has_the_sphere_area():
    n = 24
    g = _grid(n, h=1.0)
    x = g.rest_positions()
    c = np.array([11.3, 11.6, 11.1])
    r = 7.2
    D = (np.linalg.norm(x - c, axis=1) - r).astype(np.float32)
    cells, edges, verts = fusion.marching_cubes(g, D, np.ones(g.n, np.float32))
    # identify every vertex by the grid edge it lies on
    keys = []
    nx = n
    for cell, tri in zip(cells, edges):
        cx, cy, cz = cell % (nx - 1), (cell // (nx - 1)) % (nx - 1), cell // (nx - 1) ** 2
        row = []
        for e in tri:
            a, b = fusion.EDGE_CORNERS[e]
            ia = g.node_id(cx + (a & 1), cy + ((a >> 1) & 1), cz + (a >> 2))
            ib = g.node_id(cx + (b & 1), cy + ((b >> 1) & 1), cz + (b >> 2))
            row.append((int(ia), int(ib)))
        keys.append(row)
    directed = {}
    for row in keys:
        for k in range(3):
            e = (row[k], row[(k + 1) % 3])
            directed[e] = directed.get(e, 0) + 1
    assert max(directed.values()) == 1                      # consistent orientation
    for (a, b) in directed:
        assert (b, a) in directed                           # closed: every edge twice
    V = len({v for row in keys for v in row})
    E = len(directed) // 2
    F = len(keys)
    assert V - E + F == 2
    tri = verts.astype(np.float64)
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    cen = tri.mean(axis=1)
    assert np.all(np.einsum("ta,ta->t", nrm, cen - c) > 0)  # outward
    area = 0.5 * np.linalg.norm(nrm, axis=1).sum()
    assert abs(area / (4 * np.pi * r * r) - 1) < 0.02


def test_unobserved_cells_are_skipped():
    g = _grid(3)
    x = g.rest_positions()
    D = (x[:, 0] - 0.5).astype(np.float32)
    W = np.ones(g.n, np.float32)
    W[g.node_id(0, 0, 0)] = 0.0                            # a corner of cell 0 only
    cells, _, _ = fusion.marching_cubes(g, D, W)
    assert set(cells.tolist()) == {2, 4, 6}                 # the other x = 0.5 cells


def test_fronto_parallel_plane_fuses_to_the_truncated_distance():
    """Depth Z0 everywhere: every visible point of a rest lattice gets
    min(1, (Z0 - z) / tau) when z <= Z0 + tau, weight 1; points behind the
    truncation band are untouched; a second identical frame leaves D and
    raises W up to W_max."""
    cam = assoc.Camera(**SMALL)
    Z0 = 1.0
    depth = np.full((SMALL["height"], SMALL["width"]), Z0, np.float32)
    n, h = 8, 0.05
    g = _grid(n, h=h, origin=(-0.15, -0.12, 0.82))
    tau = 0.13  # no grid plane on the truncation boundary
    D0 = np.zeros(g.n, np.float32)
    W0 = np.zeros(g.n, np.float32)
    disp = np.zeros((g.n, 3))
    pose = np.concatenate([np.eye(3).ravel(), np.zeros(3)])
    allowed = np.ones(g.n, bool)
    D1, W1, k = fusion.integrate(g, D0, W0, disp, pose, cam, depth, allowed, tau, 2.0)
    z = g.rest_positions()[:, 2]
    upd = z <= Z0 + tau
    assert k == int(upd.sum()) > 0
    np.testing.assert_array_equal(W1, np.where(upd, 1.0, 0.0).astype(np.float32))
    expect = np.where(upd, np.minimum(1.0, (Z0 - z) / tau), 0.0).astype(np.float32)
    np.testing.assert_array_equal(D1, expect)
    D2, W2, _ = fusion.integrate(g, D1, W1, disp, pose, cam, depth, allowed, tau, 2.0)
    np.testing.assert_array_equal(D2, D1)
    D3, W3, _ = fusion.integrate(g, D2, W2, disp, pose, cam, depth, allowed, tau, 2.0)
    assert W3.max() == 2.0
    # a masked point is not touched
    allowed[:5] = False
    D4, W4, _ = fusion.integrate(g, D0, W0, disp, pose, cam, depth, allowed, tau, 2.0)
    assert np.all(W4[:5] == 0) and np.all(D4[:5] == 0)


def test_fusion_then_marching_cubes_recovers_a_plane():
    """A tilted plane rendered into a depth map, fused into a rest lattice:
    the extracted surface lies on the plane to the interpolation error of a
    clamped distance (well inside the truncation band)."""
    cam = dict(width=320, height=240, fx=260.0, fy=260.0, cx=160.0, cy=120.0)
    m = np.array([0.1, -0.15, -1.0])
    m /= np.linalg.norm(m)
    depth = render_planes(cam, [(m, -1.0)])
    g = _grid(20, h=0.02, origin=(-0.19, -0.19, 0.8))
    pose = np.concatenate([np.eye(3).ravel(), np.zeros(3)])
    D, W, k = fusion.integrate(g, np.zeros(g.n, np.float32), np.zeros(g.n, np.float32),
                               np.zeros((g.n, 3)), pose, assoc.Camera(**cam), depth,
                               np.ones(g.n, bool), tau=0.1, w_max=64.0)
    cells, edges, verts = fusion.marching_cubes(g, D, W)
    v = verts.reshape(-1, 3).astype(np.float64)
    assert v.shape[0] > 100
    # plane m . x = -1; projective distance along z differs from the normal
    # distance by the factor |m_z|, which is constant: still a plane
    dist = v @ m + 1.0
    assert np.abs(dist).max() < 2e-3


def test_rigid_deformation_moves_vertices_rigidly():
    g = _grid(6, h=0.3, origin=(0.1, -0.2, 0.4))
    rng = np.random.default_rng(3)
    Q = random_rotation(rng)
    c = np.array([0.2, 0.1, -0.3])
    rest = g.rest_positions()
    disp = rest @ Q.T + c - rest
    x = rest.mean(axis=0) + 0.4 * rng.uniform(-1, 1, size=(30, 3))
    pose = np.concatenate([np.eye(3).ravel(), np.zeros(3)])
    np.testing.assert_allclose(fusion.deform_vertices(g, disp, pose, x), x @ Q.T + c, atol=1e-12)
    R2 = random_rotation(rng)
    pose2 = np.concatenate([R2.ravel(), [0.5, 0.0, 0.1]])
    np.testing.assert_allclose(fusion.deform_vertices(g, np.zeros_like(disp), pose2, x),
                               x @ R2.T + [0.5, 0.0, 0.1], atol=1e-12)
