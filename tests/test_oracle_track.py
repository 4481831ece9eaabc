"""Pins of the oracle's association of lattice model samples and of the
ICP-style tracked frame: at rest and under a rigid lattice state the deformed
samples reduce to plain rigidly moved samples (trilinear interpolation
reproduces affine fields), the global pose enters as a rigid change of
frame, and on a frame rendered from a rigidly moved box corner the tracked
frame brings the lattice's energy down to the noise floor."""

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import assoc, track
from oracle.lattice import level_grids
from synth import LatticeSpec
from synth.scenes import make_box_frame

PRM = assoc.AssocParams(eps_d=0.05, eps_n=0.3, eps_v=0.95)


def _box_lattice(n=10, levels=1, gn=3, pcg=10):
    # lattice covering the box corner's visible faces (metres)
    lo = np.array([-0.37, -0.52, 0.53])
    hi = np.array([0.62, 0.27, 1.12])
    h = float((hi - lo).max() / (n - 1))
    return LatticeSpec(dims=(n, n, n), spacing=h, origin=tuple(lo.tolist()), num_levels=levels,
                       gn_iters=(gn,) * levels, pcg_iters=(pcg,) * levels)


def _frame_dict(f, pose=None):
    d = dict(camera=f.camera, depth=f.depth, model_canon=f.model_canon,
             model_normal=f.model_normal)
    if pose is not None:
        d["pose"] = pose
    return d


def _grid(spec):
    return level_grids(spec.dims, spec.spacing, spec.origin, spec.num_levels)[-1]


def test_rest_state_is_the_plain_association():
    spec = _box_lattice()
    g = _grid(spec)
    f = make_box_frame(step=7)
    cam = assoc.Camera(**f.camera)
    tl, nl, w, px = track.lattice_associate(g, np.zeros((g.n, 3)),
                                            np.broadcast_to(np.eye(3), (g.n, 3, 3)),
                                            _frame_dict(f), PRM)
    pa, na, w0, px0 = assoc.associate(cam, f.depth, f.model_canon, f.model_normal, PRM)
    np.testing.assert_array_equal(px, px0)
    np.testing.assert_array_equal(w > 0, w0 > 0)
    np.testing.assert_allclose(w, w0, rtol=1e-12)
    np.testing.assert_allclose(tl, pa, atol=1e-15)
    np.testing.assert_allclose(nl, na, atol=1e-15)
    assert (w > 0).mean() > 0.9


def test_rigid_lattice_state_moves_samples_rigidly():
    """d_i = Q t_hat_i + c - t_hat_i, R_i = Q: the samples deform to
    Q p_hat + c with normals Q n_hat (affine reproduction of Sec. 4)."""
    spec = _box_lattice()
    g = _grid(spec)
    rng = np.random.default_rng(0)
    Q = Rotation.from_rotvec(np.deg2rad(1.2) * rng.normal(size=3) / 1.7).as_matrix()
    c = np.array([0.006, -0.004, 0.009])
    rest = g.rest_positions()
    disp = rest @ Q.T + c - rest
    rot = np.broadcast_to(Q, (g.n, 3, 3)).copy()
    f = make_box_frame(Q, c, step=7)
    q, nq = track.deform_samples(g, disp, rot, f.model_canon, f.model_normal,
                                 np.concatenate([np.eye(3).ravel(), np.zeros(3)]))
    x = f.model_canon.astype(np.float64)
    np.testing.assert_allclose(q, x @ Q.T + c, atol=1e-13)
    np.testing.assert_allclose(nq, f.model_normal.astype(np.float64) @ Q.T, atol=1e-13)
    tl, nl, w, _ = track.lattice_associate(g, disp, rot, _frame_dict(f), PRM)
    keep = w > 0
    assert keep.mean() > 0.9
    # the moved box is exactly explained: every residual n^a . (p_c - p^a) ~ 0
    r = np.einsum("ca,ca->c", nl[keep], (x @ Q.T + c)[keep] - tl[keep])
    assert np.abs(r).max() < 1e-6  # the depth map is stored as float32


def test_global_pose_is_a_change_of_frame():
    """Rest lattice with global pose (Rg, tg) associates like the samples
    moved by the pose, with targets and normals brought back by its inverse."""
    spec = _box_lattice()
    g = _grid(spec)
    Rg = Rotation.from_rotvec(np.deg2rad([0.7, -0.4, 0.9])).as_matrix()
    tg = np.array([0.005, 0.003, -0.007])
    pose = np.concatenate([Rg.ravel(), tg])
    f = make_box_frame(Rg, tg, step=7)
    cam = assoc.Camera(**f.camera)
    tl, nl, w, px = track.lattice_associate(g, np.zeros((g.n, 3)),
                                            np.broadcast_to(np.eye(3), (g.n, 3, 3)),
                                            _frame_dict(f, pose), PRM)
    x = f.model_canon.astype(np.float64)
    pa, na, w0, px0 = assoc.associate(cam, f.depth, x @ Rg.T + tg,
                                      f.model_normal.astype(np.float64) @ Rg.T, PRM)
    same = px == px0
    assert same.mean() > 0.999
    np.testing.assert_allclose(w[same], w0[same], rtol=1e-9, atol=1e-12)
    k = same & (w0 > 0)
    np.testing.assert_allclose(tl[k], (pa[k] - tg) @ Rg, atol=1e-12)
    np.testing.assert_allclose(nl[k], na[k] @ Rg, atol=1e-12)


def test_tracked_frame_recovers_a_rigid_motion():
    """The box corner moved by a small rigid motion: two association + solve
    rounds bring the dense energy to a small fraction of its start."""
    spec = _box_lattice(n=8, gn=4, pcg=12)
    rng = np.random.default_rng(1)
    Q = Rotation.from_rotvec(np.deg2rad(0.8) * rng.normal(size=3) / 1.7).as_matrix()
    c = np.array([0.004, -0.003, 0.006])
    f = make_box_frame(Q, c, step=11)
    g = _grid(spec)
    tl, nl, w, _ = track.lattice_associate(g, np.zeros((g.n, 3)),
                                           np.broadcast_to(np.eye(3), (g.n, 3, 3)),
                                           _frame_dict(f), PRM)
    r0 = np.einsum("ca,ca->c", nl, f.model_canon.astype(np.float64) - tl)
    e0 = float(np.sum(w * r0 * r0))
    hist = []
    out = track.solve_frame_icp(spec, _frame_dict(f), PRM, 3, history=hist)
    e = [h[0][1] for h in hist]   # w_d E_dense after each round
    print("dense energy at rest", e0, "per round:", e, "associated:", [h[1] for h in hist])
    assert e[-1] < 0.05 * e0
    assert np.isfinite(out["t"]).all()


def test_tracked_frame_with_pose_explains_a_rigid_motion_by_the_pose():
    """The box corner moved rigidly by (Q, c): the pose found first (Sec. 6)
    recovers (Q, c), so the non-rigid rounds that follow leave the lattice at
    rest (a rigid motion costs the lattice nothing once the pose holds it)."""
    spec = _box_lattice(n=8, gn=2, pcg=10)
    rng = np.random.default_rng(4)
    Q = Rotation.from_rotvec(np.deg2rad(1.0) * rng.normal(size=3) / 1.7).as_matrix()
    c = np.array([0.006, 0.004, -0.005])
    f = make_box_frame(Q, c, step=9)
    out, P, hist = track.track_frame(spec, _frame_dict(f), PRM, rigid_iters=8, icp_iters=1)
    np.testing.assert_allclose(P[:9].reshape(3, 3), Q, atol=1e-5)
    np.testing.assert_allclose(P[9:], c, atol=1e-5)
    assert hist[-1][0] < 1e-6 * hist[0][0]
    g = _grid(spec)
    disp = out["t"] - g.rest_positions()
    assert np.abs(disp).max() < 1e-4 * spec.spacing * 100
