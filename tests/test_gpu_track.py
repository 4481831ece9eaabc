"""Projective association (Sec. 5.1), the rigid pose by projective ICP
(Sec. 4, Sec. 6) and the ICP-style tracked frame (Sec. 3) through the C-ABI
(include/vd_track.h) against the FP64 oracle (oracle/assoc.py,
oracle/track.py) on the same seeded inputs.

Association decisions are integer results taken in float64 on both sides in
the same operation order, so pixels and the kept/pruned split must be
bit-exact, and the float32 outputs equal to the oracle's float64 values
rounded to float32."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import assoc, track
from oracle.lattice import level_grids
from synth import LatticeSpec
from synth.scenes import CAM, make_box_frame, make_config1, render_planes

pytestmark = pytest.mark.gpu

EPS = (0.05, 0.3, 0.95)
PRM = assoc.AssocParams(*EPS)


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32)


def _check_assoc(gpu, ref):
    t, n, w, px = gpu
    tr, nr, wr, pr = ref
    np.testing.assert_array_equal(px, pr)
    np.testing.assert_array_equal(w > 0, wr > 0)
    np.testing.assert_array_equal(w, _f32(wr))
    np.testing.assert_array_equal(t, _f32(tr))
    np.testing.assert_array_equal(n, _f32(nr))


def _edge_samples(rng, f, k=3000):
    """Model samples of a frame moved and perturbed so that every branch is
    taken: kept pairs, far pairs (Phi_d < 0), tilted normals (Phi_n < 0),
    grazing normals (Phi_v < 0), zero normals, points behind the camera,
    outside the image, on the border pixels and on missing depth."""
    x = f.model_canon.astype(np.float64)
    n = f.model_normal.astype(np.float64)
    pick = rng.choice(x.shape[0], size=min(k, x.shape[0]), replace=False)
    p = x[pick] + rng.normal(scale=0.01, size=(pick.size, 3))
    q = n[pick] + rng.normal(scale=0.3, size=(pick.size, 3))
    m = pick.size // 12
    q[:m] = 0.0                                   # zero normals
    p[m:2 * m, 2] *= -1.0                         # behind the camera
    p[2 * m:3 * m, 0] += 5.0                      # outside the image
    p[3 * m:4 * m] *= 1.5                         # far from the measurement
    q[4 * m:5 * m] = np.cross(q[4 * m:5 * m], p[4 * m:5 * m])  # grazing
    # border pixels u = 0 and v = H-1 (no measured normal there)
    z = p[5 * m:6 * m, 2:3]
    u = np.where(np.arange(m) % 2 == 0, 0.5, CAM["width"] - 0.5)
    p[5 * m:6 * m, 0] = (u - CAM["cx"]) * z[:, 0] / CAM["fx"]
    return _f32(p), _f32(q)


@pytest.mark.parametrize("which", ["box", "torus"])
def test_associate_matches_oracle(which):
    from paper_1603_08161_amd import associate
    rng = np.random.default_rng(3)
    if which == "box":
        f = make_box_frame(Rotation.from_rotvec([0.01, -0.02, 0.015]).as_matrix(),
                           np.array([0.01, 0.0, -0.01]), step=5, noise=1e-3)
    else:
        _, f = make_config1(seed=1, n=32, num_levels=2, depth_frame=True)
    p, q = _edge_samples(rng, f)
    gpu = associate(f.camera, f.depth, p, q, EPS)
    ref = assoc.associate(assoc.Camera(**f.camera), f.depth, p, q, PRM)
    _check_assoc(gpu, ref)
    kept = int((gpu[2] > 0).sum())
    print(f"{which}: {p.shape[0]} samples, {kept} kept")
    assert 0.2 * p.shape[0] < kept < 0.9 * p.shape[0]


def test_associate_empty_and_errors():
    from paper_1603_08161_amd import VDError, associate
    f = make_box_frame(step=40)
    z = np.zeros((0, 3), np.float32)
    t, n, w, px = associate(f.camera, f.depth, z, z, EPS)
    assert t.shape == (0, 3) and w.shape == (0,)
    with pytest.raises(VDError):
        associate(f.camera, f.depth, f.model_canon, f.model_normal, (0.05, 0.0, 0.9))
    bad = dict(f.camera, fx=-1.0)
    with pytest.raises(VDError):
        associate(bad, f.depth, f.model_canon, f.model_normal, EPS)


def test_rigid_pose_matches_oracle():
    """Box corner moved by a rigid motion: the GPU's ICP iterations follow the
    oracle's (same kept counts, energies, poses to float64 rounding) and
    recover the motion."""
    from paper_1603_08161_amd import rigid_pose
    rng = np.random.default_rng(5)
    Q = Rotation.from_rotvec(np.deg2rad(1.5) * rng.normal(size=3) / 1.7).as_matrix()
    c = np.array([0.008, -0.006, 0.01])
    f = make_box_frame(Q, c, step=4)
    P, hist = rigid_pose(f.camera, f.depth, f.model_canon, f.model_normal, EPS, 6)
    R_o, t_o, hist_o = assoc.rigid_pose(assoc.Camera(**f.camera), f.depth, f.model_canon,
                                        f.model_normal, PRM, 6)
    hist_o = np.array(hist_o)
    np.testing.assert_array_equal(hist[:, 1], hist_o[:, 1])
    np.testing.assert_allclose(hist[:, 0], hist_o[:, 0], rtol=1e-9, atol=1e-12 * hist_o[0, 0])
    np.testing.assert_allclose(P[:9].reshape(3, 3), R_o, atol=1e-12)
    np.testing.assert_allclose(P[9:], t_o, atol=1e-12)
    np.testing.assert_allclose(P[:9].reshape(3, 3), Q, atol=1e-6)
    np.testing.assert_allclose(P[9:], c, atol=1e-6)
    print("rigid ICP E per iteration:", hist[:, 0], "kept:", hist[:, 1])


def test_rigid_pose_singular_system_keeps_the_pose():
    """A single plane constrains 3 of the 6 degrees of freedom: the 6x6
    system is singular and the pose stays where it started (oracle too)."""
    from paper_1603_08161_amd import rigid_pose
    m = np.array([0.2, -0.1, -1.0])
    m /= np.linalg.norm(m)
    depth = render_planes(CAM, [(m, -0.9)])
    W, H = CAM["width"], CAM["height"]
    vv, uu = np.mgrid[8:H - 8:9, 8:W - 8:9]
    z = depth[vv, uu].astype(np.float64)
    pts = np.stack([(uu + 0.5 - CAM["cx"]) * z / CAM["fx"],
                    (vv + 0.5 - CAM["cy"]) * z / CAM["fy"], z], -1).reshape(-1, 3)
    pts += 0.002 * m  # off the plane, so the step would move it
    nrm = np.broadcast_to(m, pts.shape)
    P0 = np.concatenate([np.eye(3).ravel(), np.zeros(3)])
    P, hist = rigid_pose(CAM, depth, _f32(pts), _f32(nrm), EPS, 2, P0)
    R_o, t_o, hist_o = assoc.rigid_pose(assoc.Camera(**CAM), depth, _f32(pts), _f32(nrm), PRM, 2)
    np.testing.assert_array_equal(P, P0)
    np.testing.assert_array_equal(R_o, np.eye(3))
    assert hist[0, 1] == hist_o[0][1] > 6


def _box_spec(n=10, levels=2, gn=3, pcg=10):
    lo = np.array([-0.37, -0.52, 0.53])
    hi = np.array([0.62, 0.27, 1.12])
    h = float((hi - lo).max() / (n - 1))
    return LatticeSpec(dims=(n, n, n), spacing=h, origin=tuple(lo.tolist()), num_levels=levels,
                       gn_iters=(gn,) * levels, pcg_iters=(pcg,) * levels)


def _frame_dict(f, pose=None, sparse=None):
    d = dict(camera=f.camera, depth=f.depth, model_canon=f.model_canon,
             model_normal=f.model_normal)
    if pose is not None:
        d["pose"] = pose
    if sparse is not None:
        d["sparse_canon"], d["sparse_target"] = sparse
    return d


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_lattice_association_matches_oracle(precision):
    """Model samples deformed by a random lattice state (displacements and
    rotations) and a global pose, associated on the GPU as the tracked frame
    does it, against oracle/track.py's lattice association."""
    from paper_1603_08161_amd import Lattice
    from helpers import random_state
    spec = _box_spec(n=12, levels=1)
    g = level_grids(spec.dims, spec.spacing, spec.origin, 1)[-1]
    rng = np.random.default_rng(11)
    Rg = Rotation.from_rotvec([0.012, -0.008, 0.01]).as_matrix()
    tg = np.array([0.004, -0.002, 0.006])
    pose = np.concatenate([Rg.ravel(), tg])
    f = make_box_frame(Rg, tg, step=6, noise=5e-4)
    lat = Lattice.from_spec(spec, precision=precision)
    lat.set_depth_frame(f, eps=EPS)
    lat.set_pose(pose)
    np.testing.assert_array_equal(lat.get_pose(), pose)
    pos, rot = random_state(g, rng, amp=0.02, rot_amp=0.05)
    disp = (pos.astype(np.float64) - g.rest_positions()).astype(np.float32)
    gpu = lat.debug_associate(disp, rot)
    ref = track.lattice_associate(g, disp.astype(np.float64), rot.astype(np.float64),
                                  _frame_dict(f, pose), PRM)
    _check_assoc(gpu, ref)
    kept = int((gpu[2] > 0).sum())
    print(f"{precision}: {f.model_canon.shape[0]} samples, {kept} kept")
    assert kept > 0.5 * f.model_canon.shape[0]


def test_tracked_frame_matches_oracle_box():
    """Rigid pose first, then two association + solve rounds on a 2-level box
    lattice (11^3, float64 by the small-lattice precision rule) whose frame
    moved rigidly, with depth noise: final energy within 1e-4 of the oracle,
    positions within 1e-3 of the spacing, the pose to float64 rounding of the
    same ICP iterations."""
    from paper_1603_08161_amd import Lattice
    spec = _box_spec(n=11, levels=2, gn=3, pcg=10)
    rng = np.random.default_rng(2)
    Q = Rotation.from_rotvec(np.deg2rad(1.0) * rng.normal(size=3) / 1.7).as_matrix()
    c = np.array([0.006, 0.004, -0.005])
    f = make_box_frame(Q, c, step=9, noise=1e-3, seed=4)
    lat = Lattice.from_spec(spec, graph=True, precision="fp64")
    lat.set_depth_frame(f, eps=EPS)
    rep = lat.track_frame(rigid_iters=4, icp_iters=2, reset=True)
    hist = []
    out, P, rh = track.track_frame(spec, _frame_dict(f), PRM, 4, 2, history=hist)
    np.testing.assert_allclose(rep["pose"], P, atol=1e-9)
    np.testing.assert_array_equal(rep["rigid_hist"][:, 1], np.array(rh)[:, 1])
    assert list(rep["assoc_kept"]) == [h[1] for h in hist]
    e_rel = abs(rep["energy"][0] / out["energy"][0] - 1.0)
    pos = lat.get_state64()[0]
    dp = np.abs(pos - out["t"]).max() / spec.spacing
    print(f"tracked box frame: E gpu {rep['energy'][0]:.9g} oracle {out['energy'][0]:.9g} "
          f"rel {e_rel:.2e}, max |dt|/h {dp:.2e}, kept {rep['assoc_kept']}")
    # float64 lattice, same kept pairs: rounding-order differences only
    assert e_rel <= 1e-12
    assert dp <= 1e-10


@pytest.mark.parametrize("n,precision", [(40, "fp32"), (32, "fp64")])
def test_tracked_frame_matches_oracle_torus(n, precision):
    """The warped torus (the 64^3 workload's surface) on an n^3, 2-level
    lattice: model samples of the undeformed surface, its noisy depth map and
    sparse pairs; two association + solve rounds without a pose change."""
    from paper_1603_08161_amd import Lattice
    scene, f = make_config1(seed=2, n=n, num_levels=2, gn=4, pcg=12, depth_frame=True)
    spec = scene.spec
    sparse = (scene.sparse_canon, scene.sparse_target)
    lat = Lattice.from_spec(spec, precision=precision)
    lat.set_depth_frame(f, sparse_canon=sparse[0], sparse_target=sparse[1], eps=EPS)
    rep = lat.track_frame(rigid_iters=0, icp_iters=2, reset=True)
    hist = []
    out = track.solve_frame_icp(spec, _frame_dict(f, sparse=sparse), PRM, 2, history=hist)
    kept_o = [h[1] for h in hist]
    e_rel = abs(rep["energy"][0] / out["energy"][0] - 1.0)
    pos = lat.get_state64()[0]
    dp = np.abs(pos - out["t"]).max() / spec.spacing
    print(f"tracked torus frame {n}^3 {precision}: kept gpu {list(rep['assoc_kept'])} oracle {kept_o}; "
          f"E rel {e_rel:.2e}, max |dt|/h {dp:.2e}")
    assert rep["assoc_kept"][0] == kept_o[0]
    if precision == "fp64":
        # the second round associates the float64 solve of the first: the
        # same pairs, and the results to rounding-order differences
        assert list(rep["assoc_kept"]) == kept_o
        assert e_rel <= 1e-12
        assert dp <= 1e-10
    else:
        assert abs(rep["assoc_kept"][1] - kept_o[1]) <= 2
        assert e_rel <= 1e-4
        assert dp <= 1e-3


def test_track_frame_errors():
    from paper_1603_08161_amd import Lattice, VDError, VD_ESTATE, VD_EINVAL, VD_ERANGE
    spec = _box_spec(n=8, levels=1)
    lat = Lattice.from_spec(spec)
    with pytest.raises(VDError) as ei:
        lat.track_frame(icp_iters=1)
    assert ei.value.code == VD_ESTATE
    f = make_box_frame(step=20)
    lat.set_depth_frame(f, eps=EPS)
    with pytest.raises(VDError) as ei:
        lat.track_frame(icp_iters=65)
    assert ei.value.code == VD_EINVAL
    far = type(f)(depth=f.depth, camera=f.camera, model_canon=f.model_canon + 10.0,
                  model_normal=f.model_normal)
    with pytest.raises(VDError) as ei:
        lat.set_depth_frame(far, eps=EPS)
    assert ei.value.code == VD_ERANGE
    nan_depth = f.depth.copy()
    nan_depth[3, 3] = np.nan
    bad = type(f)(depth=nan_depth, camera=f.camera, model_canon=f.model_canon,
                  model_normal=f.model_normal)
    with pytest.raises(VDError) as ei:
        lat.set_depth_frame(bad, eps=EPS)
    assert ei.value.code == VD_EINVAL
    with pytest.raises(VDError):
        lat.set_pose([np.nan] + [0.0] * 11)
