"""Non-rigid TSDF fusion (Sec. 8) and marching cubes (Sec. 4) through the
C-ABI (include/vd_fusion.h) against oracle/fusion.py on the same inputs: the
fused distances and confidences bit for bit (decisions and stored values are
float64 from float32 in the same order on both sides), the mesh's cells,
edge numbers and canonical vertices bit for bit, deformed vertices to float32
rounding."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import assoc, fusion
from oracle.lattice import level_grids
from synth.scenes import make_config1

from helpers import random_state

pytestmark = pytest.mark.gpu

EPS = (0.05, 0.3, 0.95)


def _torus(n=40, levels=2):
    scene, frame = make_config1(seed=3, n=n, num_levels=levels, gn=3, pcg=8, depth_frame=True)
    return scene, frame


def _lattice(scene, frame, **kw):
    from paper_1603_08161_amd import Lattice
    lat = Lattice.from_spec(scene.spec, **kw)
    lat.set_depth_frame(frame, sparse_canon=scene.sparse_canon,
                        sparse_target=scene.sparse_target, eps=EPS)
    return lat


def _finest(scene):
    s = scene.spec
    return level_grids(s.dims, s.spacing, s.origin, s.num_levels)[-1]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fusion_of_a_deformed_state_matches_oracle(precision):
    """A random lattice state and pose, a TSDF with some prior content: one
    fusion step into every point against the oracle's."""
    scene, frame = _torus()
    g = _finest(scene)
    lat = _lattice(scene, frame, precision=precision)
    rng = np.random.default_rng(4)
    pos, rot = random_state(g, rng, amp=0.15, rot_amp=0.05)
    lat.set_state(pos, rot)
    Rg = Rotation.from_rotvec([0.01, -0.02, 0.015]).as_matrix()
    pose = np.concatenate([Rg.ravel(), [0.004, -0.003, 0.006]])
    lat.set_pose(pose)
    D0 = rng.uniform(-1, 1, size=g.n).astype(np.float32)
    W0 = rng.integers(0, 4, size=g.n).astype(np.float32)
    lat.set_tsdf(D0, W0)
    tau = 2.5 * scene.spec.spacing
    n = lat.fuse_depth(tau=tau, w_max=3.0, all_points=True)
    D, W, _ = lat.get_tsdf()
    # the state as the GPU holds it: displacements from the exported positions
    disp = (lat.get_state()[0].astype(np.float64) - g.rest_positions())
    if precision == "fp32":
        disp = disp.astype(np.float32).astype(np.float64)
    Do, Wo, no = fusion.integrate(g, D0, W0, disp, pose, assoc.Camera(**frame.camera),
                                  frame.depth, np.ones(g.n, bool), tau, 3.0)
    print(f"{precision}: {n} of {g.n} points fused")
    # the state reaches the oracle through exported float32 positions, so its
    # displacements can differ from the GPU's in the last bits: decisions
    # agree except at ties, values to float32 rounding
    same = W == Wo
    assert same.mean() > 0.999
    np.testing.assert_allclose(D[same], Do[same], rtol=0, atol=2e-7 if precision == "fp64" else 1e-5)
    assert n > 0.05 * g.n


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fusion_at_rest_with_a_pose_is_bitwise(precision):
    """At rest (d = 0 exactly on both sides) with a global pose: the fused
    distances and confidences equal the oracle's bit for bit."""
    scene, frame = _torus()
    g = _finest(scene)
    lat = _lattice(scene, frame, precision=precision)
    Rg = Rotation.from_rotvec([-0.012, 0.02, 0.01]).as_matrix()
    pose = np.concatenate([Rg.ravel(), [-0.006, 0.002, 0.004]])
    lat.set_pose(pose)
    rng = np.random.default_rng(6)
    D0 = rng.uniform(-1, 1, size=g.n).astype(np.float32)
    W0 = rng.integers(0, 4, size=g.n).astype(np.float32)
    lat.set_tsdf(D0, W0)
    tau = 2.5 * scene.spec.spacing
    n = lat.fuse_depth(tau=tau, w_max=3.0, all_points=True)
    D, W, _ = lat.get_tsdf()
    Do, Wo, no = fusion.integrate(g, D0, W0, np.zeros((g.n, 3)), pose,
                                  assoc.Camera(**frame.camera), frame.depth, np.ones(g.n, bool),
                                  tau, 3.0)
    assert n == no > 0
    np.testing.assert_array_equal(W, Wo)
    np.testing.assert_array_equal(D, Do)


def test_fusion_respects_the_optimised_set_and_k_min():
    """With the active set, only points of M optimised for k_min frames in a
    row are fused."""
    scene, frame = _torus(n=32)
    lat = _lattice(scene, frame, active_set=True, precision="fp64")
    for k in range(2):
        lat.track_frame(rigid_iters=0, icp_iters=1, reset=(k == 0), report=False)
    _, _, frames = lat.get_tsdf()
    act, _, _ = lat.get_active()
    np.testing.assert_array_equal(frames, np.where(act, 2, 0))
    assert lat.fuse_depth(tau=0.05, k_min=3) == 0           # two frames so far
    lat.track_frame(rigid_iters=0, icp_iters=1, report=False)
    n = lat.fuse_depth(tau=0.05, k_min=3)
    D, W, frames = lat.get_tsdf()
    assert 0 < n <= int(act.sum())
    assert np.all(W[~act] == 0)


def test_marching_cubes_matches_oracle_bitwise():
    """A TSDF of a warped torus surface (fused from its depth map at rest),
    with a random lattice state: cells, edges and canonical vertices equal,
    deformed vertices to float32 rounding."""
    scene, frame = _torus(n=40)
    g = _finest(scene)
    lat = _lattice(scene, frame, precision="fp64")
    lat.fuse_depth(tau=3.0 * scene.spec.spacing, all_points=True)
    rng = np.random.default_rng(5)
    pos, rot = random_state(g, rng, amp=0.1, rot_amp=0.02)
    lat.set_state(pos, rot)
    canon, deformed, cells, edges = lat.extract_mesh()
    D, W, _ = lat.get_tsdf()
    c_o, e_o, v_o = fusion.marching_cubes(g, D, W)
    print(f"{cells.size} triangles")
    assert cells.size > 1000
    np.testing.assert_array_equal(cells, c_o)
    np.testing.assert_array_equal(edges, e_o)
    np.testing.assert_array_equal(canon, v_o)
    disp = lat.get_state()[0].astype(np.float64) - g.rest_positions()
    ref = fusion.deform_vertices(g, disp, np.concatenate([np.eye(3).ravel(), np.zeros(3)]),
                                 v_o.reshape(-1, 3)).reshape(-1, 3, 3)
    np.testing.assert_allclose(deformed, ref, rtol=0, atol=1e-6)


def test_mesh_capacity_and_empty_volume():
    from paper_1603_08161_amd import VD_ERANGE, lib
    import ctypes as C
    scene, frame = _torus(n=24)
    lat = _lattice(scene, frame)
    canon, deformed, cells, edges = lat.extract_mesh()      # nothing observed yet
    assert cells.size == 0
    lat.fuse_depth(tau=0.05, all_points=True)
    n = C.c_int64()
    buf = np.empty((4, 3, 3), np.float32)
    rc = lib().vd_extract_mesh(lat._h, 4, buf.ctypes.data, None, None, None, C.byref(n), 0)
    assert rc == VD_ERANGE and n.value > 4
