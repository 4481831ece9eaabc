"""The no-allocation rigid pose (vd_rigid_pose_noalloc) against the
allocating entry point (vd_rigid_pose): the same kernels on the same inputs,
so the poses and per-iteration histories must be equal bit for bit; two calls
in a row, the second on a smaller input (fewer reduction workgroups), so the
second reads none of the first call's partials."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from synth.scenes import make_box_frame

pytestmark = pytest.mark.gpu

EPS = (0.05, 0.3, 0.95)


def test_noalloc_rigid_pose_equals_rigid_pose_twice():
    import torch

    from paper_1603_08161_amd import rigid_pose, rigid_pose_noalloc
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(21)
    frames = []
    for step in (3, 11):  # about 30k, then about 2.6k samples
        Q = Rotation.from_rotvec(np.deg2rad(1.2) * rng.normal(size=3) / 1.7).as_matrix()
        c = rng.uniform(-0.008, 0.008, size=3)
        frames.append(make_box_frame(Q, c, step=step, noise=5e-4, seed=step))
    assert frames[1].model_canon.shape[0] < frames[0].model_canon.shape[0] // 4
    iters = 5
    for f in frames:
        P_ref, H_ref = rigid_pose(f.camera, f.depth, f.model_canon, f.model_normal, EPS, iters)
        depth = torch.from_numpy(np.ascontiguousarray(f.depth)).to(dev)
        pts = torch.from_numpy(np.ascontiguousarray(f.model_canon)).to(dev)
        nrm = torch.from_numpy(np.ascontiguousarray(f.model_normal)).to(dev)
        pose = torch.tensor(np.concatenate([np.eye(3).ravel(), np.zeros(3)]),
                            dtype=torch.float64, device=dev)
        hist = torch.zeros(2 * iters, dtype=torch.float64, device=dev)
        rigid_pose_noalloc(f.camera, depth, pts, nrm, EPS, iters, pose, hist)
        torch.cuda.synchronize()
        P = pose.cpu().numpy()
        H = hist.cpu().numpy().reshape(iters, 2)
        print(f"{pts.shape[0]} samples: kept {H[:, 1]}, E {H[:, 0]}")
        np.testing.assert_array_equal(P, P_ref)
        np.testing.assert_array_equal(H, H_ref)
        assert H[-1, 0] < 0.05 * H[0, 0]  # down to the depth-noise floor


def test_noalloc_rejects_bad_arguments():
    import torch

    from paper_1603_08161_amd import VDError, rigid_pose_noalloc
    dev = torch.device("cuda", 0)
    f = make_box_frame(step=30)
    depth = torch.from_numpy(np.ascontiguousarray(f.depth)).to(dev)
    pts = torch.from_numpy(np.ascontiguousarray(f.model_canon)).to(dev)
    pose = torch.zeros(12, dtype=torch.float64, device=dev)
    with pytest.raises(VDError):
        rigid_pose_noalloc(f.camera, depth, pts, pts, (0.05, -1.0, 0.9), 1, pose)
    with pytest.raises(ValueError):
        rigid_pose_noalloc(f.camera, f.depth, pts, pts, EPS, 1, pose)  # host depth


def test_noalloc_rejects_sizes_beyond_its_maximum():
    """More samples than VD_NOALLOC_MAX_SAMPLES: VD_ERANGE before any launch."""
    import ctypes as C

    import torch

    from paper_1603_08161_amd import VD_ERANGE, lib
    from paper_1603_08161_amd._lib import VD_NOALLOC_MAX_SAMPLES, _assoc, _camera
    dev = torch.device("cuda", 0)
    f = make_box_frame(step=30)
    depth = torch.from_numpy(np.ascontiguousarray(f.depth)).to(dev)
    pts = torch.from_numpy(np.ascontiguousarray(f.model_canon)).to(dev)
    pose = torch.zeros(12, dtype=torch.float64, device=dev)
    cam, prm = _camera(f.camera), _assoc(EPS)
    rc = lib().vd_rigid_pose_noalloc(C.byref(cam), depth.data_ptr(), pts.data_ptr(),
                                     pts.data_ptr(), VD_NOALLOC_MAX_SAMPLES + 1, C.byref(prm),
                                     1, pose.data_ptr(), None, None)
    assert rc == VD_ERANGE
