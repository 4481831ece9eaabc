"""ctypes binding of libvd.so (the C-ABI in include/vd.h, include/vd_net.h,
include/vd_track.h and include/vd_fusion.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Arrays may be numpy (host memory) or torch CUDA tensors (device
memory of the handle's GPU); a call takes one kind for all its arrays.  If
libvd.so has not been built this module raises at import time -- there is no
fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

try:  # load torch's HIP runtime first so the library shares it
    import torch  # noqa: F401
    _HAVE_TORCH = True
except Exception:  # pragma: no cover
    torch = None
    _HAVE_TORCH = False

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvd.so")

VD_OK, VD_EINVAL, VD_ERANGE, VD_ENOMEM, VD_EHIP, VD_ESTATE = 0, -1, -2, -3, -4, -5
VD_FP32_FP64RED, VD_FP64 = 0, 1
VD_MEM_HOST, VD_MEM_DEVICE = 0, 1
VD_FLAG_GRAPH, VD_FLAG_TRACE, VD_FLAG_PROFILE, VD_FLAG_PERSIST = 1, 2, 4, 8
VD_FLAG_ACTIVE_SET = 16
VD_FLAG_ITERATIVE = 32
VD_PROF_KINDS = 8
PROF_NAMES = ("gradient", "cg_a", "cg_b", "rotation", "energy", "transfer", "cg_loop")
VD_REPORT_PCG_GUARD, VD_REPORT_POLAR_FP64, VD_REPORT_POLAR_KEEP = 1, 2, 4
VD_REPORT_WARM_REJECTED = 8
VD_REPORT_BARRIER_TIMEOUT = 16
VD_MAX_LEVELS = 4
VD_TILE_KINDS = 8
VD_MAX_TRACE = 512

EXPORTED = (
    "vd_lattice_create", "vd_lattice_destroy", "vd_set_constraints", "vd_solve_frame",
    "vd_get_energy", "vd_get_state", "vd_set_state", "vd_level_info", "vd_strerror",
    "vd_debug_apply", "vd_debug_gradient", "vd_debug_energy", "vd_debug_diag",
    "vd_debug_rotations", "vd_debug_fit_rotations", "vd_debug_prolong", "vd_tune",
    "vd_batch_create", "vd_batch_solve", "vd_batch_destroy", "vd_batch_profile",
    "vd_get_profile", "vd_warm_features", "vd_net_param_count", "vd_net_create", "vd_net_destroy",
    "vd_net_set_params", "vd_net_get_params", "vd_net_forward", "vd_net_gradients",
    "vd_net_train_step", "vd_associate", "vd_rigid_pose", "vd_set_depth_frame", "vd_get_pose",
    "vd_set_pose", "vd_track_frame", "vd_debug_associate", "vd_rigid_pose_noalloc",
    "vd_get_active", "vd_fuse_depth", "vd_get_tsdf", "vd_set_tsdf", "vd_extract_mesh",
    "vd_debug_sort_pairs", "vd_debug_exclusive_scan", "vd_batch_tune", "vd_get_state64",
)
VD_TRACK_MAX_ITERS = 64
VD_NOALLOC_MAX_SAMPLES = 1 << 30


class LatticeDesc(C.Structure):
    _fields_ = [
        ("dims", C.c_int32 * 3),
        ("spacing", C.c_double),
        ("origin", C.c_double * 3),
        ("num_levels", C.c_int32),
        ("gn_iters", C.c_int32 * VD_MAX_LEVELS),
        ("pcg_iters", C.c_int32 * VD_MAX_LEVELS),
        ("w_dense", C.c_double),
        ("w_sparse", C.c_double),
        ("w_arap", C.c_double),
        ("precision", C.c_int32),
        ("flags", C.c_uint32),
        ("tile", C.c_int32 * VD_MAX_LEVELS),
    ]


class Constraints(C.Structure):
    _fields_ = [
        ("n_dense", C.c_int64),
        ("canon", C.c_void_p),
        ("target", C.c_void_p),
        ("normal", C.c_void_p),
        ("weight", C.c_void_p),
        ("n_sparse", C.c_int64),
        ("sparse_canon", C.c_void_p),
        ("sparse_target", C.c_void_p),
        ("mem", C.c_int32),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("reset_to_rest", C.c_int32),
        ("init_mem", C.c_int32),
        ("init_delta", C.c_void_p),
        ("energy_target", C.c_double),
        ("max_gn", C.c_int32),
        ("warm_mode", C.c_int32),
    ]


class SolveReport(C.Structure):
    _fields_ = [
        ("energy", C.c_double * 4),
        ("bits", C.c_uint32),
        ("polar_fp64", C.c_int32),
        ("polar_keep", C.c_int32),
        ("n_trace", C.c_int32),
        ("trace", C.c_double * VD_MAX_TRACE),
        ("prof_us", C.c_double * VD_PROF_KINDS),
        ("prof_n", C.c_int32 * VD_PROF_KINDS),
        ("init_energy", C.c_double * 2),
        ("warm_used", C.c_int32),
        ("gn_done", C.c_int32),
        ("target_reached", C.c_int32),
        ("reserved", C.c_int32),
    ]


class Camera(C.Structure):
    _fields_ = [
        ("width", C.c_int32),
        ("height", C.c_int32),
        ("fx", C.c_double),
        ("fy", C.c_double),
        ("cx", C.c_double),
        ("cy", C.c_double),
    ]


class AssocParams(C.Structure):
    _fields_ = [("eps_d", C.c_double), ("eps_n", C.c_double), ("eps_v", C.c_double)]


class DepthFrameC(C.Structure):
    _fields_ = [
        ("camera", Camera),
        ("depth", C.c_void_p),
        ("n_model", C.c_int64),
        ("model_canon", C.c_void_p),
        ("model_normal", C.c_void_p),
        ("n_sparse", C.c_int64),
        ("sparse_canon", C.c_void_p),
        ("sparse_target", C.c_void_p),
        ("assoc", AssocParams),
        ("mem", C.c_int32),
        ("reserved", C.c_int32),
    ]


class FuseOpts(C.Structure):
    _fields_ = [
        ("tau", C.c_double),
        ("w_max", C.c_double),
        ("k_min", C.c_int32),
        ("all_points", C.c_int32),
    ]


class TrackOpts(C.Structure):
    _fields_ = [
        ("rigid_iters", C.c_int32),
        ("icp_iters", C.c_int32),
        ("reset_to_rest", C.c_int32),
        ("reserved", C.c_int32),
    ]


class TrackReport(C.Structure):
    _fields_ = [
        ("energy", C.c_double * 4),
        ("pose", C.c_double * 12),
        ("rigid_hist", C.c_double * (2 * VD_TRACK_MAX_ITERS)),
        ("assoc_kept", C.c_int32 * VD_TRACK_MAX_ITERS),
        ("bits", C.c_uint32),
        ("reserved", C.c_int32),
    ]


def _camera(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    return c


def _assoc(eps) -> AssocParams:
    a = AssocParams()
    a.eps_d, a.eps_n, a.eps_v = (float(e) for e in eps)
    return a


class VDError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python paper_1603_08161_amd/build.py` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "vd_lattice_create": ([C.POINTER(LatticeDesc), vp, C.POINTER(vp)], C.c_int),
        "vd_lattice_destroy": ([vp], C.c_int),
        "vd_set_constraints": ([vp, C.POINTER(Constraints)], C.c_int),
        "vd_solve_frame": ([vp, C.POINTER(SolveOpts), C.POINTER(SolveReport)], C.c_int),
        "vd_get_energy": ([vp, dp], C.c_int),
        "vd_get_state": ([vp, vp, vp, i32], C.c_int),
        "vd_set_state": ([vp, vp, vp, i32], C.c_int),
        "vd_level_info": ([vp, i32, C.POINTER(C.c_int32), dp], C.c_int),
        "vd_strerror": ([C.c_int], C.c_char_p),
        "vd_debug_apply": ([vp, i32, vp, vp, i32], C.c_int),
        "vd_debug_gradient": ([vp, i32, vp, vp, vp, i32], C.c_int),
        "vd_debug_energy": ([vp, i32, vp, vp, dp, i32], C.c_int),
        "vd_debug_diag": ([vp, i32, vp, i32], C.c_int),
        "vd_debug_rotations": ([vp, i32, vp, vp, vp, i32], C.c_int),
        "vd_debug_fit_rotations": ([vp, vp, vp, vp, i64, i32, i32, vp], C.c_int),
        "vd_debug_sort_pairs": ([vp, vp, vp, vp, i64, i32, i32, vp], C.c_int),
        "vd_debug_exclusive_scan": ([vp, vp, i64, i32, vp], C.c_int),
        "vd_batch_tune": ([vp, i32, C.POINTER(C.c_int32), dp], C.c_int),
        "vd_get_state64": ([vp, vp, vp, i32], C.c_int),
        "vd_debug_prolong": ([vp, i32, vp, vp, i32], C.c_int),
        "vd_tune": ([vp, i32, C.POINTER(C.c_int32), dp], C.c_int),
        "vd_batch_create": ([C.POINTER(vp), i32, C.POINTER(vp)], C.c_int),
        "vd_batch_solve": ([vp, C.POINTER(SolveOpts), dp], C.c_int),
        "vd_batch_destroy": ([vp], C.c_int),
        "vd_batch_profile": ([vp, dp, C.POINTER(C.c_int32)], C.c_int),
        "vd_get_profile": ([vp, dp, C.POINTER(C.c_int32)], C.c_int),
        "vd_warm_features": ([vp, vp, vp, i32], C.c_int),
        "vd_net_param_count": ([], i64),
        "vd_net_create": ([i32, i32, i32, i32, vp, C.POINTER(vp)], C.c_int),
        "vd_net_destroy": ([vp], C.c_int),
        "vd_net_set_params": ([vp, vp, i32], C.c_int),
        "vd_net_get_params": ([vp, vp, i32], C.c_int),
        "vd_net_forward": ([vp, vp, i32, vp, i32], C.c_int),
        "vd_net_gradients": ([vp, vp, vp, i32, vp, dp, i32], C.c_int),
        "vd_net_train_step": ([vp, vp, vp, i32, C.c_float, i32, dp], C.c_int),
        "vd_associate": ([C.POINTER(Camera), vp, vp, vp, i64, C.POINTER(AssocParams), vp, vp, vp,
                          vp, i32, vp], C.c_int),
        "vd_rigid_pose": ([C.POINTER(Camera), vp, vp, vp, i64, C.POINTER(AssocParams), i32, vp, vp,
                           i32, vp], C.c_int),
        "vd_set_depth_frame": ([vp, C.POINTER(DepthFrameC)], C.c_int),
        "vd_get_pose": ([vp, dp], C.c_int),
        "vd_set_pose": ([vp, dp], C.c_int),
        "vd_track_frame": ([vp, C.POINTER(TrackOpts), C.POINTER(TrackReport)], C.c_int),
        "vd_debug_associate": ([vp, vp, vp, vp, vp, vp, vp, i32], C.c_int),
        "vd_rigid_pose_noalloc": ([C.POINTER(Camera), vp, vp, vp, i64, C.POINTER(AssocParams),
                                   i32, vp, vp, vp], C.c_int),
        "vd_get_active": ([vp, i32, vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
        "vd_fuse_depth": ([vp, C.POINTER(FuseOpts), C.POINTER(C.c_int64)], C.c_int),
        "vd_get_tsdf": ([vp, vp, vp, vp, i32], C.c_int),
        "vd_set_tsdf": ([vp, vp, vp, i32], C.c_int),
        "vd_extract_mesh": ([vp, i64, vp, vp, vp, vp, C.POINTER(C.c_int64), i32], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib() -> C.CDLL:
    return _lib


def strerror(code: int) -> str:
    return _lib.vd_strerror(code).decode()


def _check(code: int, what: str) -> None:
    if code != VD_OK:
        raise VDError(code, what)


def _is_device(a) -> bool:
    return _HAVE_TORCH and isinstance(a, torch.Tensor) and a.is_cuda


def _prep(arrays, allow_none=()):
    """Return (pointers, mem, keepalive) for a list of arrays of one kind."""
    present = [a for a in arrays if a is not None]
    dev = [_is_device(a) for a in present]
    if any(dev) and not all(dev):
        raise ValueError("mix of host and device arrays in one call")
    mem = VD_MEM_DEVICE if (present and dev[0]) else VD_MEM_HOST
    ptrs, keep = [], []
    for a in arrays:
        if a is None:
            ptrs.append(None)
            continue
        if mem == VD_MEM_DEVICE:
            if a.dtype != torch.float32 or not a.is_contiguous():
                raise ValueError("device arrays must be contiguous float32 tensors")
            ptrs.append(a.data_ptr())
            keep.append(a)
        else:
            h = np.ascontiguousarray(a, dtype=np.float32)
            keep.append(h)
            ptrs.append(h.ctypes.data)
    return ptrs, mem, keep


def _host(a) -> np.ndarray:
    if _HAVE_TORCH and isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float32)


def _current_stream() -> int:
    if _HAVE_TORCH and torch.cuda.is_available():
        return int(torch.cuda.current_stream().cuda_stream)
    return 0


class Lattice:
    """A lattice handle (vd_lattice*)."""

    def __init__(self, dims, spacing, origin, num_levels=1, gn_iters=(5,), pcg_iters=(10,),
                 w_dense=1.0, w_sparse=10.0, w_arap=5.0, precision="fp32",
                 graph=False, trace=False, profile=False, tiles=None, persistent=False,
                 active_set=False, iterative=False, stream: Optional[int] = None):
        d = LatticeDesc()
        for k in range(3):
            d.dims[k] = int(dims[k])
            d.origin[k] = float(origin[k])
        d.spacing = float(spacing)
        d.num_levels = int(num_levels)
        for k in range(VD_MAX_LEVELS):
            d.gn_iters[k] = int(gn_iters[k]) if k < len(gn_iters) else 0
            d.pcg_iters[k] = int(pcg_iters[k]) if k < len(pcg_iters) else 0
        d.w_dense, d.w_sparse, d.w_arap = float(w_dense), float(w_sparse), float(w_arap)
        d.precision = VD_FP64 if precision == "fp64" else VD_FP32_FP64RED
        d.flags = ((VD_FLAG_GRAPH if graph else 0) | (VD_FLAG_TRACE if trace else 0)
                   | (VD_FLAG_PROFILE if profile else 0)
                   | (VD_FLAG_PERSIST if persistent else 0)
                   | (VD_FLAG_ACTIVE_SET if active_set else 0)
                   | (VD_FLAG_ITERATIVE if iterative else 0))
        for k in range(VD_MAX_LEVELS):
            d.tile[k] = int(tiles[k]) if tiles is not None and k < len(tiles) else 0
        self.desc = d
        self.stream = _current_stream() if stream is None else int(stream)
        h = C.c_void_p()
        _check(_lib.vd_lattice_create(C.byref(d), C.c_void_p(self.stream), C.byref(h)),
               "vd_lattice_create")
        self._h = h
        self.num_levels = int(num_levels)

    @classmethod
    def from_spec(cls, spec, **kw):
        return cls(spec.dims, spec.spacing, spec.origin, spec.num_levels, spec.gn_iters,
                   spec.pcg_iters, spec.w_dense, spec.w_sparse, spec.w_arap, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.vd_lattice_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def level_info(self, level: int) -> Tuple[Tuple[int, int, int], float]:
        dims = (C.c_int32 * 3)()
        h = C.c_double()
        _check(_lib.vd_level_info(self._h, level, dims, C.byref(h)), "vd_level_info")
        return (dims[0], dims[1], dims[2]), h.value

    def n_nodes(self, level: int = -1) -> int:
        lvl = self.num_levels - 1 if level < 0 else level
        d, _ = self.level_info(lvl)
        return d[0] * d[1] * d[2]

    def set_constraints(self, canon, target, normal, weight=None, sparse_canon=None,
                        sparse_target=None) -> None:
        ptrs, mem, keep = _prep([canon, target, normal, weight, sparse_canon, sparse_target])
        c = Constraints()
        c.n_dense = 0 if canon is None else int(canon.shape[0])
        c.canon, c.target, c.normal, c.weight = ptrs[0], ptrs[1], ptrs[2], ptrs[3]
        c.n_sparse = 0 if sparse_canon is None else int(sparse_canon.shape[0])
        c.sparse_canon, c.sparse_target = ptrs[4], ptrs[5]
        c.mem = mem
        _check(_lib.vd_set_constraints(self._h, C.byref(c)), "vd_set_constraints")
        del keep

    def set_scene(self, scene) -> None:
        self.set_constraints(scene.canon, scene.target, scene.normal, scene.weight,
                             scene.sparse_canon, scene.sparse_target)

    def solve_frame(self, reset: bool = False, report: bool = False, init_delta=None,
                    energy_target: float = 0.0, max_gn: int = 0, warm_step: bool = False):
        """Solve one frame.  init_delta ([3][N] float32, units of the finest
        spacing, numpy or CUDA tensor) asks for the judged warm start (with
        warm_step: the exact line minimum of E along init_delta instead of
        adding it); energy_target > 0 runs finest-level iterations until
        E <= it (at most max_gn, 0 = the schedule's count)."""
        o = SolveOpts()
        o.reset_to_rest = 1 if reset else 0
        o.warm_mode = 1 if warm_step else 0
        keep = None
        if init_delta is not None:
            (ptr,), mem, keep = _prep([init_delta])
            o.init_delta = ptr
            o.init_mem = mem
        o.energy_target = float(energy_target)
        o.max_gn = int(max_gn)
        if not report:
            _check(_lib.vd_solve_frame(self._h, C.byref(o), None), "vd_solve_frame")
            return None
        r = SolveReport()
        _check(_lib.vd_solve_frame(self._h, C.byref(o), C.byref(r)), "vd_solve_frame")
        del keep
        return {"energy": np.array(r.energy[:]), "bits": int(r.bits),
                "polar_fp64": int(r.polar_fp64), "polar_keep": int(r.polar_keep),
                "trace": np.array(r.trace[:r.n_trace]),
                "prof_us": {PROF_NAMES[k]: float(r.prof_us[k]) for k in range(len(PROF_NAMES))
                            if r.prof_n[k] > 0},
                "prof_n": {PROF_NAMES[k]: int(r.prof_n[k]) for k in range(len(PROF_NAMES))
                           if r.prof_n[k] > 0},
                "init_energy": np.array(r.init_energy[:]), "warm_used": int(r.warm_used),
                "gn_done": int(r.gn_done), "target_reached": int(r.target_reached)}

    def warm_features(self, prev2=None, out=None):
        """Input features of the warm-start network (vd_warm_features) as
        [nz][ny][nx][8] bfloat16 bit patterns: a uint16 numpy array, or written
        into `out` (a contiguous int16 CUDA tensor of 8N elements)."""
        n = self.n_nodes()
        if out is not None:
            if not (_is_device(out) and out.dtype == torch.int16 and out.is_contiguous()
                    and out.numel() == 8 * n):
                raise ValueError("out must be a contiguous int16 CUDA tensor of 8N elements")
            p2 = None
            if prev2 is not None:
                (p2,), mem, keep = _prep([prev2])
                if mem != VD_MEM_DEVICE:
                    raise ValueError("prev2 must be on the device when out is")
            _check(_lib.vd_warm_features(self._h, p2, out.data_ptr(), VD_MEM_DEVICE),
                   "vd_warm_features")
            return out
        p2 = None
        keep = None
        if prev2 is not None:
            p2h = _host(prev2)
            keep = p2h
            p2 = p2h.ctypes.data
        x = np.empty(8 * n, np.uint16)
        _check(_lib.vd_warm_features(self._h, p2, x.ctypes.data, VD_MEM_HOST), "vd_warm_features")
        del keep
        return x.reshape(self.level_info(self.num_levels - 1)[0][::-1] + (8,))

    def profile(self):
        """Mean us per launch by kernel class over the last frame (profile=True)."""
        us = (C.c_double * VD_PROF_KINDS)()
        n = (C.c_int32 * VD_PROF_KINDS)()
        _check(_lib.vd_get_profile(self._h, us, n), "vd_get_profile")
        return ({PROF_NAMES[k]: float(us[k]) for k in range(len(PROF_NAMES)) if n[k] > 0},
                {PROF_NAMES[k]: int(n[k]) for k in range(len(PROF_NAMES)) if n[k] > 0})

    def tune(self, iters: int = 10):
        """Run the library's tile autotuner; returns (tiles per level, us per CG
        iteration with the gradient pass included [level][kind])."""
        tiles = (C.c_int32 * VD_MAX_LEVELS)()
        us = (C.c_double * (VD_TILE_KINDS * VD_MAX_LEVELS))()
        _check(_lib.vd_tune(self._h, int(iters), tiles, us), "vd_tune")
        n = self.num_levels
        return ([int(tiles[k]) for k in range(n)],
                [[float(us[VD_TILE_KINDS * k + j]) for j in range(VD_TILE_KINDS)]
                 for k in range(n)])

    def get_energy(self) -> np.ndarray:
        out = (C.c_double * 4)()
        _check(_lib.vd_get_energy(self._h, out), "vd_get_energy")
        return np.array(out[:])

    def get_state(self):
        n = self.n_nodes()
        pos = np.empty((n, 3), np.float32)
        rot = np.empty((n, 3, 3), np.float32)
        _check(_lib.vd_get_state(self._h, pos.ctypes.data, rot.ctypes.data, VD_MEM_HOST),
               "vd_get_state")
        return pos, rot

    def get_state64(self):
        """The finest state in float64: (positions (N, 3), rotations (N, 3, 3))."""
        n = self.n_nodes()
        pos = np.empty((n, 3), np.float64)
        rot = np.empty((n, 3, 3), np.float64)
        _check(_lib.vd_get_state64(self._h, pos.ctypes.data, rot.ctypes.data, VD_MEM_HOST),
               "vd_get_state64")
        return pos, rot

    def set_state(self, pos, rot=None) -> None:
        ptrs, mem, keep = _prep([pos, rot])
        _check(_lib.vd_set_state(self._h, ptrs[0], ptrs[1], mem), "vd_set_state")
        del keep

    # ---- test entry points ------------------------------------------
    def get_active(self, level: int = -1):
        """(mask (N,) bool, count, growth layers of the last build) of the
        optimised set M of a level (every point without active_set)."""
        lvl = self.num_levels - 1 if level < 0 else level
        n = self.n_nodes(lvl)
        mask = np.empty(n, np.uint8)
        cnt = C.c_int64()
        layers = C.c_int32()
        _check(_lib.vd_get_active(self._h, lvl, mask.ctypes.data, C.byref(cnt), C.byref(layers)),
               "vd_get_active")
        return mask.astype(bool), int(cnt.value), int(layers.value)

    # ---- fusion and mesh extraction (vd_fusion.h) ------------------------
    def fuse_depth(self, tau: float, w_max: float = 64.0, k_min: int = 3,
                   all_points: bool = False, count: bool = True):
        """Fuse the handle's depth frame into its TSDF; returns the number of
        grid points updated (None with count=False: asynchronous)."""
        o = FuseOpts()
        o.tau, o.w_max, o.k_min, o.all_points = float(tau), float(w_max), int(k_min), int(all_points)
        if not count:
            _check(_lib.vd_fuse_depth(self._h, C.byref(o), None), "vd_fuse_depth")
            return None
        n = C.c_int64()
        _check(_lib.vd_fuse_depth(self._h, C.byref(o), C.byref(n)), "vd_fuse_depth")
        return int(n.value)

    def get_tsdf(self):
        n = self.n_nodes()
        D = np.empty(n, np.float32)
        W = np.empty(n, np.float32)
        F = np.empty(n, np.int32)
        _check(_lib.vd_get_tsdf(self._h, D.ctypes.data, W.ctypes.data, F.ctypes.data,
                                VD_MEM_HOST), "vd_get_tsdf")
        return D, W, F

    def set_tsdf(self, D, W) -> None:
        D = np.ascontiguousarray(D, np.float32)
        W = np.ascontiguousarray(W, np.float32)
        _check(_lib.vd_set_tsdf(self._h, D.ctypes.data, W.ctypes.data, VD_MEM_HOST),
               "vd_set_tsdf")

    def extract_mesh(self):
        """Marching cubes: (canonical vertices (T,3,3), deformed vertices
        (T,3,3), cells (T,), edge numbers (T,3))."""
        n = C.c_int64()
        rc = _lib.vd_extract_mesh(self._h, 0, None, None, None, None, C.byref(n), VD_MEM_HOST)
        if rc not in (VD_OK, VD_ERANGE):
            _check(rc, "vd_extract_mesh")
        T = int(n.value)
        canon = np.empty((T, 3, 3), np.float32)
        deformed = np.empty((T, 3, 3), np.float32)
        cells = np.empty(T, np.int32)
        edges = np.empty((T, 3), np.int32)
        if T:
            _check(_lib.vd_extract_mesh(self._h, T, canon.ctypes.data, deformed.ctypes.data,
                                        cells.ctypes.data, edges.ctypes.data, C.byref(n),
                                        VD_MEM_HOST), "vd_extract_mesh")
        return canon, deformed, cells, edges

    # ---- tracking (vd_track.h) --------------------------------------------
    def set_depth_frame(self, frame, sparse_canon=None, sparse_target=None,
                        eps=(0.05, 0.3, 0.95)) -> None:
        """Upload one sensor frame (depth map, camera, canonical model samples
        and normals; optional sparse pairs with camera-frame targets)."""
        ptrs, mem, keep = _prep([frame.depth, frame.model_canon, frame.model_normal,
                                 sparse_canon, sparse_target])
        f = DepthFrameC()
        f.camera = _camera(frame.camera)
        f.depth = ptrs[0]
        f.n_model = int(frame.model_canon.shape[0])
        f.model_canon, f.model_normal = ptrs[1], ptrs[2]
        f.n_sparse = 0 if sparse_canon is None else int(sparse_canon.shape[0])
        f.sparse_canon, f.sparse_target = ptrs[3], ptrs[4]
        f.assoc = _assoc(eps)
        f.mem = mem
        _check(_lib.vd_set_depth_frame(self._h, C.byref(f)), "vd_set_depth_frame")
        self.n_model = int(f.n_model)
        del keep

    def get_pose(self) -> np.ndarray:
        out = (C.c_double * 12)()
        _check(_lib.vd_get_pose(self._h, out), "vd_get_pose")
        return np.array(out[:])

    def set_pose(self, pose) -> None:
        arr = (C.c_double * 12)(*[float(x) for x in np.asarray(pose, np.float64).ravel()])
        _check(_lib.vd_set_pose(self._h, arr), "vd_set_pose")

    def track_frame(self, rigid_iters: int = 0, icp_iters: int = 1, reset: bool = False,
                    report: bool = True):
        o = TrackOpts()
        o.rigid_iters, o.icp_iters, o.reset_to_rest = int(rigid_iters), int(icp_iters), int(reset)
        if not report:
            _check(_lib.vd_track_frame(self._h, C.byref(o), None), "vd_track_frame")
            return None
        r = TrackReport()
        _check(_lib.vd_track_frame(self._h, C.byref(o), C.byref(r)), "vd_track_frame")
        return {"energy": np.array(r.energy[:]), "pose": np.array(r.pose[:]),
                "rigid_hist": np.array(r.rigid_hist[:2 * o.rigid_iters]).reshape(-1, 2),
                "assoc_kept": np.array(r.assoc_kept[:o.icp_iters]), "bits": int(r.bits)}

    def debug_associate(self, disp, rot):
        """Association of the frame's model samples at a finest state
        (displacements (N,3), rotations (N,3,3)) and the handle's pose."""
        n = self.n_model
        d = np.ascontiguousarray(disp, np.float32).reshape(-1)
        R = np.ascontiguousarray(rot, np.float32).reshape(-1)
        t = np.empty((n, 3), np.float32)
        nn = np.empty((n, 3), np.float32)
        w = np.empty(n, np.float32)
        px = np.empty(n, np.int32)
        _check(_lib.vd_debug_associate(self._h, d.ctypes.data, R.ctypes.data, t.ctypes.data,
                                       nn.ctypes.data, w.ctypes.data, px.ctypes.data,
                                       VD_MEM_HOST), "vd_debug_associate")
        return t, nn, w, px

    # ------------------------------------------------------------------
    def debug_apply(self, level: int, p) -> np.ndarray:
        n = self.n_nodes(level)
        p = _host(p)
        out = np.empty((n, 3), np.float32)
        _check(_lib.vd_debug_apply(self._h, level, p.ctypes.data, out.ctypes.data, VD_MEM_HOST),
               "vd_debug_apply")
        return out

    def debug_gradient(self, level: int, pos, rot) -> np.ndarray:
        n = self.n_nodes(level)
        pos, rot = _host(pos), _host(rot)
        out = np.empty((n, 3), np.float32)
        _check(_lib.vd_debug_gradient(self._h, level, pos.ctypes.data, rot.ctypes.data,
                                      out.ctypes.data, VD_MEM_HOST), "vd_debug_gradient")
        return out

    def debug_energy(self, level: int, pos, rot) -> np.ndarray:
        pos, rot = _host(pos), _host(rot)
        out = (C.c_double * 4)()
        _check(_lib.vd_debug_energy(self._h, level, pos.ctypes.data, rot.ctypes.data, out,
                                    VD_MEM_HOST), "vd_debug_energy")
        return np.array(out[:])

    def debug_diag(self, level: int) -> np.ndarray:
        n = self.n_nodes(level)
        out = np.empty((n, 3), np.float32)
        _check(_lib.vd_debug_diag(self._h, level, out.ctypes.data, VD_MEM_HOST), "vd_debug_diag")
        return out

    def debug_rotations(self, level: int, pos, rot_prev) -> np.ndarray:
        n = self.n_nodes(level)
        pos, rot_prev = _host(pos), _host(rot_prev)
        out = np.empty((n, 3, 3), np.float32)
        _check(_lib.vd_debug_rotations(self._h, level, pos.ctypes.data, rot_prev.ctypes.data,
                                       out.ctypes.data, VD_MEM_HOST), "vd_debug_rotations")
        return out

    def debug_prolong(self, level: int, coarse) -> np.ndarray:
        n = self.n_nodes(level)
        coarse = _host(coarse)
        out = np.empty((n, 3), np.float32)
        _check(_lib.vd_debug_prolong(self._h, level, coarse.ctypes.data, out.ctypes.data,
                                     VD_MEM_HOST), "vd_debug_prolong")
        return out


class Batch:
    """A batch of lattice handles solved together (vd_batch*): one launch per
    schedule step covers every lattice.  Keeps references to the handles."""

    def __init__(self, lattices):
        self.lattices = list(lattices)
        arr = (C.c_void_p * len(self.lattices))(*[l._h.value for l in self.lattices])
        h = C.c_void_p()
        _check(_lib.vd_batch_create(arr, len(self.lattices), C.byref(h)), "vd_batch_create")
        self._h = h

    def solve(self, reset: bool = False, energies: bool = False):
        o = SolveOpts()
        o.reset_to_rest = 1 if reset else 0
        if not energies:
            _check(_lib.vd_batch_solve(self._h, C.byref(o), None), "vd_batch_solve")
            return None
        out = (C.c_double * (4 * len(self.lattices)))()
        _check(_lib.vd_batch_solve(self._h, C.byref(o), out), "vd_batch_solve")
        return np.array(out[:]).reshape(-1, 4)

    def profile(self):
        """Mean us per finest-level launch by kernel class (profiled batches)."""
        us = (C.c_double * VD_PROF_KINDS)()
        n = (C.c_int32 * VD_PROF_KINDS)()
        _check(_lib.vd_batch_profile(self._h, us, n), "vd_batch_profile")
        return {PROF_NAMES[k]: float(us[k]) for k in range(len(PROF_NAMES)) if n[k] > 0}

    def tune(self, iters: int = 10):
        """Batch tile autotuner (vd_batch_tune): returns ({"fp32": tiles per
        level, "fp64": ...} for the parts present, us per CG iteration with
        the gradient pass included [part][level][kind])."""
        tiles = (C.c_int32 * (2 * VD_MAX_LEVELS))()
        us = (C.c_double * (2 * VD_MAX_LEVELS * VD_TILE_KINDS))()
        _check(_lib.vd_batch_tune(self._h, int(iters), tiles, us), "vd_batch_tune")
        out = {}
        for k, name in enumerate(("fp32", "fp64")):
            t = [int(tiles[k * VD_MAX_LEVELS + l]) for l in range(VD_MAX_LEVELS)]
            if any(t):
                out[name] = [x for x in t if x]
        u = np.array(us[:]).reshape(2, VD_MAX_LEVELS, VD_TILE_KINDS)
        return out, u

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.vd_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def associate(cam, depth, points, normals, eps, stream: Optional[int] = None):
    """Projective association of camera-frame samples (host arrays):
    returns (target (n,3), normal (n,3), weight (n,), pixel (n,))."""
    d = np.ascontiguousarray(depth, np.float32)
    p = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    q = np.ascontiguousarray(normals, np.float32).reshape(-1, 3)
    n = p.shape[0]
    t = np.empty((n, 3), np.float32)
    nn = np.empty((n, 3), np.float32)
    w = np.empty(n, np.float32)
    px = np.empty(n, np.int32)
    c, a = _camera(cam), _assoc(eps)
    s = _current_stream() if stream is None else stream
    _check(_lib.vd_associate(C.byref(c), d.ctypes.data, p.ctypes.data, q.ctypes.data, n,
                             C.byref(a), t.ctypes.data, nn.ctypes.data, w.ctypes.data,
                             px.ctypes.data, VD_MEM_HOST, C.c_void_p(s)), "vd_associate")
    return t, nn, w, px


def rigid_pose(cam, depth, points, normals, eps, iters: int, pose=None,
               stream: Optional[int] = None):
    """Rigid pose by projective ICP (host arrays): returns (pose (12,),
    history (iters, 2) of E and kept pairs)."""
    d = np.ascontiguousarray(depth, np.float32)
    p = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    q = np.ascontiguousarray(normals, np.float32).reshape(-1, 3)
    P = np.ascontiguousarray(
        np.concatenate([np.eye(3).ravel(), np.zeros(3)]) if pose is None else pose, np.float64)
    hist = np.zeros((max(iters, 1), 2), np.float64)
    c, a = _camera(cam), _assoc(eps)
    s = _current_stream() if stream is None else stream
    _check(_lib.vd_rigid_pose(C.byref(c), d.ctypes.data, p.ctypes.data, q.ctypes.data,
                              p.shape[0], C.byref(a), int(iters), P.ctypes.data,
                              hist.ctypes.data, VD_MEM_HOST, C.c_void_p(s)), "vd_rigid_pose")
    return P, hist[:iters]


def rigid_pose_noalloc(cam, depth, points, normals, eps, iters: int, pose, hist=None,
                       stream: Optional[int] = None) -> None:
    """vd_rigid_pose_noalloc: every array a contiguous CUDA tensor of the
    current GPU -- depth (H, W), points and normals (n, 3) float32; pose (12,)
    float64, updated in place; hist (2 * iters,) float64 or None.  Queued on
    the stream without waiting."""
    arrays = (depth, points, normals, pose) + (() if hist is None else (hist,))
    if not all(_is_device(a) and a.is_contiguous() for a in arrays):
        raise ValueError("vd_rigid_pose_noalloc takes contiguous device tensors only")
    if not all(a.dtype == torch.float32 for a in (depth, points, normals)) or \
            pose.dtype != torch.float64 or (hist is not None and hist.dtype != torch.float64):
        raise ValueError("depth, points, normals float32; pose and hist float64")
    if pose.numel() != 12 or (hist is not None and hist.numel() < 2 * iters):
        raise ValueError("pose needs 12 entries and hist 2 * iters")
    c, a = _camera(cam), _assoc(eps)
    s = _current_stream() if stream is None else stream
    _check(_lib.vd_rigid_pose_noalloc(C.byref(c), depth.data_ptr(), points.data_ptr(),
                                      normals.data_ptr(), points.shape[0], C.byref(a),
                                      int(iters), pose.data_ptr(),
                                      None if hist is None else hist.data_ptr(),
                                      C.c_void_p(s)), "vd_rigid_pose_noalloc")


def batch_precision(n: int) -> str:
    """Precision a batched lattice with n nodes per axis is given by the
    benchmark and the tests: float32 truncated CG (20 iterations) amplifies
    its rounding by about an order of magnitude per iteration once its Ritz
    values settle, and on lattices below 33 nodes per axis that leaves the
    final energy and positions outside 1e-4 / 1e-3 of the spacing of the
    float64 replica; those lattices are latency-bound, so float64 costs them
    no time."""
    return "fp64" if int(n) < 33 else "fp32"


def fit_rotations(M, R_prev=None, precision: str = "fp32", stream: Optional[int] = None):
    """Batched Procrustes fit (host arrays): returns (R (n,3,3), code (n,))."""
    M = np.ascontiguousarray(M, np.float32).reshape(-1, 9)
    n = M.shape[0]
    Rp = None if R_prev is None else np.ascontiguousarray(R_prev, np.float32).reshape(-1, 9)
    R = np.empty((n, 9), np.float32)
    code = np.empty(n, np.int32)
    s = _current_stream() if stream is None else stream
    _check(_lib.vd_debug_fit_rotations(M.ctypes.data, None if Rp is None else Rp.ctypes.data,
                                       R.ctypes.data, code.ctypes.data, n,
                                       VD_FP64 if precision == "fp64" else VD_FP32_FP64RED,
                                       VD_MEM_HOST, C.c_void_p(s)), "vd_debug_fit_rotations")
    return R.reshape(n, 3, 3), code


def sort_pairs(keys, vals, end_bit: int, stream: Optional[int] = None):
    """The library's stable radix sort by the low end_bit key bits (host
    arrays): returns (sorted keys, values in the same order)."""
    k = np.ascontiguousarray(keys, np.uint32).ravel()
    v = np.ascontiguousarray(vals, np.int32).ravel()
    if k.shape != v.shape:
        raise ValueError("keys and vals must have the same length")
    ko, vo = np.empty_like(k), np.empty_like(v)
    s = _current_stream() if stream is None else stream
    _check(_lib.vd_debug_sort_pairs(k.ctypes.data, v.ctypes.data, ko.ctypes.data, vo.ctypes.data,
                                    k.size, int(end_bit), VD_MEM_HOST, C.c_void_p(s)),
           "vd_debug_sort_pairs")
    return ko, vo


def exclusive_scan(values, stream: Optional[int] = None):
    """The library's exclusive prefix sum of int32 values (host arrays)."""
    x = np.ascontiguousarray(values, np.int32).ravel()
    out = np.empty_like(x)
    s = _current_stream() if stream is None else stream
    _check(_lib.vd_debug_exclusive_scan(x.ctypes.data, out.ctypes.data, x.size, VD_MEM_HOST,
                                        C.c_void_p(s)), "vd_debug_exclusive_scan")
    return out


def _bf16_ptr(x, n, what):
    """(pointer, mem, keepalive) of a bfloat16-bits array of n elements."""
    if _is_device(x):
        if x.dtype not in (torch.int16, torch.bfloat16) or not x.is_contiguous() or x.numel() != n:
            raise ValueError(f"{what}: contiguous int16/bfloat16 CUDA tensor of {n} elements")
        return x.data_ptr(), VD_MEM_DEVICE, x
    h = np.ascontiguousarray(x, dtype=np.uint16).reshape(-1)
    if h.size != n:
        raise ValueError(f"{what}: {n} elements expected, got {h.size}")
    return h.ctypes.data, VD_MEM_HOST, h


class Net:
    """The warm-start network (vd_net*) for nx*ny*nz grids, up to max_batch
    samples per call."""

    def __init__(self, dims, max_batch: int = 1, stream: Optional[int] = None):
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        s = _current_stream() if stream is None else stream
        _check(_lib.vd_net_create(self.dims[0], self.dims[1], self.dims[2], self.max_batch,
                                  C.c_void_p(s), C.byref(h)), "vd_net_create")
        self._h = h
        self.n = self.dims[0] * self.dims[1] * self.dims[2]

    @staticmethod
    def param_count() -> int:
        return int(_lib.vd_net_param_count())

    def close(self):
        if getattr(self, "_h", None):
            _lib.vd_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p) -> None:
        (ptr,), mem, keep = _prep([p])
        _check(_lib.vd_net_set_params(self._h, ptr, mem), "vd_net_set_params")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count(), np.float32)
        _check(_lib.vd_net_get_params(self._h, out.ctypes.data, VD_MEM_HOST), "vd_net_get_params")
        return out

    def forward(self, x, batch: int = 1, out=None):
        """x: [batch][nz][ny][nx][8] bfloat16 bits; returns [batch][3][N] float32
        (numpy, or `out` filled for device inputs)."""
        xp, mem, keep = _bf16_ptr(x, batch * self.n * 8, "x")
        if mem == VD_MEM_DEVICE:
            if out is None:
                out = torch.empty(batch * 3 * self.n, dtype=torch.float32, device=x.device)
            _check(_lib.vd_net_forward(self._h, xp, batch, out.data_ptr(), mem), "vd_net_forward")
            return out
        res = np.empty(batch * 3 * self.n, np.float32)
        _check(_lib.vd_net_forward(self._h, xp, batch, res.ctypes.data, mem), "vd_net_forward")
        return res.reshape(batch, 3, self.n)

    def gradients(self, x, target, batch: int = 1):
        """(loss, gradient) at the current parameters, host arrays."""
        xp, mem, keep = _bf16_ptr(x, batch * self.n * 8, "x")
        if mem != VD_MEM_HOST:
            raise ValueError("gradients() takes host arrays")
        t = np.ascontiguousarray(target, dtype=np.float32).reshape(-1)
        g = np.empty(self.param_count(), np.float32)
        loss = C.c_double()
        _check(_lib.vd_net_gradients(self._h, xp, t.ctypes.data, batch, g.ctypes.data,
                                     C.byref(loss), mem), "vd_net_gradients")
        return float(loss.value), g

    def train_step(self, x, target, batch: int = 1, lr: float = 1e-3, want_loss: bool = False):
        xp, mem, keep = _bf16_ptr(x, batch * self.n * 8, "x")
        if mem == VD_MEM_DEVICE:
            if not (_is_device(target) and target.dtype == torch.float32
                    and target.is_contiguous() and target.numel() == batch * 3 * self.n):
                raise ValueError("target: contiguous float32 CUDA tensor of batch*3*N")
            tp, tk = target.data_ptr(), target
        else:
            tk = np.ascontiguousarray(target, dtype=np.float32).reshape(-1)
            tp = tk.ctypes.data
        loss = C.c_double()
        _check(_lib.vd_net_train_step(self._h, xp, tp, batch, float(lr), mem,
                                      C.byref(loss) if want_loss else None),
               "vd_net_train_step")
        return float(loss.value) if want_loss else None
