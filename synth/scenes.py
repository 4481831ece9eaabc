"""Seeded scene generators for the lattice deformation solve.

Every generator takes a seed and returns a :class:`Scene`: float32 arrays in the
layout the C-ABI accepts (array-of-structs xyz triples) plus the lattice
description.  The recipes follow the workloads the solve is benchmarked on:

* ``make_config0`` -- a 16^3 unit-spaced lattice around a sphere of radius 6,
  2000 surface samples warped by 8 Gaussian RBF displacements (amplitude 0.8,
  width 4) plus N(0, 0.02) noise, 50 sparse point pairs, weights 1/10/5,
  5 GN x 10 PCG on one level.
* ``make_config1`` -- a 64^3 lattice (h = 15.625 mm) around a noisy torus,
  rendered into a 640x480 depth map (fx = fy = 525, cx = 320, cy = 240) under
  a 32-centre RBF warp (amplitude 2 voxels); one dense constraint per valid
  pixel (about 1e5), 500 sparse pairs, 3 levels x 8 GN x 20 PCG.
* ``make_tiny`` -- small random problems for exhaustive checks.

Only inputs are produced here.  The RBF warp W(x) = x + sum_k a_k
exp(-|x - c_k|^2 / (2 sigma^2)) is the *ground truth* that makes targets; it is
not the lattice deformation the solver fits.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Tuple

import numpy as np


@dataclass
class LatticeSpec:
    """Lattice description: finest node counts, spacing, origin, hierarchy and
    schedule (listed coarse -> fine), and the energy weights w_d, w_s, w_r."""

    dims: Tuple[int, int, int]
    spacing: float
    origin: Tuple[float, float, float]
    num_levels: int
    gn_iters: Tuple[int, ...]
    pcg_iters: Tuple[int, ...]
    w_dense: float = 1.0
    w_sparse: float = 10.0
    w_arap: float = 5.0


@dataclass
class Scene:
    spec: LatticeSpec
    canon: np.ndarray          # (C,3) float32, canonical surface samples p_hat
    target: np.ndarray         # (C,3) float32, observed points p^a
    normal: np.ndarray         # (C,3) float32, observed unit normals n^a
    weight: np.ndarray         # (C,)  float32, per-correspondence confidence w_c
    sparse_canon: np.ndarray   # (S,3) float32, canonical feature positions f_hat
    sparse_target: np.ndarray  # (S,3) float32, observed feature positions f
    meta: Dict = field(default_factory=dict)

    @property
    def n_dense(self) -> int:
        return int(self.canon.shape[0])

    @property
    def n_sparse(self) -> int:
        return int(self.sparse_canon.shape[0])


@dataclass
class DepthFrame:
    """One sensor frame and the model samples a projective association starts
    from: depth (H, W) float32 (0 = no measurement), pinhole intrinsics
    (width, height, fx, fy, cx, cy), canonical sample positions and normals
    (M, 3) float32."""

    depth: np.ndarray
    camera: Dict
    model_canon: np.ndarray
    model_normal: np.ndarray


# ---------------------------------------------------------------------------
# ground-truth warp used to make targets
# ---------------------------------------------------------------------------

def _random_directions(rng: np.random.Generator, k: int) -> np.ndarray:
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


class RBFWarp:
    """W(x) = x + sum_k a_k exp(-|x-c_k|^2 / (2 sigma^2)) and its Jacobian."""

    def __init__(self, centres: np.ndarray, amps: np.ndarray, sigma: float):
        self.c = np.asarray(centres, np.float64)
        self.a = np.asarray(amps, np.float64)
        self.sigma = float(sigma)

    def _phi(self, x: np.ndarray) -> np.ndarray:
        d2 = ((x * x).sum(1)[:, None] - 2.0 * (x @ self.c.T)
              + (self.c * self.c).sum(1)[None, :])
        return np.exp(-np.maximum(d2, 0.0) / (2.0 * self.sigma ** 2))

    def apply(self, x: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
        x = np.asarray(x, np.float64)
        out = np.empty_like(x)
        for s in range(0, x.shape[0], chunk):
            xs = x[s:s + chunk]
            out[s:s + chunk] = xs + self._phi(xs) @ self.a
        return out

    def jacobian(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, np.float64)
        phi = self._phi(x)                                   # (n,K)
        diff = x[:, None, :] - self.c[None, :, :]            # (n,K,3)
        grad_phi = -phi[:, :, None] * diff / self.sigma ** 2  # (n,K,3)
        jac = np.einsum("ka,nkb->nab", self.a, grad_phi)
        jac += np.eye(3)[None]
        return jac

    def transform_normals(self, x: np.ndarray, n: np.ndarray) -> np.ndarray:
        jac = self.jacobian(x)
        m = np.linalg.inv(jac).transpose(0, 2, 1)
        out = np.einsum("nab,nb->na", m, n)
        return out / np.linalg.norm(out, axis=1, keepdims=True)


def _uniform_sphere(rng, k, centre, radius):
    u = _random_directions(rng, k)
    return np.asarray(centre)[None, :] + radius * u, u


# ---------------------------------------------------------------------------
# configuration 0: 16^3 sphere
# ---------------------------------------------------------------------------

def make_config0(seed: int = 0) -> Scene:
    rng = np.random.default_rng(seed)
    n = 16
    spec = LatticeSpec(dims=(n, n, n), spacing=1.0, origin=(0.0, 0.0, 0.0),
                       num_levels=1, gn_iters=(5,), pcg_iters=(10,),
                       w_dense=1.0, w_sparse=10.0, w_arap=5.0)
    centre = np.array([7.5, 7.5, 7.5])
    radius = 6.0
    canon, nhat = _uniform_sphere(rng, 2000, centre, radius)
    centres = rng.uniform(1.5, 13.5, size=(8, 3))
    amps = 0.8 * _random_directions(rng, 8)
    warp = RBFWarp(centres, amps, sigma=4.0)
    target = warp.apply(canon) + rng.normal(scale=0.02, size=canon.shape)
    normal = warp.transform_normals(canon, nhat)
    sp_canon, _ = _uniform_sphere(rng, 50, centre, radius)
    sp_target = warp.apply(sp_canon) + rng.normal(scale=0.02, size=sp_canon.shape)
    return Scene(spec=spec,
                 canon=canon.astype(np.float32), target=target.astype(np.float32),
                 normal=normal.astype(np.float32),
                 weight=np.ones(canon.shape[0], np.float32),
                 sparse_canon=sp_canon.astype(np.float32),
                 sparse_target=sp_target.astype(np.float32),
                 meta={"config": 0, "seed": seed, "rbf_centres": centres,
                       "rbf_amps": amps, "rbf_sigma": 4.0})


# ---------------------------------------------------------------------------
# configuration 1: 64^3 torus rendered to a 640x480 depth map
# ---------------------------------------------------------------------------

CAM = dict(width=640, height=480, fx=525.0, fy=525.0, cx=320.0, cy=240.0)

# Geometry constants chosen so that a seed gives roughly 1e5 valid pixels.
CFG1_H = 0.015625           # 15.625 mm node spacing, 64 nodes ~ 1 m
CFG1_DEPTH = 0.95           # camera distance of the torus centre (m)
CFG1_MAJOR = 0.26           # torus major radius (m)
CFG1_MINOR = 0.10           # torus minor radius (m)
CFG1_TILT_DEG = 30.0        # tilt of the torus axis away from the view axis


def _torus_points(rng, n_theta, n_phi, major, minor, noise_amp, with_normals=False):
    """Canonical torus points (local frame, axis = z) with a smooth random
    perturbation of the tube radius (low-frequency signed-distance noise).
    With ``with_normals`` also the outward unit normals of that surface
    (cross product of its parameter derivatives), drawn from the same rng
    state, so the points are the same either way."""
    th = (np.arange(n_theta) + rng.uniform()) * (2 * np.pi / n_theta)
    ph = (np.arange(n_phi) + rng.uniform()) * (2 * np.pi / n_phi)
    T, P = np.meshgrid(th, ph, indexing="ij")
    T = T.ravel()
    P = P.ravel()
    terms = []
    freqs = [(1, 1), (2, 1), (3, 2), (1, 2), (2, 3)]
    for (m, k) in freqs:
        terms.append((rng.normal(), m, k, rng.uniform(0, 2 * np.pi)))

    def surface(T, P):
        eta = np.zeros_like(T)
        for (a, m, k, ph0) in terms:
            eta += a * np.sin(m * T + k * P + ph0)
        return eta

    eta = surface(T, P)
    scale = noise_amp / max(np.abs(eta).max(), 1e-12)

    def embed(T, P):
        rr = minor + scale * surface(T, P)
        return np.stack([(major + rr * np.cos(P)) * np.cos(T),
                         (major + rr * np.cos(P)) * np.sin(T), rr * np.sin(P)], axis=1)

    pts = embed(T, P)
    if not with_normals:
        return pts
    d = 1e-5
    dT = embed(T + d, P) - embed(T - d, P)
    dP = embed(T, P + d) - embed(T, P - d)
    nrm = np.cross(dT, dP)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ring = np.stack([major * np.cos(T), major * np.sin(T), np.zeros_like(T)], axis=1)
    out = np.einsum("na,na->n", nrm, pts - ring) < 0
    nrm[out] = -nrm[out]
    return pts, nrm


def _rot_x(deg):
    a = np.deg2rad(deg)
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], np.float64)


def _render(points_world, cam, noise_sigma, rng):
    """Point-splat z-buffer: nearest warped point per pixel wins.

    Returns (clean depth, noisy depth, winner index) images; winner = -1 where
    no point landed."""
    W, H = cam["width"], cam["height"]
    X, Y, Z = points_world[:, 0], points_world[:, 1], points_world[:, 2]
    ok = Z > 1e-3
    u = np.floor(cam["fx"] * X / np.where(ok, Z, 1) + cam["cx"]).astype(np.int64)
    v = np.floor(cam["fy"] * Y / np.where(ok, Z, 1) + cam["cy"]).astype(np.int64)
    ok &= (u >= 0) & (u < W) & (v >= 0) & (v < H)
    idx = np.nonzero(ok)[0]
    pix = v[idx] * W + u[idx]
    order = np.lexsort((Z[idx], pix))
    pix_sorted = pix[order]
    first = np.ones(order.size, bool)
    first[1:] = pix_sorted[1:] != pix_sorted[:-1]
    win = idx[order[first]]
    winpix = pix_sorted[first]
    winner = -np.ones(W * H, np.int64)
    winner[winpix] = win
    clean = np.zeros(W * H, np.float64)
    clean[winpix] = Z[win]
    noisy = clean.copy()
    noisy[winpix] += rng.normal(scale=noise_sigma, size=winpix.size)
    return clean.reshape(H, W), noisy.reshape(H, W), winner.reshape(H, W)


def _backproject(depth, cam):
    H, W = depth.shape
    uu, vv = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    x = (uu - cam["cx"]) / cam["fx"] * depth
    y = (vv - cam["cy"]) / cam["fy"] * depth
    return np.stack([x, y, depth], axis=-1)


def _depth_normals(depth, cam, max_jump=0.02, min_cos=0.2):
    """Normals from central differences of the back-projected depth map,
    oriented toward the camera; invalid where a neighbour is missing, across
    depth jumps, or at grazing angles."""
    P = _backproject(depth, cam)
    valid = depth > 0
    H, W = depth.shape
    nrm = np.zeros_like(P)
    ok = np.zeros((H, W), bool)
    c = (slice(1, H - 1), slice(1, W - 1))
    dx = P[1:-1, 2:] - P[1:-1, :-2]
    dy = P[2:, 1:-1] - P[:-2, 1:-1]
    n = np.cross(dx, dy)
    ln = np.linalg.norm(n, axis=-1)
    nb = (valid[1:-1, 2:] & valid[1:-1, :-2] & valid[2:, 1:-1] & valid[:-2, 1:-1]
          & valid[c])
    d0 = depth[c]
    jump = np.maximum.reduce([np.abs(depth[1:-1, 2:] - d0), np.abs(depth[1:-1, :-2] - d0),
                              np.abs(depth[2:, 1:-1] - d0), np.abs(depth[:-2, 1:-1] - d0)])
    good = nb & (jump < max_jump) & (ln > 0)
    n = n / np.where(ln > 0, ln, 1)[..., None]
    pn = np.linalg.norm(P[c], axis=-1, keepdims=True)
    view = -P[c] / np.where(pn > 0, pn, 1.0)
    cosv = (n * view).sum(-1)
    n = np.where((cosv < 0)[..., None], -n, n)
    good &= np.abs(cosv) > min_cos
    nrm[c] = n
    ok[c] = good
    return nrm, ok


def make_config1(seed: int = 0, n: int = 64, num_levels: int = 3,
                 gn: int = 8, pcg: int = 20, n_sparse: int = 500,
                 n_theta: int = 2400, n_phi: int = 900,
                 rbf_centres_override=None, depth_frame: bool = False):
    """The 64^3 workload.  With ``depth_frame`` also returns a
    :class:`DepthFrame` of the same frame: the noisy depth map the dense
    constraints were read from and the model samples a projective
    association starts from (the canonical surface points that are visible
    when the undeformed surface is rendered with the same camera, with their
    outward normals)."""
    rng = np.random.default_rng(seed)
    h = CFG1_H * 64.0 / n
    coarse_span = (2 ** (num_levels - 1)) * h * (int(np.ceil(n / 2 ** (num_levels - 1))) - 1)
    centre = np.array([0.0, 0.0, CFG1_DEPTH])
    origin = centre - 0.5 * coarse_span
    spec = LatticeSpec(dims=(n, n, n), spacing=h, origin=tuple(origin.tolist()),
                       num_levels=num_levels, gn_iters=(gn,) * num_levels,
                       pcg_iters=(pcg,) * num_levels,
                       w_dense=1.0, w_sparse=10.0, w_arap=5.0)
    local, local_n = _torus_points(rng, n_theta, n_phi, CFG1_MAJOR, CFG1_MINOR, 0.5 * CFG1_H,
                                   with_normals=True)
    canon = local @ _rot_x(CFG1_TILT_DEG).T + centre[None, :]
    ext = CFG1_MAJOR + CFG1_MINOR
    if rbf_centres_override is None:
        centres = centre[None, :] + rng.uniform(-ext, ext, size=(32, 3))
    else:
        centres = np.asarray(rbf_centres_override, np.float64)
    amps = 2.0 * CFG1_H * _random_directions(rng, centres.shape[0])
    warp = RBFWarp(centres, amps, sigma=16.0 * CFG1_H)
    warped = warp.apply(canon)
    clean, noisy, winner = _render(warped, CAM, 1e-3, rng)
    nrm, ok = _depth_normals(clean, CAM)
    ok &= noisy > 0
    vv, uu = np.nonzero(ok)
    P = _backproject(noisy, CAM)
    target = P[vv, uu]
    normal = nrm[vv, uu]
    win = winner[vv, uu]
    p_hat = canon[win]
    # sparse pairs: distinct visible canonical points, targets from the warp
    pick = rng.choice(win.size, size=min(n_sparse, win.size), replace=False)
    sp_canon = p_hat[pick]
    sp_target = warp.apply(sp_canon) + rng.normal(scale=1e-3, size=sp_canon.shape)
    scene = Scene(spec=spec,
                  canon=p_hat.astype(np.float32), target=target.astype(np.float32),
                  normal=normal.astype(np.float32),
                  weight=np.ones(p_hat.shape[0], np.float32),
                  sparse_canon=sp_canon.astype(np.float32),
                  sparse_target=sp_target.astype(np.float32),
                  meta={"config": 1, "seed": seed, "valid_pixels": int(p_hat.shape[0]),
                        "rbf_centres": centres, "rbf_amps": amps,
                        "rbf_sigma": 16.0 * CFG1_H, "camera": CAM})
    if not depth_frame:
        return scene
    canon_n = local_n @ _rot_x(CFG1_TILT_DEG).T
    # model samples: the undeformed surface rendered with the same camera
    # (drawn after every other random number, so the scene is unchanged)
    _, _, win0 = _render(canon, CAM, 0.0, rng)
    vis = win0[win0 >= 0]
    frame = DepthFrame(depth=noisy.astype(np.float32), camera=dict(CAM),
                       model_canon=canon[vis].astype(np.float32),
                       model_normal=canon_n[vis].astype(np.float32))
    return scene, frame


# ---------------------------------------------------------------------------
# small random problems
# ---------------------------------------------------------------------------

def make_tiny(seed: int = 0, dims=(4, 4, 4), spacing: float = 1.0,
              origin=(0.0, 0.0, 0.0), n_dense: int = 40, n_sparse: int = 6,
              num_levels: int = 1, gn: int = 3, pcg: int = 8,
              amp: float = 0.3, weights=(1.0, 10.0, 5.0)) -> Scene:
    """Random samples inside the lattice, targets displaced by up to ``amp``
    (in units of the spacing), random unit normals and weights in [0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(d) for d in dims)
    o = np.asarray(origin, np.float64)
    # keep samples inside the coarsest level's extent
    nc = np.asarray(dims)
    for _ in range(num_levels - 1):
        nc = (nc + 1) // 2
    span = (nc - 1) * spacing * (2 ** (num_levels - 1))
    canon = o + rng.uniform(0.0, 1.0, size=(n_dense, 3)) * span
    target = canon + amp * spacing * rng.normal(size=canon.shape)
    normal = _random_directions(rng, n_dense)
    weight = rng.uniform(0.5, 1.5, size=n_dense)
    sp_canon = o + rng.uniform(0.0, 1.0, size=(n_sparse, 3)) * span
    sp_target = sp_canon + amp * spacing * rng.normal(size=sp_canon.shape)
    spec = LatticeSpec(dims=dims, spacing=spacing, origin=tuple(o.tolist()),
                       num_levels=num_levels, gn_iters=(gn,) * num_levels,
                       pcg_iters=(pcg,) * num_levels,
                       w_dense=weights[0], w_sparse=weights[1], w_arap=weights[2])
    return Scene(spec=spec, canon=canon.astype(np.float32),
                 target=target.astype(np.float32), normal=normal.astype(np.float32),
                 weight=weight.astype(np.float32),
                 sparse_canon=sp_canon.astype(np.float32),
                 sparse_target=sp_target.astype(np.float32),
                 meta={"config": "tiny", "seed": seed})


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def make_rigid_scene(base: Scene, Q: np.ndarray, c: np.ndarray) -> Scene:
    """Targets and normals moved by the rigid map x -> Q x + c, without noise:
    the lattice state t_i = Q t_hat_i + c, R_i = Q explains them exactly."""
    Q = np.asarray(Q, np.float64)
    c = np.asarray(c, np.float64)
    canon = base.canon.astype(np.float64)
    sp = base.sparse_canon.astype(np.float64)
    return Scene(spec=base.spec, canon=base.canon,
                 target=(canon @ Q.T + c).astype(np.float32),
                 normal=(base.normal.astype(np.float64) @ Q.T).astype(np.float32),
                 weight=base.weight, sparse_canon=base.sparse_canon,
                 sparse_target=(sp @ Q.T + c).astype(np.float32),
                 meta=dict(base.meta, rigid=True))


def make_identity_scene(base: Scene) -> Scene:
    """Targets equal to the canonical samples: the rest state is optimal."""
    return Scene(spec=base.spec, canon=base.canon, target=base.canon.copy(),
                 normal=base.normal, weight=base.weight,
                 sparse_canon=base.sparse_canon,
                 sparse_target=base.sparse_canon.copy(),
                 meta=dict(base.meta, identity=True))


def make_sequence_frame(seed: int, frame: int, n: int = 64, num_levels: int = 3,
                        gn: int = 8, pcg: int = 20, speed_voxels: float = 0.3,
                        n_sparse: int = 500) -> Scene:
    """Frame ``frame`` of a deforming sequence: the config-1 torus whose RBF
    centres move ``speed_voxels`` node spacings per frame along fixed random
    directions (the same canonical surface for every frame of a seed)."""
    rng = np.random.default_rng(10_000 + seed)
    ext = CFG1_MAJOR + CFG1_MINOR
    centre = np.array([0.0, 0.0, CFG1_DEPTH])
    c0 = centre[None, :] + rng.uniform(-ext, ext, size=(32, 3))
    dirs = _random_directions(rng, 32)
    h = CFG1_H * 64.0 / n
    centres = c0 + frame * speed_voxels * h * dirs
    return make_config1(seed=seed, n=n, num_levels=num_levels, gn=gn, pcg=pcg,
                        n_sparse=n_sparse, rbf_centres_override=centres)


# ---------------------------------------------------------------------------
# configuration 2: a batch of uneven lattices, each with its own 320x240 frame
# ---------------------------------------------------------------------------

CAM2 = dict(width=320, height=240, fx=262.5, fy=262.5, cx=160.0, cy=120.0)


def _sphere_points(rng, n_pts, radius, noise_amp):
    """Fibonacci-sphere points with a smooth random radial perturbation."""
    k = np.arange(n_pts) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / n_pts)
    th = np.pi * (1.0 + 5.0 ** 0.5) * k
    u = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)
    eta = np.zeros(n_pts)
    for _ in range(5):
        a = _random_directions(rng, 1)[0]
        eta += rng.normal() * np.sin(3.0 * (u @ a) + rng.uniform(0, 2 * np.pi))
    eta *= noise_amp / max(np.abs(eta).max(), 1e-12)
    return (radius + eta)[:, None] * u


def make_batch_lattice(seed: int, n: int, target_valid: int, n_sparse: int,
                       num_levels: int = 3, gn: int = 8, pcg: int = 20) -> Scene:
    """One member of the batched workload: an n^3 lattice around a noisy torus
    or sphere rendered into a 320x240 depth map (fx = fy = 262.5) with about
    ``target_valid`` valid pixels, warped by 16 RBFs (amplitude 1.5 node
    spacings, width n/4 spacings), depth noise 0.05 spacings."""
    rng = np.random.default_rng(seed)
    torus = rng.uniform() < 0.5
    if torus:
        major = rng.uniform(0.2, 0.3)
        minor = rng.uniform(0.3, 0.45) * major
        ext = major + minor
        area = 4.0 * np.pi * major * minor * np.cos(np.deg2rad(30.0))
    else:
        ext = rng.uniform(0.2, 0.35)
        area = np.pi * ext ** 2
    nc = n
    for _ in range(num_levels - 1):
        nc = (nc + 1) // 2
    span = 2.0 * 1.12 * ext
    h = span / ((nc - 1) * 2 ** (num_levels - 1))
    depth = CAM2["fx"] * np.sqrt(area / target_valid)
    centre = np.array([0.0, 0.0, depth])
    origin = centre - 0.5 * span
    spec = LatticeSpec(dims=(n, n, n), spacing=h, origin=tuple(origin.tolist()),
                       num_levels=num_levels, gn_iters=(gn,) * num_levels,
                       pcg_iters=(pcg,) * num_levels)
    if torus:
        local = _torus_points(rng, 1200, 500, major, minor, 0.5 * h)
        local = local @ _rot_x(30.0).T
    else:
        local = _sphere_points(rng, 600_000, ext, 0.5 * h)
    centres = centre[None, :] + rng.uniform(-ext, ext, size=(16, 3))
    amps = 1.5 * h * _random_directions(rng, 16)
    warp = RBFWarp(centres, amps, sigma=0.25 * n * h)
    for attempt in range(2):
        canon = local + centre[None, :]
        warped = warp.apply(canon)
        clean, noisy, winner = _render(warped, CAM2, 0.05 * h, rng)
        nrm, ok = _depth_normals(clean, CAM2, max_jump=4.0 * h)
        ok &= noisy > 0
        count = int(ok.sum())
        if attempt == 0 and count > 0:
            # move the camera so that the valid-pixel count nears the target
            scale = np.sqrt(count / target_valid)
            shift = depth * (scale - 1.0)
            centre = centre + np.array([0.0, 0.0, shift])
            origin = origin + np.array([0.0, 0.0, shift])
            centres = centres + np.array([0.0, 0.0, shift])
            depth += shift
            warp = RBFWarp(centres, amps, sigma=0.25 * n * h)
            spec.origin = tuple(origin.tolist())
    vv, uu = np.nonzero(ok)
    P = _backproject(noisy, CAM2)
    target = P[vv, uu]
    normal = nrm[vv, uu]
    p_hat = canon[winner[vv, uu]]
    pick = rng.choice(p_hat.shape[0], size=min(n_sparse, p_hat.shape[0]), replace=False)
    sp_canon = p_hat[pick]
    sp_target = warp.apply(sp_canon) + rng.normal(scale=0.05 * h, size=sp_canon.shape)
    return Scene(spec=spec, canon=p_hat.astype(np.float32), target=target.astype(np.float32),
                 normal=normal.astype(np.float32),
                 weight=np.ones(p_hat.shape[0], np.float32),
                 sparse_canon=sp_canon.astype(np.float32),
                 sparse_target=sp_target.astype(np.float32),
                 meta={"config": 2, "seed": seed, "shape": "torus" if torus else "sphere",
                       "valid_pixels": int(p_hat.shape[0]), "target_valid": target_valid})


def make_config2(seed: int = 0, count: int = 32, n_range=(24, 64), valid_range=(5000, 60000),
                 sparse_range=(100, 400)):
    """The batched workload: ``count`` lattices with node counts per axis drawn
    uniformly from ``n_range``, each with its own seeded surface and frame."""
    ns, valid, sparse = config2_sizes(seed, count, n_range, valid_range, sparse_range)
    return [make_batch_lattice(1000 * seed + k, int(ns[k]), int(valid[k]), int(sparse[k]))
            for k in range(count)]


def config2_sizes(seed: int = 0, count: int = 32, n_range=(24, 64), valid_range=(5000, 60000),
                  sparse_range=(100, 400)):
    """Node counts per axis, valid-pixel targets and sparse-pair counts of the
    batched workload's lattices (the draws ``make_config2`` uses)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    valid = rng.integers(valid_range[0], valid_range[1] + 1, size=count)
    sparse = rng.integers(sparse_range[0], sparse_range[1] + 1, size=count)
    return ns, valid, sparse


def make_config2_member(seed: int, k: int, count: int = 32) -> Scene:
    """Lattice k of ``make_config2(seed, count)`` alone (the same scene)."""
    ns, valid, sparse = config2_sizes(seed, count)
    return make_batch_lattice(1000 * seed + k, int(ns[k]), int(valid[k]), int(sparse[k]))


# ---------------------------------------------------------------------------
# planar scenes with exact depth maps (association and rigid-pose checks)
# ---------------------------------------------------------------------------

def render_planes(cam: Dict, planes, dtype=np.float32) -> np.ndarray:
    """Depth map of the inside of a convex region {x : m_k . x >= b_k} seen
    from the camera at the origin (which must lie inside, b_k <= 0): each
    pixel-centre ray (u + 1/2 - cx)/fx, (v + 1/2 - cy)/fy, 1) leaves the
    region through the first plane it reaches; that distance along z is the
    depth.  planes: list of (unit normal m (3,), offset b)."""
    W, H = cam["width"], cam["height"]
    uu, vv = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    d = np.stack([(uu - cam["cx"]) / cam["fx"], (vv - cam["cy"]) / cam["fy"],
                  np.ones_like(uu)], axis=-1)
    depth = np.full((H, W), np.inf)
    for m, b in planes:
        md = d @ np.asarray(m, np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(md < 0, b / md, np.inf)
        depth = np.minimum(depth, s)
    depth[~np.isfinite(depth)] = 0.0
    return depth.astype(dtype)


BOX_PLANES = (  # inside corner of a box, in front of the camera (metres)
    (np.array([1.0, 0.0, 0.0]), -0.35),    # wall  x >= -0.35
    (np.array([0.0, -1.0, 0.0]), -0.25),   # floor y <= 0.25
    (np.array([0.0, 0.0, -1.0]), -1.10),   # back  z <= 1.10
    (np.array([-1.0, 0.0, 0.0]), -0.60),   # wall  x <= 0.60 (keeps rays bounded)
)


def moved_planes(planes, Q: np.ndarray, c: np.ndarray):
    """The planes after the rigid motion x -> Q x + c."""
    out = []
    for m, b in planes:
        mq = np.asarray(Q, np.float64) @ m
        out.append((mq, b + mq @ np.asarray(c, np.float64)))
    return out


def make_box_frame(Q=None, c=None, cam: Dict = CAM, step: int = 3, margin: int = 4,
                   noise: float = 0.0, seed: int = 0) -> DepthFrame:
    """Depth map of the box corner after the rigid motion (Q, c), with model
    samples taken from the unmoved corner: pixel-centre points of its exact
    depth map on a ``step``-pixel grid, at least ``margin`` pixels from any
    crease or image border, with the plane normals facing the camera."""
    Q = np.eye(3) if Q is None else np.asarray(Q, np.float64)
    c = np.zeros(3) if c is None else np.asarray(c, np.float64)
    rng = np.random.default_rng(seed)
    depth = render_planes(cam, moved_planes(BOX_PLANES, Q, c)).astype(np.float64)
    if noise > 0:
        depth = np.where(depth > 0, depth + rng.normal(scale=noise, size=depth.shape), 0.0)
    rest = render_planes(cam, BOX_PLANES).astype(np.float64)
    W, H = cam["width"], cam["height"]
    uu, vv = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    d = np.stack([(uu - cam["cx"]) / cam["fx"], (vv - cam["cy"]) / cam["fy"],
                  np.ones_like(uu)], axis=-1)
    # which plane each pixel sees, and whether its neighbourhood sees the same
    label = np.full((H, W), -1)
    best = np.full((H, W), np.inf)
    for k, (m, b) in enumerate(BOX_PLANES):
        md = d @ m
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(md < 0, b / md, np.inf)
        upd = s < best
        best[upd] = s[upd]
        label[upd] = k
    ok = np.zeros((H, W), bool)
    ok[margin:H - margin:step, margin:W - margin:step] = True
    for dy in range(-margin, margin + 1):
        for dx in range(-margin, margin + 1):
            ok &= np.roll(np.roll(label, dy, 0), dx, 1) == label
    vv_i, uu_i = np.nonzero(ok)
    pts = d[vv_i, uu_i] * rest[vv_i, uu_i][:, None]
    # the inward normals m_k of the region's faces point toward the camera
    nrm = np.stack([BOX_PLANES[k][0] for k in label[vv_i, uu_i]])
    return DepthFrame(depth=depth.astype(np.float32), camera=dict(cam),
                      model_canon=pts.astype(np.float32), model_normal=nrm.astype(np.float32))


def make_patch(seed: int = 0, dims=(12, 12, 12), spacing: float = 1.0, n_dense: int = 600,
               n_sparse: int = 12, num_levels: int = 1, gn: int = 3, pcg: int = 10,
               amp: float = 0.4, extent: float = 0.6, weights=(1.0, 10.0, 5.0)) -> Scene:
    """A surface patch inside the lattice: samples on a disc of the tilted
    plane through the lattice centre (radius ``extent`` of the half-span), so
    that only the cells near the plane hold samples; targets pushed along the
    plane normal by a smooth bump of amplitude ``amp`` spacings plus noise,
    normals the plane normal; sparse pairs on the same disc."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(d) for d in dims)
    nc = np.asarray(dims)
    for _ in range(num_levels - 1):
        nc = (nc + 1) // 2
    span = (nc - 1) * spacing * (2 ** (num_levels - 1))
    centre = 0.5 * span
    m = np.array([0.3, -0.2, 1.0])
    m /= np.linalg.norm(m)
    u = np.cross(m, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(m, u)
    rad = extent * 0.5 * float(span.min())

    def disc(k):
        r = rad * np.sqrt(rng.uniform(size=k))
        th = rng.uniform(0.0, 2 * np.pi, size=k)
        return centre + (r * np.cos(th))[:, None] * u + (r * np.sin(th))[:, None] * v

    canon = disc(n_dense)
    s = (canon - centre) @ u / rad
    bump = amp * spacing * np.exp(-4.0 * s * s)
    target = canon + bump[:, None] * m + 0.02 * spacing * rng.normal(size=canon.shape)
    normal = np.broadcast_to(m, canon.shape)
    sp_canon = disc(n_sparse)
    s2 = (sp_canon - centre) @ u / rad
    sp_target = sp_canon + (amp * spacing * np.exp(-4.0 * s2 * s2))[:, None] * m
    spec = LatticeSpec(dims=dims, spacing=spacing, origin=(0.0, 0.0, 0.0),
                       num_levels=num_levels, gn_iters=(gn,) * num_levels,
                       pcg_iters=(pcg,) * num_levels,
                       w_dense=weights[0], w_sparse=weights[1], w_arap=weights[2])
    return Scene(spec=spec, canon=canon.astype(np.float32), target=target.astype(np.float32),
                 normal=normal.astype(np.float32),
                 weight=np.ones(n_dense, np.float32), sparse_canon=sp_canon.astype(np.float32),
                 sparse_target=sp_target.astype(np.float32),
                 meta={"config": "patch", "seed": seed})
