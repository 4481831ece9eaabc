"""Projective depth association (Sec. 5.1) and the global rigid pose by dense
projective ICP (Sec. 4, Sec. 6).

Part of the FP64 CPU oracle -- test infrastructure only.

Camera model (pinhole, the sensor's intrinsics fx, fy, cx, cy; the camera
sits at the origin looking along +z).  Pixel (u, v) covers [u, u+1) x [v, v+1)
in image coordinates, so a point (x, y, z) with z > 0 falls on pixel
(floor(fx x / z + cx), floor(fy y / z + cy)) and the depth D(u, v) of a pixel
back-projects at its centre to ((u + 1/2 - cx) D / fx, (v + 1/2 - cy) D / fy, D).
A depth <= 0 marks a pixel without a measurement.

Association of one model sample p_c with normal n_c (Sec. 5.1): project p_c
into the depth map and read the measurement p_c^a of the pixel it falls on,
with the normal n_c^a of the measured surface there.  Three kernels
Phi_r(x) = 1 - x / eps_r measure
  * the distance          Phi_d(|p_c - p_c^a|),
  * the normal deviation  Phi_n(1 - n_c . n_c^a),
  * the view angle        Phi_v(1 - n_c . v_c);
if any of them is negative the pair is pruned (w_c = 0), otherwise
w_c = ((Phi_d + Phi_n + Phi_v) / 3)^2.

Readings where the paper is silent:
  * A1 the measured normal n^a at pixel (u, v) is the normalised cross product
    (P(u+1, v) - P(u-1, v)) x (P(u, v+1) - P(u, v-1)) of back-projected
    neighbours, turned to face the camera (n . P(u, v) <= 0).  It exists only
    for pixels with all four neighbours inside the image, all five depths > 0
    and a non-zero cross product.
  * A2 v_c is the unit vector from p_c toward the camera centre, -p_c / |p_c|
    (n_c . v_c = 1 for a surface facing the camera, 0 at a silhouette).
  * A3 a sample with z <= 0, a pixel outside the image, no depth or no
    normal gets w_c = 0; pruned samples report target = normal = 0.
  * A4 the model normal of a lattice sample is the canonical normal rotated
    by the trilinearly interpolated rotation field, renormalised:
    n_c = normalise(sum_i alpha_i(p_hat_c) R_i n_hat_c).
  * A5 decisions (the pixel, pruning) are taken in float64 from the float32
    inputs, in the operation order written here.

Global pose (Sec. 4: S(x) = R [sum_i alpha_i t_i] + t; Sec. 6: it is found
by dense projective ICP first).  One ICP iteration at pose (R, t): transform
the model samples q_c = R p_c + t (normals R n_c), associate them as above,
and take the Gauss-Newton step of the point-to-plane energy
  E(R, t) = sum_c w_c (n_c^a . (q_c - p_c^a))^2
with weights and targets held fixed, linearised in a small rotation w and
translation tau applied after the current pose, q -> q + w x q + tau:
  r_c = n^a . (q_c - p^a),   J_c = [q_c x n^a, n^a],   (sum w J J^T) xi = -sum w J r.
The update is R <- Rot(w) R, t <- Rot(w) t + tau with Rot(w) the rotation by
|w| about w / |w| (Rodrigues).  Reading A6: when fewer than six pairs survive
or the 6x6 system is numerically singular -- rank below 6 at the tolerance
1e-8 times its largest diagonal entry -- the pose is left unchanged.  (A
single plane constrains 3 of the 6 unknowns; float32 depth quantisation tilts
its measured normals by about 1e-5, which leaves eigenvalues near 1e-11 of
the largest instead of 0, and a step along them would be driven by that
noise; three planes at large angles give about 1e-2.)
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclass(frozen=True)
class AssocParams:
    eps_d: float   # distance threshold (world units)
    eps_n: float   # normal deviation threshold (on 1 - cos)
    eps_v: float   # view-angle threshold (on 1 - cos)


def _dot(a, b):
    """a . b summed as x, then y, then z (the same order for one sample or many)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1] + a[..., 2] * b[..., 2]


def _cross(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def backproject(cam: Camera, depth: np.ndarray, u: int, v: int) -> np.ndarray:
    """Measurement of pixel (u, v) at its centre."""
    z = float(depth[v, u])
    return np.array([(u + 0.5 - cam.cx) * z / cam.fx, (v + 0.5 - cam.cy) * z / cam.fy, z])


def pixel_of(cam: Camera, x: np.ndarray):
    """Pixel (u, v) a point falls on, or None (z <= 0 or outside the image)."""
    x = np.asarray(x, np.float64)
    if not x[2] > 0.0:
        return None
    u = int(np.floor(cam.fx * x[0] / x[2] + cam.cx))
    v = int(np.floor(cam.fy * x[1] / x[2] + cam.cy))
    if u < 0 or u >= cam.width or v < 0 or v >= cam.height:
        return None
    return u, v


def measured_normal(cam: Camera, depth: np.ndarray, u: int, v: int):
    """Reading A1: normal of the measured surface at pixel (u, v), or None."""
    if u < 1 or u > cam.width - 2 or v < 1 or v > cam.height - 2:
        return None
    for (a, b) in ((u, v), (u + 1, v), (u - 1, v), (u, v + 1), (u, v - 1)):
        if not depth[b, a] > 0.0:
            return None
    dx = backproject(cam, depth, u + 1, v) - backproject(cam, depth, u - 1, v)
    dy = backproject(cam, depth, u, v + 1) - backproject(cam, depth, u, v - 1)
    n = _cross(dx, dy)
    ln = np.sqrt(_dot(n, n))
    if not ln > 0.0:
        return None
    n = n / ln
    if _dot(n, backproject(cam, depth, u, v)) > 0.0:
        n = -n
    return n


def kernel(x: float, eps: float) -> float:
    """Phi_r(x) = 1 - x / eps_r (Sec. 5.1)."""
    return 1.0 - x / eps


def associate_one(cam: Camera, depth: np.ndarray, p, n, prm: AssocParams):
    """(target p^a, normal n^a, w_c, pixel index v*W+u or -1) of one sample."""
    p = np.asarray(p, np.float64)
    n = np.asarray(n, np.float64)
    zero = np.zeros(3)
    pix = pixel_of(cam, p)
    if pix is None:
        return zero, zero, 0.0, -1
    u, v = pix
    idx = v * cam.width + u
    if not depth[v, u] > 0.0:
        return zero, zero, 0.0, idx
    na = measured_normal(cam, depth, u, v)
    if na is None:
        return zero, zero, 0.0, idx
    pa = backproject(cam, depth, u, v)
    ln = np.sqrt(_dot(n, n))
    if not ln > 0.0:
        return zero, zero, 0.0, idx
    nc = n / ln
    d = p - pa
    phi_d = kernel(np.sqrt(_dot(d, d)), prm.eps_d)
    phi_n = kernel(1.0 - _dot(nc, na), prm.eps_n)
    view = -p / np.sqrt(_dot(p, p))
    phi_v = kernel(1.0 - _dot(nc, view), prm.eps_v)
    if phi_d < 0.0 or phi_n < 0.0 or phi_v < 0.0:
        return zero, zero, 0.0, idx
    w = ((phi_d + phi_n + phi_v) / 3.0) ** 2
    return pa, na, w, idx


def associate_loop(cam: Camera, depth: np.ndarray, points: np.ndarray, normals: np.ndarray,
                   prm: AssocParams):
    """``associate`` one sample at a time (for small inputs)."""
    depth = np.asarray(depth, np.float64)
    points = np.asarray(points, np.float64).reshape(-1, 3)
    normals = np.asarray(normals, np.float64).reshape(-1, 3)
    C = points.shape[0]
    tg = np.zeros((C, 3))
    nm = np.zeros((C, 3))
    w = np.zeros(C)
    px = np.full(C, -1, np.int64)
    for c in range(C):
        tg[c], nm[c], w[c], px[c] = associate_one(cam, depth, points[c], normals[c], prm)
    return tg, nm, w, px


def _bp(cam: Camera, depth: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    z = depth[v, u]
    return np.stack([(u + 0.5 - cam.cx) * z / cam.fx, (v + 0.5 - cam.cy) * z / cam.fy, z], axis=1)


def associate(cam: Camera, depth: np.ndarray, points: np.ndarray, normals: np.ndarray,
              prm: AssocParams):
    """Every sample at once: (targets (C,3), normals (C,3), weights (C,),
    pixels (C,)); the same arithmetic as ``associate_one`` per sample."""
    depth = np.asarray(depth, np.float64)
    p = np.asarray(points, np.float64).reshape(-1, 3)
    n = np.asarray(normals, np.float64).reshape(-1, 3)
    C = p.shape[0]
    W, H = cam.width, cam.height
    tg = np.zeros((C, 3))
    nm = np.zeros((C, 3))
    w = np.zeros(C)
    px = np.full(C, -1, np.int64)
    front = p[:, 2] > 0.0
    z = np.where(front, p[:, 2], 1.0)
    uf = np.floor(cam.fx * p[:, 0] / z + cam.cx)
    vf = np.floor(cam.fy * p[:, 1] / z + cam.cy)
    inimg = front & (uf >= 0) & (uf < W) & (vf >= 0) & (vf < H)
    u = np.where(inimg, uf, 0).astype(np.int64)
    v = np.where(inimg, vf, 0).astype(np.int64)
    px[inimg] = v[inimg] * W + u[inimg]
    ok = inimg & (depth[v, u] > 0.0)
    ok &= (u >= 1) & (u <= W - 2) & (v >= 1) & (v <= H - 2)
    uc, vc = np.clip(u, 1, W - 2), np.clip(v, 1, H - 2)
    for (a, b) in ((uc + 1, vc), (uc - 1, vc), (uc, vc + 1), (uc, vc - 1)):
        ok &= depth[b, a] > 0.0
    dx = _bp(cam, depth, uc + 1, vc) - _bp(cam, depth, uc - 1, vc)
    dy = _bp(cam, depth, uc, vc + 1) - _bp(cam, depth, uc, vc - 1)
    na = _cross(dx, dy)
    ln = np.sqrt(_dot(na, na))
    ok &= ln > 0.0
    na = na / np.where(ln > 0.0, ln, 1.0)[:, None]
    pa = _bp(cam, depth, uc, vc)
    flip = _dot(na, pa) > 0.0
    na = np.where(flip[:, None], -na, na)
    lc = np.sqrt(_dot(n, n))
    ok &= lc > 0.0
    nc = n / np.where(lc > 0.0, lc, 1.0)[:, None]
    d = p - pa
    phi_d = kernel(np.sqrt(_dot(d, d)), prm.eps_d)
    phi_n = kernel(1.0 - _dot(nc, na), prm.eps_n)
    lp = np.sqrt(_dot(p, p))
    view = -p / np.where(lp > 0.0, lp, 1.0)[:, None]
    phi_v = kernel(1.0 - _dot(nc, view), prm.eps_v)
    ok &= (phi_d >= 0.0) & (phi_n >= 0.0) & (phi_v >= 0.0)
    tg[ok] = pa[ok]
    nm[ok] = na[ok]
    w[ok] = ((phi_d[ok] + phi_n[ok] + phi_v[ok]) / 3.0) ** 2
    return tg, nm, w, px


def rodrigues(w: np.ndarray) -> np.ndarray:
    """Rotation by the angle |w| about the axis w / |w|."""
    w = np.asarray(w, np.float64)
    th = np.sqrt(w @ w)
    if th == 0.0:
        return np.eye(3)
    k = w / th
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def transform(points: np.ndarray, normals: np.ndarray, R: np.ndarray, t: np.ndarray):
    """q = R p + t and R n, each component summed left to right as written
    (reading A5: the association decisions that follow depend on the bits)."""
    p = np.asarray(points, np.float64).reshape(-1, 3)
    n = np.asarray(normals, np.float64).reshape(-1, 3)
    q = np.empty_like(p)
    nq = np.empty_like(n)
    for r in range(3):
        q[:, r] = R[r, 0] * p[:, 0] + R[r, 1] * p[:, 1] + R[r, 2] * p[:, 2] + t[r]
        nq[:, r] = R[r, 0] * n[:, 0] + R[r, 1] * n[:, 1] + R[r, 2] * n[:, 2]
    return q, nq


def icp_step(cam: Camera, depth: np.ndarray, points: np.ndarray, normals: np.ndarray,
             prm: AssocParams, R: np.ndarray, t: np.ndarray):
    """One Gauss-Newton iteration of the projective point-to-plane ICP.
    Returns (R', t', E at (R, t), number of associated samples)."""
    q, nq = transform(np.asarray(points, np.float64), np.asarray(normals, np.float64), R, t)
    pa, na, w, _ = associate(cam, depth, q, nq, prm)
    keep = w > 0.0
    r = _dot(na, q - pa)
    E = float(np.sum(w * r * r))
    J = np.concatenate([_cross(q, na), na], axis=1)[keep]
    H = (J * w[keep, None]).T @ J
    g = (J * w[keep, None]).T @ r[keep]
    if int(keep.sum()) < 6 or np.linalg.matrix_rank(H, tol=1e-8 * np.max(np.diag(H))) < 6:
        return R.copy(), t.copy(), E, int(keep.sum())
    xi = -np.linalg.solve(H, g)
    Q = rodrigues(xi[:3])
    return Q @ R, Q @ t + xi[3:], E, int(keep.sum())


def rigid_pose(cam: Camera, depth: np.ndarray, points: np.ndarray, normals: np.ndarray,
               prm: AssocParams, iters: int, R0=None, t0=None):
    """`iters` ICP iterations from (R0, t0) (default identity).  Returns the
    final (R, t) and the per-iteration list of (E, associated count) measured
    at the pose each iteration started from."""
    R = np.eye(3) if R0 is None else np.asarray(R0, np.float64)
    t = np.zeros(3) if t0 is None else np.asarray(t0, np.float64)
    hist = []
    for _ in range(iters):
        R, t, E, cnt = icp_step(cam, depth, points, normals, prm, R, t)
        hist.append((E, cnt))
    return R, t, hist
