/*
 * vd_track.h -- C-ABI of the per-frame tracking around the lattice solve:
 * projective depth association (Sec. 5.1), the global rigid pose by dense
 * projective ICP (Sec. 4, Sec. 6) and the tracked frame that repeats
 * association and the flip-flop solve ICP-style (Sec. 3).
 *
 * Camera model.  A pinhole camera at the origin looking along +z with the
 * sensor's intrinsics (fx, fy, cx, cy).  Pixel (u, v) covers [u, u+1) x
 * [v, v+1) in image coordinates: a point (x, y, z) with z > 0 falls on pixel
 * (floor(fx x / z + cx), floor(fy y / z + cy)), and the depth D(u, v) of a
 * pixel back-projects at the pixel centre to ((u + 1/2 - cx) D / fx,
 * (v + 1/2 - cy) D / fy, D).  Depth maps are float32 [height][width] in world
 * units (row v, column u); a depth <= 0 marks a pixel without a measurement.
 *
 * Association of a sample p_c with normal n_c (Sec. 5.1): project p_c, read
 * the measured point p_c^a of its pixel and the measured normal n_c^a there,
 * and weigh the pair by the three kernels Phi(x) = 1 - x / eps of the
 * distance |p_c - p_c^a|, the normal deviation 1 - n_c . n_c^a and the view
 * angle 1 - n_c . v_c: w_c = ((Phi_d + Phi_n + Phi_v) / 3)^2, and w_c = 0
 * (pruned) if any kernel is negative.  Readings where the paper is silent:
 *   - the measured normal at pixel (u, v) is the normalised cross product
 *     (P(u+1,v) - P(u-1,v)) x (P(u,v+1) - P(u,v-1)) of back-projected
 *     neighbours turned to face the camera; it exists only when the pixel's
 *     four neighbours lie inside the image, all five depths are > 0 and the
 *     cross product is non-zero;
 *   - v_c is the unit vector from p_c toward the camera centre, -p_c/|p_c|;
 *   - a sample with z <= 0, outside the image, without depth or without a
 *     measured normal is pruned; pruned samples report target = normal = 0;
 *   - decisions (the pixel, pruning) are taken in float64 from the float32
 *     inputs, in the operation order of the formulas above.
 *
 * Rigid pose.  A pose is 12 float64: R row-major (9) then t (3); it maps the
 * lattice (model) frame to the camera frame, x -> R x + t.  One ICP
 * iteration at (R, t) associates the samples q_c = R p_c + t (normals
 * R n_c) and takes the Gauss-Newton step of E(R, t) = sum_c w_c (n_c^a .
 * (q_c - p_c^a))^2 with the weights and targets fixed, linearised in a small
 * rotation w and translation tau applied after the pose (q -> q + w x q +
 * tau): (sum w J J^T) xi = -sum w J r with J_c = [q_c x n_c^a, n_c^a],
 * r_c = n_c^a . (q_c - p_c^a).  The update is R <- Rot(w) R, t <- Rot(w) t +
 * tau, Rot(w) the rotation by |w| about w/|w|.  When fewer than six pairs
 * survive or the 6x6 system is numerically singular (a pivot of its Cholesky
 * factorisation at or below 1e-8 times the largest diagonal entry: a single
 * plane, whose float32-quantised measured normals leave eigenvalues near
 * 1e-11 of the largest instead of 0) the pose is left unchanged.
 *
 * Conventions as in vd.h: VD_* status codes, `mem` = VD_MEM_HOST or
 * VD_MEM_DEVICE for every caller pointer of a call, the caller owns all
 * buffers, nothing is kept after a call returns.
 */
#ifndef VD_TRACK_H
#define VD_TRACK_H

#include <stdint.h>

#include "vd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t width, height; /* pixels (>= 3 each) */
  double fx, fy;         /* focal lengths in pixels (> 0) */
  double cx, cy;         /* principal point in pixels */
} vd_camera;

typedef struct {
  double eps_d; /* distance threshold of Phi_d, world units (> 0) */
  double eps_n; /* threshold of Phi_n on 1 - n_c . n_c^a (> 0) */
  double eps_v; /* threshold of Phi_v on 1 - n_c . v_c (> 0) */
} vd_assoc_params;

/* Association of n camera-frame samples with a depth map (Sec. 5.1).
 *   depth[height*width]            the measurement (float32, see above)
 *   points[3n], normals[3n]        samples p_c and their normals n_c (the
 *                                  normals are renormalised; a zero normal is
 *                                  pruned)
 *   target[3n], normal_out[3n]     p_c^a and n_c^a of every kept pair, 0 for
 *                                  pruned ones (float32 roundings of the
 *                                  float64 values)
 *   weight[n]                      w_c (0: pruned)
 *   pixel[n] (may be NULL)         v * width + u of the pixel a sample falls
 *                                  on, -1 if none
 * VD_EINVAL on a bad camera, a non-positive eps or a NULL buffer with n > 0.
 * Synchronous, on `stream` (a hipStream_t or NULL). */
int vd_associate(const vd_camera* cam, const float* depth, const float* points,
                 const float* normals, int64_t n, const vd_assoc_params* prm, float* target,
                 float* normal_out, float* weight, int32_t* pixel, int32_t mem, void* stream);

/* Global rigid pose by `iters` iterations of projective point-to-plane ICP
 * (Sec. 6: solved first, before the non-rigid step) on n model-frame samples
 * points[3n] with normals normals[3n], against the depth map.  pose[12] is
 * read as the start and overwritten with the result.  hist (may be NULL)
 * receives 2 * iters float64: per iteration, E(R, t) at the pose the
 * iteration started from and the number of kept pairs.  Device scratch of
 * the reduction is allocated by the call.  VD_EINVAL as vd_associate, or
 * iters < 0 or a non-finite pose.  Synchronous, on `stream`. */
int vd_rigid_pose(const vd_camera* cam, const float* depth, const float* points,
                  const float* normals, int64_t n, const vd_assoc_params* prm, int32_t iters,
                  double* pose, double* hist, int32_t mem, void* stream);

/* ---- tracking of a lattice (a vd_lattice handle of vd.h) --------------- */

/* One sensor frame for a lattice.  The model samples are canonical surface
 * samples p_hat_c with canonical normals n_hat_c (the isosurface of Sec. 5.1);
 * at the lattice state (d_i = t_i - t_hat_i, R_i) and pose (R, t) they sit at
 *   p_c = R (p_hat_c + sum_k alpha_k d_k) + t,
 *   n_c = R sum_k alpha_k R_k n_hat_c  (renormalised by the association)
 * (the trilinear field of Sec. 4 over the finest level's cell corners k =
 * dx + 2 dy + 4 dz, summed in that order).  The
 * sparse pairs are canonical points and camera-frame targets (eq. (3)). */
typedef struct {
  vd_camera camera;
  const float* depth;        /* [height*width] */
  int64_t n_model;
  const float* model_canon;  /* [3 n_model], inside the coarsest level's box */
  const float* model_normal; /* [3 n_model] */
  int64_t n_sparse;
  const float* sparse_canon;  /* [3 n_sparse] */
  const float* sparse_target; /* [3 n_sparse], camera frame */
  vd_assoc_params assoc;
  int32_t mem; /* VD_MEM_HOST or VD_MEM_DEVICE for every pointer above */
  int32_t reserved;
} vd_depth_frame;

/* Replace the handle's frame: copies and validates the depth map, the model
 * samples and the sparse pairs (VD_EINVAL: non-finite value, bad camera or
 * eps; VD_ERANGE: a canonical point outside the coarsest level) and builds
 * the per-level row structure of the samples (Sec. 7.1), whose weights the
 * association of vd_track_frame fills.  Replaces constraints set by
 * vd_set_constraints.  Waits for the validation result. */
int vd_set_depth_frame(vd_lattice* l, const vd_depth_frame* f);

/* Pose of the handle (12 float64, see above; identity at creation). */
int vd_get_pose(vd_lattice* l, double pose[12]);
int vd_set_pose(vd_lattice* l, const double pose[12]);

typedef struct {
  int32_t rigid_iters;   /* ICP iterations of the global pose first (Sec. 6) */
  int32_t icp_iters;     /* rounds of association + flip-flop solve (Sec. 3) */
  int32_t reset_to_rest; /* start the lattice from t = t_hat, R = I */
  int32_t reserved;
} vd_track_opts;

#define VD_TRACK_MAX_ITERS 64

typedef struct {
  double energy[4];   /* eq. (1) terms at the final state (as vd_get_energy) */
  double pose[12];    /* the pose used by the non-rigid rounds */
  double rigid_hist[2 * VD_TRACK_MAX_ITERS]; /* per rigid iteration: E and
                                                kept pairs (vd_rigid_pose) */
  int32_t assoc_kept[VD_TRACK_MAX_ITERS];    /* kept pairs per round */
  uint32_t bits;      /* VD_REPORT_* of the last round's solve */
  int32_t reserved;
} vd_track_report;

/* Track one frame: `rigid_iters` ICP iterations of the global pose on the
 * deformed model samples, then `icp_iters` rounds of [associate the model
 * samples at the current state and pose, replace the dense rows' targets,
 * normals and weights with the association's (in the lattice frame:
 * R^T (p^a - t), R^T n^a), and run the flip-flop schedule of vd_solve_frame
 * from the current state].  The sparse targets enter as R^T (f - t).
 * Everything stays on the GPU (the pose too); asynchronous unless `report`
 * is given.  VD_ESTATE without a frame; VD_EINVAL for iteration counts
 * outside [0, VD_TRACK_MAX_ITERS]. */
int vd_track_frame(vd_lattice* l, const vd_track_opts* o, vd_track_report* report);

/* Test entry point (unstable): association of the frame's model samples at a
 * given finest state -- displacements disp[3N] (xyz triples, d = t - t_hat)
 * and rotations rot[9N] -- and the handle's pose, as vd_track_frame does it:
 * target[3M], normal_out[3M] in the lattice frame, weight[M], pixel[M]
 * (may be NULL).  Synchronous. */
int vd_debug_associate(vd_lattice* l, const float* disp, const float* rot, float* target,
                       float* normal_out, float* weight, int32_t* pixel, int32_t mem);

/* ---- no-allocation entry point ------------------------------------------ */

#define VD_NOALLOC_MAX_SAMPLES (1ll << 30)

/* vd_rigid_pose for callers that cannot allocate device memory: code under
 * HIP graph capture, serving loops and harnesses that forbid hipMalloc.
 * Arguments and results as vd_rigid_pose with mem = VD_MEM_DEVICE: every
 * pointer is device memory of the current GPU, pose[12] is read and updated
 * in place on the device, hist (may be NULL) receives 2 * iters float64
 * there.  The reduction's workgroup partials live in a fixed library-owned
 * device array (256 KiB per GPU, held until the process ends); the call
 * allocates nothing and does not wait for the GPU.  Every partial a call
 * reads it has written before in the same call, so nothing has to start at
 * zero.  Calls that overlap on one GPU share that array and race: serialise
 * them (one stream, or events).  VD_ERANGE for n > VD_NOALLOC_MAX_SAMPLES;
 * otherwise VD_EINVAL as vd_rigid_pose (the pose, being device memory, is not
 * checked for finite values). */
int vd_rigid_pose_noalloc(const vd_camera* cam, const float* depth, const float* points,
                          const float* normals, int64_t n, const vd_assoc_params* prm,
                          int32_t iters, double* pose, double* hist, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VD_TRACK_H */
