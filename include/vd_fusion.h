/*
 * vd_fusion.h -- C-ABI of the reconstruction around the lattice solve:
 * non-rigid TSDF fusion of a depth frame into the canonical volume (Sec. 8)
 * and the data-parallel marching cubes that extracts the canonical surface
 * and deforms it by the current field (Sec. 4).
 *
 * The truncated signed distance D_i and its confidence W_i live on the
 * finest level's grid of a vd_lattice handle (one value per lattice point,
 * float32, both 0 at creation: W = 0 means never observed).  Fusion uses the
 * handle's depth frame and pose (vd_track.h) and its current state.
 *
 * Fusion of grid point i (readings where the paper is silent):
 *   - its deformed position x_i = R (t_hat_i + d_i) + t is projected into
 *     the depth map (the camera model of vd_track.h); with a measurement
 *     z > 0 at that pixel, eta = z - x_i.z is the projective signed distance;
 *   - eta < -tau (behind the truncation band): no update; otherwise the
 *     sample s = min(1, eta / tau) enters the weighted floating average
 *     D_i <- (W_i D_i + s) / (W_i + 1), W_i <- min(W_i + 1, W_max), computed
 *     in float64 from the stored float32 values;
 *   - only points of the optimised set M (every point without
 *     VD_FLAG_ACTIVE_SET) that have been in it for at least k_min frames in a
 *     row are updated (Sec. 8: K_min = 3), unless all_points is set (the
 *     first frame, before any surface exists).  The frame count of a point
 *     grows by one at the end of every vd_solve_frame / vd_track_frame call
 *     in which it is in M and drops to 0 otherwise.
 *
 * Marching cubes: every cell whose 8 corners have W > 0 is cut by D = 0
 * (a corner is inside when D < 0); the vertex on an edge (a, b) whose
 * corners differ is x_a + (D_a / (D_a - D_b)) (x_b - x_a) (float64, rounded
 * to float32).  A cell's polygon is built face by face: walking each face's
 * corners counter-clockwise as seen from outside the cube, each run of inside
 * corners gives a segment from the edge entering it to the edge leaving it
 * (diagonal inside corners of a face are cut off separately); the segments
 * chain into loops, each split into a fan from its lowest-numbered edge, so
 * triangles face away from the inside.  Corners are k = dx + 2 dy + 4 dz; the
 * 12 edges are numbered 4 q + j along axis q, j = b1 + 2 b2 from the bits of
 * the other two axes in increasing order.  Triangles are emitted in
 * increasing cell order (x fastest), within a cell in loop and fan order,
 * found by a prefix sum of the per-cell triangle counts.  Deformed vertices
 * are S(x) = R (x + sum_k alpha_k(x) d_k) + t over the finest cell holding x.
 */
#ifndef VD_FUSION_H
#define VD_FUSION_H

#include <stdint.h>

#include "vd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double tau;         /* truncation distance, world units (> 0) */
  double w_max;       /* confidence cap (>= 1) */
  int32_t k_min;      /* frames in M before a point is fused (>= 0) */
  int32_t all_points; /* 1: fuse into every grid point (first frame) */
} vd_fuse_opts;

/* Fuse the handle's depth frame (vd_set_depth_frame) into its TSDF at the
 * current state and pose (Sec. 8).  *n_updated (may be NULL) receives the
 * number of grid points updated, after waiting for the stream; without it
 * the call is asynchronous.  VD_ESTATE without a depth frame; VD_EINVAL for
 * bad options. */
int vd_fuse_depth(vd_lattice* l, const vd_fuse_opts* o, int64_t* n_updated);

/* Copy the TSDF out: D[N], W[N] (float32) and frames[N] (int32, frames in a
 * row each point has been in M); any pointer may be NULL.  Waits for the
 * stream. */
int vd_get_tsdf(vd_lattice* l, float* D, float* W, int32_t* frames, int32_t mem);

/* Overwrite the TSDF (checkpoint / resume, tests).  VD_EINVAL on non-finite
 * or negative-confidence input.  Waits for the stream. */
int vd_set_tsdf(vd_lattice* l, const float* D, const float* W, int32_t mem);

/* Extract the canonical surface by marching cubes and deform it (Sec. 4):
 * canon[9 T] and deformed[9 T] receive each triangle's three vertices
 * (canonical and deformed, xyz float32), cells[T] its cell's linear index and
 * edges[3 T] its three edge numbers (deformed, cells and edges may be NULL).
 * *n_triangles receives T.  If capacity < T nothing is written, *n_triangles
 * holds the T needed and the call returns VD_ERANGE.  Waits for the
 * stream. */
int vd_extract_mesh(vd_lattice* l, int64_t capacity, float* canon, float* deformed,
                    int32_t* cells, int32_t* edges, int64_t* n_triangles, int32_t mem);

#ifdef __cplusplus
}
#endif

#endif /* VD_FUSION_H */
