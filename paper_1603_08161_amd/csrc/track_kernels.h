// Launchers of the tracking kernels (track.hip): projective depth
// association (Sec. 5.1), the rigid pose by projective ICP (Sec. 4, Sec. 6)
// and the association of a lattice's deformed model samples.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vd {

// Pinhole camera and the association thresholds.
struct CamAssoc {
  int W, H;
  double fx, fy, cx, cy;
  double eps_d, eps_n, eps_v;
};

// Model samples deformed by a lattice level's state (displacements d, SoA
// [3][N], rotations SoA [9][N] row-major entries).
template <typename T>
struct ModelView {
  const float* canon;    // [3M] canonical positions
  const float* cnormal;  // [3M] canonical normals
  int M;
  const T* d;
  const T* rot;
  int nx, ny, nz, N;
  double h, ox, oy, oz;
};

// Rigid-pose reduction: 21 entries of sum w J J^T (upper triangle, row
// major), 6 of sum w J r, E and the kept count per workgroup.
constexpr int kRigidSums = 29;
constexpr int kRigidStride = 32;  // doubles per workgroup partial
constexpr int kRigidMaxBlocks = 1024;

// Workgroups of a rigid-pose reduction over n samples.
int rigid_blocks(int64_t n);

// Camera-frame samples (float32 AoS) -> association outputs (float32).
hipError_t launch_associate(const CamAssoc& c, const float* depth, const float* pts,
                            const float* nrm, int n, float* target, float* normal_out,
                            float* weight, int* pixel, hipStream_t s);

// Lattice samples at `pose` (device float64[12]) -> lattice-frame targets,
// normals and weights; kept (may be null) counts pairs with w > 0.
template <typename T>
hipError_t launch_assoc_lattice(const CamAssoc& c, const float* depth, const ModelView<T>& m,
                                const double* pose, float* target, float* normal_out,
                                float* weight, int* pixel, int* kept, hipStream_t s);

// One rigid ICP iteration: per-workgroup partial sums (blocks workgroups)...
hipError_t launch_rigid_reduce_points(const CamAssoc& c, const float* depth, const float* pts,
                                      const float* nrm, int n, const double* pose,
                                      double* partials, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_rigid_reduce_lattice(const CamAssoc& c, const float* depth,
                                       const ModelView<T>& m, const double* pose,
                                       double* partials, int blocks, hipStream_t s);
// ... then the 6x6 solve and the pose update in place; hist (may be null)
// receives E and the kept count.
hipError_t launch_rigid_solve(const double* partials, int blocks, double* pose, double* hist,
                              hipStream_t s);

// out[3S] = R^T (in - t) for camera-frame points (float32 AoS).
hipError_t launch_to_model_frame(const double* pose, const float* in, float* out, int S,
                                 hipStream_t s);

// p[0..n) = v.
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s);
hipError_t launch_fill_float(float* p, int64_t n, float v, hipStream_t s);

// AoS [n][k] float32 -> SoA [k][n] T.
template <typename T>
hipError_t launch_aos_to_soa(const float* in, T* out, int n, int k, hipStream_t s);

}  // namespace vd
