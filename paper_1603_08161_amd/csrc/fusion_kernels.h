// Launchers of the TSDF fusion and marching-cubes kernels (fusion.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vd_kernels.h"

namespace vd {

// Camera, grid and fusion parameters of one fusion step.
struct FuseParams {
  int W, H;
  double fx, fy, cx, cy;
  double ox, oy, oz, h;  // the finest level's origin and spacing
  double tau, w_max;
  int k_min;
  int all_points;
};

// Grid of the mesh extraction (the finest level).
struct MeshParams {
  double ox, oy, oz, h;
};

// Upload the marching-cubes case table to the current GPU (once per
// device); 0 on success.
int mc_table_ready();

template <typename T>
hipError_t launch_fuse(const FuseParams& p, const LevelView<T>& L, const float* depth,
                       const double* pose, const int* frames, float* D, float* W, int* n_updated,
                       hipStream_t s);

// frames[i] = frames[i] + 1 for the points of M (every point without M), 0
// for the others: frames in a row a point has been optimised.
template <typename T>
hipError_t launch_count_frames(const LevelView<T>& L, int* frames, hipStream_t s);

// Triangles per cell (0 for cells with an unobserved corner).
hipError_t launch_mc_count(const float* D, const float* W, int nx, int ny, int nz, int* counts,
                           hipStream_t s);

// Triangles of every cell at its exclusive-scan offset: canonical vertices
// [9 per triangle], deformed vertices (may be null), cell ids and edge
// numbers (may be null).
template <typename T>
hipError_t launch_mc_emit(const MeshParams& p, const LevelView<T>& L, const float* D,
                          const float* W, const int* counts, const int* offsets,
                          const double* pose, float* canon, float* deformed, int* cells,
                          int* edges, hipStream_t s);

}  // namespace vd
