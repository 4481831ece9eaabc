// The no-allocation variant of the rigid pose (vd_rigid_pose_noalloc in
// include/vd_track.h).  Its only device memory beyond the caller's inputs and
// outputs is the reduction's workgroup partials, kept in a file-scope device
// array; each GPU holds its own copy, whose address is looked up once per
// device and used for every launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/vd_track.h"
#include "track_kernels.h"

namespace {

// Workgroup partials of one rigid-ICP reduction: kRigidMaxBlocks workgroups
// of kRigidStride float64 (256 KiB).
constexpr int kScratchDoubles = vd::kRigidMaxBlocks * vd::kRigidStride;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_scratch[kMaxDevices] = {nullptr};

// Device address of the current GPU's copy of `scratch` (looked up on the
// first call on that GPU).
int scratch_of_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VD_EHIP;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return VD_EHIP;
    }
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return VD_OK;
}

}  // namespace

extern "C" int vd_rigid_pose_noalloc(const vd_camera* cam, const float* depth,
                                     const float* points, const float* normals, int64_t n,
                                     const vd_assoc_params* prm, int32_t iters, double* pose,
                                     double* hist, void* stream) {
  if (!cam || !prm || !depth || !pose || iters < 0) return VD_EINVAL;
  if (n < 0 || (n > 0 && (!points || !normals))) return VD_EINVAL;
  if (n > VD_NOALLOC_MAX_SAMPLES) return VD_ERANGE;
  if (cam->width < 3 || cam->height < 3 || (int64_t)cam->width * cam->height > (1ll << 30))
    return VD_EINVAL;
  const double v[7] = {cam->fx, cam->fy, cam->cx, cam->cy, prm->eps_d, prm->eps_n, prm->eps_v};
  for (double x : v)
    if (!std::isfinite(x)) return VD_EINVAL;
  if (!(cam->fx > 0.0) || !(cam->fy > 0.0) || !(prm->eps_d > 0.0) || !(prm->eps_n > 0.0) ||
      !(prm->eps_v > 0.0))
    return VD_EINVAL;
  const int G = vd::rigid_blocks(n);
  if (G > vd::kRigidMaxBlocks) return VD_ERANGE;
  if (iters == 0) return VD_OK;
  double* part = nullptr;
  const int rc = scratch_of_current_device(&part);
  if (rc != VD_OK) return rc;
  vd::CamAssoc c;
  c.W = cam->width; c.H = cam->height;
  c.fx = cam->fx; c.fy = cam->fy; c.cx = cam->cx; c.cy = cam->cy;
  c.eps_d = prm->eps_d; c.eps_n = prm->eps_n; c.eps_v = prm->eps_v;
  hipStream_t s = (hipStream_t)stream;
  for (int it = 0; it < iters; ++it) {
    if (vd::launch_rigid_reduce_points(c, depth, points, normals, (int)n, pose, part, G, s) !=
            hipSuccess ||
        vd::launch_rigid_solve(part, G, pose, hist ? hist + 2 * it : nullptr, s) != hipSuccess)
      return VD_EHIP;
  }
  return VD_OK;
}
