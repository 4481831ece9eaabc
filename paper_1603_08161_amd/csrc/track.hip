// Tracking kernels (gfx950): projective depth association (Sec. 5.1), the
// global rigid pose by projective point-to-plane ICP (Sec. 4, Sec. 6) and the
// association of a lattice's deformed model samples (Sec. 3: repeated
// ICP-style around the non-rigid solve).
//
// Every decision (the pixel a sample falls on, pruning) is taken in float64
// from the float32 inputs, in the operation order of the formulas written
// here; this file is compiled without floating-point contraction, so no
// product is fused into a following sum behind the written order.

#include "track_kernels.h"
#include "vd_device.h"

namespace vd {

namespace {

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Measurement of pixel (u, v) at its centre: ((u + 1/2 - cx) z / fx,
// (v + 1/2 - cy) z / fy, z).
__device__ __forceinline__ void backproject(const CamAssoc& c, int u, int v, double z,
                                            double P[3]) {
  P[0] = (((double)u + 0.5) - c.cx) * z / c.fx;
  P[1] = (((double)v + 0.5) - c.cy) * z / c.fy;
  P[2] = z;
}

struct Pair {
  double pa[3];  // measured point p^a
  double na[3];  // measured normal n^a (facing the camera)
  double w;      // w_c; 0 when pruned
  int pix;       // v * W + u, -1 outside the image
};

// Association of one camera-frame sample p with normal n (Sec. 5.1).
__device__ __forceinline__ Pair associate(const CamAssoc& c, const float* __restrict__ depth,
                                          const double p[3], const double n[3]) {
  Pair o;
  for (int k = 0; k < 3; ++k) {
    o.pa[k] = 0.0;
    o.na[k] = 0.0;
  }
  o.w = 0.0;
  o.pix = -1;
  if (!(p[2] > 0.0)) return o;
  const double uf = floor(c.fx * p[0] / p[2] + c.cx);
  const double vf = floor(c.fy * p[1] / p[2] + c.cy);
  if (!(uf >= 0.0 && uf < (double)c.W && vf >= 0.0 && vf < (double)c.H)) return o;
  const int u = (int)uf, v = (int)vf;
  o.pix = v * c.W + u;
  const size_t W = (size_t)c.W;
  const double z = (double)depth[(size_t)v * W + u];
  if (!(z > 0.0)) return o;
  if (u < 1 || u > c.W - 2 || v < 1 || v > c.H - 2) return o;
  const double zr = (double)depth[(size_t)v * W + u + 1];
  const double zl = (double)depth[(size_t)v * W + u - 1];
  const double zd = (double)depth[(size_t)(v + 1) * W + u];
  const double zu = (double)depth[(size_t)(v - 1) * W + u];
  if (!(zr > 0.0 && zl > 0.0 && zd > 0.0 && zu > 0.0)) return o;
  double Pr[3], Pl[3], Pd[3], Pu[3], pa[3];
  backproject(c, u + 1, v, zr, Pr);
  backproject(c, u - 1, v, zl, Pl);
  backproject(c, u, v + 1, zd, Pd);
  backproject(c, u, v - 1, zu, Pu);
  backproject(c, u, v, z, pa);
  double dx[3], dy[3], na[3];
  for (int k = 0; k < 3; ++k) {
    dx[k] = Pr[k] - Pl[k];
    dy[k] = Pd[k] - Pu[k];
  }
  na[0] = dx[1] * dy[2] - dx[2] * dy[1];
  na[1] = dx[2] * dy[0] - dx[0] * dy[2];
  na[2] = dx[0] * dy[1] - dx[1] * dy[0];
  const double ln = sqrt(dot3(na, na));
  if (!(ln > 0.0)) return o;
  for (int k = 0; k < 3; ++k) na[k] = na[k] / ln;
  if (dot3(na, pa) > 0.0)
    for (int k = 0; k < 3; ++k) na[k] = -na[k];
  const double lc = sqrt(dot3(n, n));
  if (!(lc > 0.0)) return o;
  double nc[3], d[3], view[3];
  const double lp = sqrt(dot3(p, p));
  for (int k = 0; k < 3; ++k) {
    nc[k] = n[k] / lc;
    d[k] = p[k] - pa[k];
    view[k] = -p[k] / lp;
  }
  const double phi_d = 1.0 - sqrt(dot3(d, d)) / c.eps_d;
  const double phi_n = 1.0 - (1.0 - dot3(nc, na)) / c.eps_n;
  const double phi_v = 1.0 - (1.0 - dot3(nc, view)) / c.eps_v;
  if (!(phi_d >= 0.0 && phi_n >= 0.0 && phi_v >= 0.0)) return o;
  const double s = (phi_d + phi_n + phi_v) / 3.0;
  for (int k = 0; k < 3; ++k) {
    o.pa[k] = pa[k];
    o.na[k] = na[k];
  }
  o.w = s * s;
  return o;
}

// Model sample i deformed by the lattice state (Sec. 4): p = p_hat +
// sum_k alpha_k d_k and the un-normalised normal sum_k alpha_k R_k n_hat,
// over the corners k = dx + 2 dy + 4 dz of the finest cell holding p_hat.
template <typename T>
__device__ __forceinline__ void deform(const ModelView<T>& m, int i, double p[3], double nc[3]) {
  double x[3], nh[3], f[3];
  int cc[3];
  const double o[3] = {m.ox, m.oy, m.oz};
  const int nn[3] = {m.nx, m.ny, m.nz};
  for (int k = 0; k < 3; ++k) {
    x[k] = (double)m.canon[3 * (size_t)i + k];
    nh[k] = (double)m.cnormal[3 * (size_t)i + k];
    const double u = (x[k] - o[k]) / m.h;
    double fl = floor(u);
    if (fl < 0.0) fl = 0.0;
    if (fl > (double)(nn[k] - 2)) fl = (double)(nn[k] - 2);
    cc[k] = (int)fl;
    f[k] = u - fl;
  }
  double s[3] = {0.0, 0.0, 0.0};
  nc[0] = nc[1] = nc[2] = 0.0;
  const size_t N = (size_t)m.N;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ex = k & 1, ey = (k >> 1) & 1, ez = (k >> 2) & 1;
    const double wx = ex ? f[0] : 1.0 - f[0];
    const double wy = ey ? f[1] : 1.0 - f[1];
    const double wz = ez ? f[2] : 1.0 - f[2];
    const double a = wx * wy * wz;
    const size_t id = (size_t)(cc[0] + ex) +
                      (size_t)m.nx * ((size_t)(cc[1] + ey) + (size_t)m.ny * (cc[2] + ez));
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      s[r] += a * (double)m.d[r * N + id];
      const double rn = (double)m.rot[(3 * r) * N + id] * nh[0] +
                        (double)m.rot[(3 * r + 1) * N + id] * nh[1] +
                        (double)m.rot[(3 * r + 2) * N + id] * nh[2];
      nc[r] += a * rn;
    }
  }
  for (int r = 0; r < 3; ++r) p[r] = x[r] + s[r];
}

// x -> R x + t and n -> R n for pose P = (R row-major, t).
__device__ __forceinline__ void apply_pose(const double* P, const double p[3], const double n[3],
                                           double q[3], double nq[3]) {
  for (int r = 0; r < 3; ++r) {
    q[r] = P[3 * r] * p[0] + P[3 * r + 1] * p[1] + P[3 * r + 2] * p[2] + P[9 + r];
    nq[r] = P[3 * r] * n[0] + P[3 * r + 1] * n[1] + P[3 * r + 2] * n[2];
  }
}

// R^T (x - t); with t_is_zero the subtraction is skipped (x - 0 = x).
__device__ __forceinline__ void to_model(const double* P, const double x[3], bool t_is_zero,
                                         double out[3]) {
  double dx[3];
  for (int k = 0; k < 3; ++k) dx[k] = t_is_zero ? x[k] : x[k] - P[9 + k];
  for (int r = 0; r < 3; ++r) out[r] = P[r] * dx[0] + P[3 + r] * dx[1] + P[6 + r] * dx[2];
}

// Per-sample terms of the rigid ICP normal equations, added to acc.
__device__ __forceinline__ void rigid_terms(const Pair& a, const double q[3], double (&acc)[kRigidSums]) {
  if (!(a.w > 0.0)) return;
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = q[k] - a.pa[k];
  const double r = dot3(a.na, d);
  double J[6];
  J[0] = q[1] * a.na[2] - q[2] * a.na[1];
  J[1] = q[2] * a.na[0] - q[0] * a.na[2];
  J[2] = q[0] * a.na[1] - q[1] * a.na[0];
  J[3] = a.na[0];
  J[4] = a.na[1];
  J[5] = a.na[2];
  int e = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double wj = J[i] * a.w;
#pragma unroll
    for (int j = i; j < 6; ++j) acc[e++] += wj * J[j];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) acc[21 + i] += J[i] * a.w * r;
  acc[27] += a.w * r * r;
  acc[28] += 1.0;
}

__device__ __forceinline__ void write_rigid_partials(double (&acc)[kRigidSums], double* partials) {
  __shared__ double lds[kRigidSums * (kBlock / kWave)];
  block_sum<kRigidSums>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRigidSums; ++k) partials[(size_t)blockIdx.x * kRigidStride + k] = acc[k];
  }
}

}  // namespace

int rigid_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > kRigidMaxBlocks) b = kRigidMaxBlocks;
  return (int)b;
}

// ---------------------------------------------------------------------------
// association
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_associate(CamAssoc c, const float* __restrict__ depth,
                                                      const float* __restrict__ pts,
                                                      const float* __restrict__ nrm, int n,
                                                      float* target, float* normal_out,
                                                      float* weight, int* pixel) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double p[3], q[3];
  for (int k = 0; k < 3; ++k) {
    p[k] = (double)pts[3 * (size_t)i + k];
    q[k] = (double)nrm[3 * (size_t)i + k];
  }
  const Pair a = associate(c, depth, p, q);
  const bool keep = a.w > 0.0;
  for (int k = 0; k < 3; ++k) {
    target[3 * (size_t)i + k] = keep ? (float)a.pa[k] : 0.0f;
    normal_out[3 * (size_t)i + k] = keep ? (float)a.na[k] : 0.0f;
  }
  weight[i] = keep ? (float)a.w : 0.0f;
  if (pixel) pixel[i] = a.pix;
}

hipError_t launch_associate(const CamAssoc& c, const float* depth, const float* pts,
                            const float* nrm, int n, float* target, float* normal_out,
                            float* weight, int* pixel, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_associate<<<blocks_for(n), kBlock, 0, s>>>(c, depth, pts, nrm, n, target, normal_out, weight,
                                               pixel);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_assoc_lattice(CamAssoc c,
                                                          const float* __restrict__ depth,
                                                          ModelView<T> m,
                                                          const double* __restrict__ pose,
                                                          float* target, float* normal_out,
                                                          float* weight, int* pixel, int* kept) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < m.M) {
    double P[12];
    for (int k = 0; k < 12; ++k) P[k] = pose[k];
    double p[3], nc[3], q[3], nq[3];
    deform(m, i, p, nc);
    apply_pose(P, p, nc, q, nq);
    const Pair a = associate(c, depth, q, nq);
    const bool keep = a.w > 0.0;
    double tl[3] = {0.0, 0.0, 0.0}, nl[3] = {0.0, 0.0, 0.0};
    if (keep) {
      to_model(P, a.pa, false, tl);
      to_model(P, a.na, true, nl);
      atomicAdd(&cnt, 1);
    }
    for (int k = 0; k < 3; ++k) {
      target[3 * (size_t)i + k] = (float)tl[k];
      normal_out[3 * (size_t)i + k] = (float)nl[k];
    }
    weight[i] = keep ? (float)a.w : 0.0f;
    if (pixel) pixel[i] = a.pix;
  }
  __syncthreads();
  if (threadIdx.x == 0 && kept && cnt) atomicAdd(kept, cnt);
}

template <typename T>
hipError_t launch_assoc_lattice(const CamAssoc& c, const float* depth, const ModelView<T>& m,
                                const double* pose, float* target, float* normal_out,
                                float* weight, int* pixel, int* kept, hipStream_t s) {
  if (m.M <= 0) return hipSuccess;
  k_assoc_lattice<T><<<blocks_for(m.M), kBlock, 0, s>>>(c, depth, m, pose, target, normal_out,
                                                        weight, pixel, kept);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// rigid pose: reduction of the 6x6 normal equations, then the solve
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_rigid_reduce_points(
    CamAssoc c, const float* __restrict__ depth, const float* __restrict__ pts,
    const float* __restrict__ nrm, int n, const double* __restrict__ pose, double* partials) {
  double P[12];
  for (int k = 0; k < 12; ++k) P[k] = pose[k];
  double acc[kRigidSums];
#pragma unroll
  for (int k = 0; k < kRigidSums; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double p[3], nn[3], q[3], nq[3];
    for (int k = 0; k < 3; ++k) {
      p[k] = (double)pts[3 * (size_t)i + k];
      nn[k] = (double)nrm[3 * (size_t)i + k];
    }
    apply_pose(P, p, nn, q, nq);
    const Pair a = associate(c, depth, q, nq);
    rigid_terms(a, q, acc);
  }
  write_rigid_partials(acc, partials);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rigid_reduce_lattice(
    CamAssoc c, const float* __restrict__ depth, ModelView<T> m, const double* __restrict__ pose,
    double* partials) {
  double P[12];
  for (int k = 0; k < 12; ++k) P[k] = pose[k];
  double acc[kRigidSums];
#pragma unroll
  for (int k = 0; k < kRigidSums; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m.M; i += gridDim.x * kBlock) {
    double p[3], nc[3], q[3], nq[3];
    deform(m, i, p, nc);
    apply_pose(P, p, nc, q, nq);
    const Pair a = associate(c, depth, q, nq);
    rigid_terms(a, q, acc);
  }
  write_rigid_partials(acc, partials);
}

hipError_t launch_rigid_reduce_points(const CamAssoc& c, const float* depth, const float* pts,
                                      const float* nrm, int n, const double* pose,
                                      double* partials, int blocks, hipStream_t s) {
  if (blocks < 1 || blocks > kRigidMaxBlocks) return hipErrorInvalidValue;
  k_rigid_reduce_points<<<blocks, kBlock, 0, s>>>(c, depth, pts, nrm, n, pose, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rigid_reduce_lattice(const CamAssoc& c, const float* depth,
                                       const ModelView<T>& m, const double* pose,
                                       double* partials, int blocks, hipStream_t s) {
  if (blocks < 1 || blocks > kRigidMaxBlocks) return hipErrorInvalidValue;
  k_rigid_reduce_lattice<T><<<blocks, kBlock, 0, s>>>(c, depth, m, pose, partials);
  return hipGetLastError();
}

// One workgroup: the partial sums in fixed order (value k by 8 threads, each
// over every 8th workgroup, then the 8 in order), the Cholesky factorisation
// of the 6x6 system, the step xi = -H^-1 g and the pose update.
__global__ __launch_bounds__(kBlock) void k_rigid_solve(const double* __restrict__ partials,
                                                        int blocks, double* pose, double* hist) {
  __shared__ double part[8][kRigidStride];
  __shared__ double tot[kRigidStride];
  const int k = threadIdx.x % kRigidStride, s = threadIdx.x / kRigidStride;
  double acc = 0.0;
  if (k < kRigidSums)
    for (int b = s; b < blocks; b += 8) acc += partials[(size_t)b * kRigidStride + k];
  part[s][k] = acc;
  __syncthreads();
  if (threadIdx.x < kRigidSums) {
    double t = 0.0;
    for (int j = 0; j < 8; ++j) t += part[j][threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double E = tot[27], count = tot[28];
  if (hist) {
    hist[0] = E;
    hist[1] = count;
  }
  double H[6][6], g[6];
  int e = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      H[i][j] = tot[e];
      H[j][i] = tot[e];
      ++e;
    }
  for (int i = 0; i < 6; ++i) g[i] = tot[21 + i];
  if (count < 6.0) return;
  double dmax = 0.0;
  for (int i = 0; i < 6; ++i) dmax = fmax(dmax, H[i][i]);
  if (!(dmax > 0.0)) return;
  // H = L L^T
  double L[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) L[i][j] = 0.0;
  for (int j = 0; j < 6; ++j) {
    double dj = H[j][j];
    for (int q = 0; q < j; ++q) dj -= L[j][q] * L[j][q];
    if (!(dj > 1e-8 * dmax)) return;  // numerically singular: the pose stays
    L[j][j] = sqrt(dj);
    for (int i = j + 1; i < 6; ++i) {
      double v = H[i][j];
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      L[i][j] = v / L[j][j];
    }
  }
  double y[6], xi[6];
  for (int i = 0; i < 6; ++i) {
    double v = -g[i];
    for (int q = 0; q < i; ++q) v -= L[i][q] * y[q];
    y[i] = v / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double v = y[i];
    for (int q = i + 1; q < 6; ++q) v -= L[q][i] * xi[q];
    xi[i] = v / L[i][i];
  }
  // Rot(w): rotation by |w| about w / |w| (Rodrigues)
  double Q[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  const double th = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
  if (th > 0.0) {
    const double ax = xi[0] / th, ay = xi[1] / th, az = xi[2] / th;
    const double K[3][3] = {{0.0, -az, ay}, {az, 0.0, -ax}, {-ay, ax, 0.0}};
    const double sn = sin(th), cs = 1.0 - cos(th);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double kk = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
        Q[i][j] = Q[i][j] + sn * K[i][j] + cs * kk;
      }
  }
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = pose[i];
  for (int i = 0; i < 3; ++i) t[i] = pose[9 + i];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      pose[3 * i + j] = Q[i][0] * R[j] + Q[i][1] * R[3 + j] + Q[i][2] * R[6 + j];
    pose[9 + i] = Q[i][0] * t[0] + Q[i][1] * t[1] + Q[i][2] * t[2] + xi[3 + i];
  }
}

hipError_t launch_rigid_solve(const double* partials, int blocks, double* pose, double* hist,
                              hipStream_t s) {
  if (blocks < 1 || blocks > kRigidMaxBlocks) return hipErrorInvalidValue;
  k_rigid_solve<<<1, kBlock, 0, s>>>(partials, blocks, pose, hist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_to_model_frame(const double* __restrict__ pose,
                                                           const float* __restrict__ in,
                                                           float* out, int S) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= S) return;
  double P[12], x[3], y[3];
  for (int k = 0; k < 12; ++k) P[k] = pose[k];
  for (int k = 0; k < 3; ++k) x[k] = (double)in[3 * (size_t)i + k];
  to_model(P, x, false, y);
  for (int k = 0; k < 3; ++k) out[3 * (size_t)i + k] = (float)y[k];
}

hipError_t launch_to_model_frame(const double* pose, const float* in, float* out, int S,
                                 hipStream_t s) {
  if (S <= 0) return hipSuccess;
  k_to_model_frame<<<blocks_for(S), kBlock, 0, s>>>(pose, in, out, S);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<blocks_for(n), kBlock, 0, s>>>(p, n, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_fill_float(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

hipError_t launch_fill_float(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  k_fill_float<<<(int)b, kBlock, 0, s>>>(p, n, v);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_aos_to_soa(const float* __restrict__ in, T* out,
                                                       int n, int k) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < k; ++j) out[(size_t)j * n + i] = (T)in[(size_t)k * i + j];
}

template <typename T>
hipError_t launch_aos_to_soa(const float* in, T* out, int n, int k, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_aos_to_soa<T><<<blocks_for(n), kBlock, 0, s>>>(in, out, n, k);
  return hipGetLastError();
}

#define VD_TRACK_INSTANTIATE(T)                                                                \
  template hipError_t launch_assoc_lattice<T>(const CamAssoc&, const float*,                  \
                                              const ModelView<T>&, const double*, float*,      \
                                              float*, float*, int*, int*, hipStream_t);        \
  template hipError_t launch_rigid_reduce_lattice<T>(const CamAssoc&, const float*,           \
                                                     const ModelView<T>&, const double*,       \
                                                     double*, int, hipStream_t);               \
  template hipError_t launch_aos_to_soa<T>(const float*, T*, int, int, hipStream_t);
VD_TRACK_INSTANTIATE(float)
VD_TRACK_INSTANTIATE(double)

}  // namespace vd
