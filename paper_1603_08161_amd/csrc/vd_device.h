// Device helpers shared by the solver kernels (gfx950, wave64).
//
// - trilinear corner weights of Sec. 4;
// - wave/block reductions in float64: every reduction kernel writes one
//   partial per block, and the kernel that needs the scalar re-reduces those
//   partials in fixed order (bitwise deterministic, no cross-block fences);
// - the Procrustes rotation fit of Sec. 7.1, solved with Horn's closed form
//   (unit quaternion = dominant eigenvector of a 4x4 symmetric matrix built
//   from the cross-covariance) and a cyclic Jacobi eigen-solver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vd {

constexpr int kBlock = 256;   // threads per workgroup for every kernel
constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kXcds = 8;      // MI355X: 8 accelerator dies, workgroups dealt round-robin

// Tile of the stencil kernels: 8 x 8 x 4 nodes, one node per thread.
constexpr int kTX = 8, kTY = 8, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;  // 600

// Maps the hardware workgroup id to a logical tile id so that each XCD gets a
// contiguous range of tiles (neighbouring tiles then share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks / kXcds, r = nblocks % kXcds;
  const int xcd = bid % kXcds, slot = bid / kXcds;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

// ---------------------------------------------------------------------------
// reductions (float64 sums, fixed order => bitwise deterministic)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum K values over the block; the result is valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds /* K * kBlock/kWave */) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * (kBlock / kWave) + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / kWave; ++w) s += lds[k * (kBlock / kWave) + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Sum of n partials written by the previous kernel, computed by every block
// in the same fixed order (bitwise identical in all blocks).  No block of the
// current kernel writes them, so the kernel boundary alone makes them
// visible: no cross-workgroup fence is needed.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n) {
  __shared__ double lds[kBlock / kWave];
  __shared__ double total;
  double acc = 0.0;
  for (int b = threadIdx.x; b < n; b += kBlock) acc += p[b];
  acc = wave_sum(acc);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if (lane == 0) lds[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) s += lds[w];
    total = s;
  }
  __syncthreads();
  return total;
}

// Block-wide sums of K values written to out[k * stride + blockIdx.x].
template <int K>
__device__ __forceinline__ void write_block_partials(double (&v)[K], double* out, int stride) {
  __shared__ double lds[K * (kBlock / kWave)];
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[(size_t)k * stride + blockIdx.x] = v[k];
  }
}

// ---------------------------------------------------------------------------
// trilinear weights (Sec. 4): corner k = dx + 2 dy + 4 dz
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T corner_weight(int k, T fx, T fy, T fz) {
  const T wx = (k & 1) ? fx : T(1) - fx;
  const T wy = (k & 2) ? fy : T(1) - fy;
  const T wz = (k & 4) ? fz : T(1) - fz;
  return wx * wy * wz;
}

// ---------------------------------------------------------------------------
// symmetric 3x3 block times vector; block stored as xx xy xz yy yz zz
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void sym3_madd(const T* __restrict__ s, T px, T py, T pz,
                                          T& ox, T& oy, T& oz) {
  ox += s[0] * px + s[1] * py + s[2] * pz;
  oy += s[1] * px + s[3] * py + s[4] * pz;
  oz += s[2] * px + s[4] * py + s[5] * pz;
}

// ---------------------------------------------------------------------------
// rotation fit: maximise trace(R^T M) over SO(3)
// ---------------------------------------------------------------------------

template <typename T>
struct Fit {
  T R[9];
  T sigma1, sigma2;  // two largest singular values of M (from the eigenvalues)
  T gap;             // lambda_1 - lambda_2 of Horn's matrix = 2 (sigma2 + d sigma3)
};

template <typename T>
__device__ __forceinline__ void jacobi_rotate(T (&A)[4][4], T (&V)[4][4], int p, int q) {
  const T apq = A[p][q];
  if (apq == T(0)) return;
  const T theta = (A[q][q] - A[p][p]) / (T(2) * apq);
  const T sgn = theta >= T(0) ? T(1) : T(-1);
  const T t = sgn / (fabs(theta) + sqrt(theta * theta + T(1)));
  const T c = T(1) / sqrt(t * t + T(1));
  const T s = t * c;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T akp = A[k][p], akq = A[k][q];
    A[k][p] = c * akp - s * akq;
    A[k][q] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T apk = A[p][k], aqk = A[q][k];
    A[p][k] = c * apk - s * aqk;
    A[q][k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T vkp = V[k][p], vkq = V[k][q];
    V[k][p] = c * vkp - s * vkq;
    V[k][q] = s * vkp + c * vkq;
  }
}

// Horn (1987): with S = M^T (sum source * target^T), the rotation is given by
// the unit quaternion spanning the top eigenvector of the symmetric N below.
template <typename T, int SWEEPS>
__device__ __forceinline__ void fit_rotation(const T (&M)[9], Fit<T>& out) {
  const T Sxx = M[0], Sxy = M[3], Sxz = M[6];
  const T Syx = M[1], Syy = M[4], Syz = M[7];
  const T Szx = M[2], Szy = M[5], Szz = M[8];
  T A[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
               {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
               {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
               {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
  T V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
#pragma unroll 1
  for (int sweep = 0; sweep < SWEEPS; ++sweep) {
    jacobi_rotate(A, V, 0, 1);
    jacobi_rotate(A, V, 0, 2);
    jacobi_rotate(A, V, 0, 3);
    jacobi_rotate(A, V, 1, 2);
    jacobi_rotate(A, V, 1, 3);
    jacobi_rotate(A, V, 2, 3);
  }
  // sort the four eigenvalues (descending) while tracking the top vector
  T l[4] = {A[0][0], A[1][1], A[2][2], A[3][3]};
  int top = 0;
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (l[k] > l[top]) top = k;
  T q0 = V[0][0], q1 = V[1][0], q2 = V[2][0], q3 = V[3][0];
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (k == top) { q0 = V[0][k]; q1 = V[1][k]; q2 = V[2][k]; q3 = V[3][k]; }
  // descending order of the eigenvalues (4-element sorting network)
  T s0 = l[0], s1 = l[1], s2 = l[2], s3 = l[3], tmp;
#define VD_CSWAP(a, b) if (a < b) { tmp = a; a = b; b = tmp; }
  VD_CSWAP(s0, s1) VD_CSWAP(s2, s3) VD_CSWAP(s0, s2) VD_CSWAP(s1, s3) VD_CSWAP(s1, s2)
#undef VD_CSWAP
  out.sigma1 = T(0.5) * (s0 + s1);
  out.sigma2 = T(0.5) * (s0 + s2);
  out.gap = s0 - s1;
  const T nq = T(1) / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const T w = q0 * nq, x = q1 * nq, y = q2 * nq, z = q3 * nq;
  out.R[0] = w * w + x * x - y * y - z * z;
  out.R[1] = T(2) * (x * y - w * z);
  out.R[2] = T(2) * (x * z + w * y);
  out.R[3] = T(2) * (x * y + w * z);
  out.R[4] = w * w - x * x + y * y - z * z;
  out.R[5] = T(2) * (y * z - w * x);
  out.R[6] = T(2) * (x * z - w * y);
  out.R[7] = T(2) * (y * z + w * x);
  out.R[8] = w * w - x * x - y * y + z * z;
}

// Rank(M) <= 1 (sigma2 <= 1e-12 sigma1): the fit is not unique.
constexpr double kDegenerateRatio = 1e-12;
// A float32 fit is redone in float64 when the eigen-gap is below this
// fraction of sigma1 (its angle error grows like eps * |N| / gap).
constexpr float kRefitRatio = 3e-2f;

// Result codes of fit_or_keep.
enum FitCode { kFitOk = 0, kFitFp64 = 1, kFitKeep = 2 };

// Fit R from M; precision T, with the float64 refit / keep rules.  R_prev is
// kept when the fit is degenerate.
template <typename T>
__device__ __forceinline__ int fit_or_keep(const T (&M)[9], const T (&R_prev)[9], T (&R)[9]);

template <>
__device__ __forceinline__ int fit_or_keep<double>(const double (&M)[9], const double (&R_prev)[9],
                                                   double (&R)[9]) {
  Fit<double> f;
  fit_rotation<double, 10>(M, f);
  if (!(f.sigma2 > kDegenerateRatio * f.sigma1)) {
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = R_prev[k];
    return kFitKeep;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = f.R[k];
  return kFitOk;
}

template <>
__device__ __forceinline__ int fit_or_keep<float>(const float (&M)[9], const float (&R_prev)[9],
                                                  float (&R)[9]) {
  Fit<float> f;
  fit_rotation<float, 6>(M, f);
  if (f.gap > kRefitRatio * f.sigma1 && f.sigma1 > 0.0f) {
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = f.R[k];
    return kFitOk;
  }
  double Md[9], Rp[9], Rd[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) { Md[k] = M[k]; Rp[k] = R_prev[k]; }
  const int code = fit_or_keep<double>(Md, Rp, Rd);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (float)Rd[k];
  return code == kFitKeep ? kFitKeep : kFitFp64;
}

}  // namespace vd
