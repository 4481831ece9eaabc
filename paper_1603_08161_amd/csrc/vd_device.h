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

// Tiles of the stencil kernels: TX x TY x TZ nodes staged in LDS with a
// one-node halo; NT threads, the first OWNERS of which own NPT consecutive
// nodes along z each (with more threads than nodes, the others only stage
// the halo and evaluate data blocks).
template <int TX_, int TY_, int TZ_, int NT_ = kBlock>
struct Tile {
  static constexpr int TX = TX_, TY = TY_, TZ = TZ_, NT = NT_;
  static constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  static constexpr int HALO = HX * HY * HZ;
  static constexpr int ZG = NT / (TX * TY);          // thread layers along z
  static constexpr int NPT = ZG >= TZ ? 1 : TZ / ZG; // nodes per owning thread
  static constexpr int OWNERS = TX * TY * TZ / NPT;  // threads that own nodes
  static constexpr int HPT = (HALO + NT - 1) / NT;   // halo nodes staged per thread
};
// Tile kinds: small (most workgroups, best latency hiding), medium (half the
// block partials and 1.95x instead of 2.34x halo reads), wide (128-byte rows
// along x, 4x fewer block partials, 4 nodes per thread), wide with one node
// per thread (the wide tile on 1024 threads: its halo rows cover about half
// as many cache lines per wave load as the small tile's), and two tall tiles
// on 1024 threads (16 nodes along z: 1.76x / 1.90x halo reads, and an
// observed surface facing the camera crosses fewer of their nodes, which
// bounds the data-block work of the busiest workgroup), and the half-height
// tall tile on 512 threads (two workgroups per CU share a CU's memory
// bandwidth, so a tile heavy in data blocks is paired with an ordinary one),
// and the small tile on 512 threads for the coarse levels, where nearly
// every node carries data blocks: two threads per node, so the workgroup's
// data-block work takes half the rounds.
using TileS = Tile<8, 8, 4>;
using TileM = Tile<8, 8, 8>;
using TileW = Tile<32, 8, 4>;
using TileX = Tile<32, 8, 4, 1024>;
using TileZ = Tile<8, 8, 16, 1024>;
using TileY = Tile<16, 4, 16, 1024>;
using TileH = Tile<16, 4, 8, 512>;
using TileC = Tile<8, 8, 4, 512>;
constexpr int kTileKinds = 8;

// Maps the hardware workgroup id to a logical tile id so that each XCD gets a
// contiguous range of tiles (neighbouring tiles then share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks / kXcds, r = nblocks % kXcds;
  const int xcd = bid % kXcds, slot = bid / kXcds;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

// Global-memory (address space 1) view of a device pointer.  The lattice
// arrays reach the kernels inside structs, where the compiler only sees
// generic pointers and emits flat loads and stores.  The hardware counts a
// flat access on the LDS/scalar-memory counter as well as on the vector-memory
// counter, so every wait for an LDS or scalar-load result would also wait for
// all vector loads in flight.  Global accesses keep the two apart (and take a
// uniform base address in scalar registers).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> glob(T* p) {
  return (gptr<T>)p;
}

// ---------------------------------------------------------------------------
// reductions (float64 sums, fixed order => bitwise deterministic)
// ---------------------------------------------------------------------------

// Value of lane CTRL's DPP source (data-parallel primitive: a lane
// permutation inside rows of 16 lanes, done in the vector ALU without the
// LDS crossbar that general shuffles use).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, 0xf, 0xf,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

__device__ __forceinline__ double lane_double(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (all lanes active), the same bits in every
// lane: within each row of 16 lanes, exchanges with lane ^ 1, lane ^ 2 (quad
// permutations), the mirrored lane of the half-row and of the row -- each
// step adds two partial sums that are the same in every lane that holds them
// (x + y = y + x exactly) -- then the four row sums in fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (lane_double(v, 0) + lane_double(v, 16)) + (lane_double(v, 32) + lane_double(v, 48));
}

// Sum K values over the block; the result is valid in thread 0.
template <int K, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds /* K * NT/kWave */) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * NW + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += lds[k * NW + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Sum of n partials written by the previous kernel, computed by every block
// in the same fixed order (bitwise identical in all blocks).  No block of the
// current kernel writes them, so the kernel boundary alone makes them
// visible: no cross-workgroup fence is needed.
__device__ __forceinline__ double sum_partials(const double* __restrict__ pin, int n) {
  __shared__ double lds[kBlock / kWave];
  __shared__ double total;
  const gptr<const double> __restrict__ p = glob(pin);
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

// Sums of K partial arrays p + k*n (k < K) in one pass (one round of loads),
// identical in every block; result valid in every thread.
template <int K, int NT = kBlock>
__device__ __forceinline__ void sum_partials_k(const double* __restrict__ pin, int n,
                                               double (&out)[K]) {
  constexpr int NW = NT / kWave;
  const gptr<const double> __restrict__ p = glob(pin);
  __shared__ double lds[K * NW];
  __shared__ double total[K];
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < n; b += NT) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += p[(size_t)k * n + b];
  }
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * NW + wid] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += lds[threadIdx.x * NW + w];
    total[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = total[k];
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

// The rotation-fit routines are __host__ __device__ so their logic can also
// be exercised on the CPU.
#define VD_HD __host__ __device__ __forceinline__

// Tangent t = tan(phi) and cosine c of the Jacobi rotation in the (p, q)
// plane that annihilates a_pq, from theta = (a_qq - a_pp) / (2 a_pq) (the
// smaller root, |phi| <= pi / 4).  Returns false when there is nothing to
// rotate.
template <typename T>
VD_HD bool jacobi_tc(T app, T aqq, T apq, T& t, T& c) {
  if (apq == T(0)) return false;
  const T theta = (aqq - app) / (T(2) * apq);
  const T sgn = theta >= T(0) ? T(1) : T(-1);
  t = sgn / (fabs(theta) + sqrt(theta * theta + T(1)));
  c = T(1) / sqrt(t * t + T(1));
  return true;
}
// float32 on the GPU: the hardware reciprocal, square root and reciprocal
// square root (about 1 ulp) replace the correctly rounded sequences.  t and c
// then carry a few ulp of error, the rotation stays orthonormal to float32
// precision, and the quaternion is normalised at the end of the fit anyway.
// |a_pq| below 1e-30 is left alone (it keeps 1 / (2 a_pq) finite); beyond
// |theta| = 1e15, where theta^2 would soon overflow, t = 1 / (2 |theta|),
// the root to float32 precision there.
template <>
VD_HD bool jacobi_tc<float>(float app, float aqq, float apq, float& t, float& c) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (!(fabsf(apq) >= 1e-30f)) return false;
  const float theta = (aqq - app) * __builtin_amdgcn_rcpf(2.0f * apq);
  const float at = fabsf(theta);
  const float ta = at > 1e15f ? 0.5f * __builtin_amdgcn_rcpf(at)
                              : __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(at * at + 1.0f));
  t = theta >= 0.0f ? ta : -ta;
  c = __builtin_amdgcn_rsqf(t * t + 1.0f);
#else
  if (apq == 0.0f) return false;
  const float theta = (aqq - app) / (2.0f * apq);
  const float sgn = theta >= 0.0f ? 1.0f : -1.0f;
  t = sgn / (fabsf(theta) + sqrtf(theta * theta + 1.0f));
  c = 1.0f / sqrtf(t * t + 1.0f);
#endif
  return true;
}

// One cyclic-Jacobi rotation A <- J^T A J, V <- V J in the (p, q) plane of the
// symmetric A (Golub and Van Loan, the symmetric Schur decomposition).  Only
// rows and columns p and q change: a_pp and a_qq move by -/+ t a_pq, a_pq
// becomes exactly 0, and the other entries of the two columns rotate (their
// mirror entries are written too, so A stays exactly symmetric).
template <typename T>
VD_HD void jacobi_rotate(T (&A)[4][4], T (&V)[4][4], int p, int q) {
  T t, c;
  if (!jacobi_tc(A[p][p], A[q][q], A[p][q], t, c)) return;
  const T s = t * c;
  const T tap = t * A[p][q];
  A[p][p] -= tap;
  A[q][q] += tap;
  A[p][q] = T(0);
  A[q][p] = T(0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (r == p || r == q) continue;
    const T arp = A[r][p], arq = A[r][q];
    const T np = c * arp - s * arq, nq = s * arp + c * arq;
    A[r][p] = np;
    A[p][r] = np;
    A[r][q] = nq;
    A[q][r] = nq;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T vkp = V[k][p], vkq = V[k][q];
    V[k][p] = c * vkp - s * vkq;
    V[k][q] = s * vkp + c * vkq;
  }
}

// Unit quaternion (w, x, y, z) of a rotation matrix (Shepperd's method:
// branch on the largest of the trace and the diagonal).  Falls back to the
// identity when R is too far from a rotation to give a finite unit vector.
template <typename T>
VD_HD void rot_to_quat(const T (&R)[9], T (&q)[4]) {
  const T tr = R[0] + R[4] + R[8];
  T w, x, y, z;
  if (tr > R[0] && tr > R[4] && tr > R[8]) {
    const T s = T(2) * sqrt(fmax(tr + T(1), T(0)));
    w = T(0.25) * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const T s = T(2) * sqrt(fmax(T(1) + R[0] - R[4] - R[8], T(0)));
    w = (R[7] - R[5]) / s; x = T(0.25) * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    const T s = T(2) * sqrt(fmax(T(1) + R[4] - R[0] - R[8], T(0)));
    w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = T(0.25) * s; z = (R[5] + R[7]) / s;
  } else {
    const T s = T(2) * sqrt(fmax(T(1) + R[8] - R[0] - R[4], T(0)));
    w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = T(0.25) * s;
  }
  const T n2 = w * w + x * x + y * y + z * z;
  if (!(n2 > T(1e-6) && n2 < T(1e30))) {  // also rejects NaN and inf
    q[0] = T(1); q[1] = T(0); q[2] = T(0); q[3] = T(0);
    return;
  }
  const T inv = T(1) / sqrt(n2);
  q[0] = w * inv; q[1] = x * inv; q[2] = y * inv; q[3] = z * inv;
}

// Horn (1987): with S = M^T (sum source * target^T), the rotation is given by
// the unit quaternion spanning the top eigenvector of the symmetric N below.
// N is first expressed in the basis L(q0) (quaternion left-multiplication by
// the previous rotation's quaternion), where it is nearly diagonal with its
// top eigenvector near e0, so the cyclic Jacobi sweeps converge in one or
// two passes; they stop once the off-diagonal mass is negligible.
template <typename T, int SWEEPS>
VD_HD void fit_rotation(const T (&M)[9], const T (&q0)[4], Fit<T>& out) {
  const T Sxx = M[0], Sxy = M[3], Sxz = M[6];
  const T Syx = M[1], Syy = M[4], Syz = M[7];
  const T Szx = M[2], Szy = M[5], Szz = M[8];
  const T Nm[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
                      {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
                      {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
                      {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
  const T w = q0[0], x = q0[1], y = q0[2], z = q0[3];
  const T Lq[4][4] = {{w, -x, -y, -z}, {x, w, -z, y}, {y, z, w, -x}, {z, -y, x, w}};
  T NL[4][4], A[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      NL[r][c] = Nm[r][0] * Lq[0][c] + Nm[r][1] * Lq[1][c] + Nm[r][2] * Lq[2][c] +
                 Nm[r][3] * Lq[3][c];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      A[r][c] = Lq[0][r] * NL[0][c] + Lq[1][r] * NL[1][c] + Lq[2][r] * NL[2][c] +
                Lq[3][r] * NL[3][c];
  T V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
  const T tol = sizeof(T) == 4 ? T(1e-14) : T(1e-30);
  // fully unrolled: A and V then stay in fixed registers across sweeps (a
  // rolled loop copies a dozen of them per rotation, and the rotation-fit
  // kernel needs 117 instead of 142 VGPRs)
#pragma unroll
  for (int sweep = 0; sweep < SWEEPS; ++sweep) {
    const T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[0][3] * A[0][3] +
                  A[1][2] * A[1][2] + A[1][3] * A[1][3] + A[2][3] * A[2][3];
    const T dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2] + A[3][3] * A[3][3];
    if (off <= tol * dia) break;
    jacobi_rotate(A, V, 0, 1);
    jacobi_rotate(A, V, 0, 2);
    jacobi_rotate(A, V, 0, 3);
    jacobi_rotate(A, V, 1, 2);
    jacobi_rotate(A, V, 1, 3);
    jacobi_rotate(A, V, 2, 3);
  }
  // back to the original basis: eigenvectors of N are L(q0) V
  T W[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      W[r][c] = Lq[r][0] * V[0][c] + Lq[r][1] * V[1][c] + Lq[r][2] * V[2][c] + Lq[r][3] * V[3][c];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) V[r][c] = W[r][c];
  // sort the four eigenvalues (descending) while tracking the top vector
  T l[4] = {A[0][0], A[1][1], A[2][2], A[3][3]};
  int top = 0;
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (l[k] > l[top]) top = k;
  T e0 = V[0][0], e1 = V[1][0], e2 = V[2][0], e3 = V[3][0];
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (k == top) { e0 = V[0][k]; e1 = V[1][k]; e2 = V[2][k]; e3 = V[3][k]; }
  // descending order of the eigenvalues (4-element sorting network)
  T s0 = l[0], s1 = l[1], s2 = l[2], s3 = l[3], tmp;
#define VD_CSWAP(a, b) if (a < b) { tmp = a; a = b; b = tmp; }
  VD_CSWAP(s0, s1) VD_CSWAP(s2, s3) VD_CSWAP(s0, s2) VD_CSWAP(s1, s3) VD_CSWAP(s1, s2)
#undef VD_CSWAP
  out.sigma1 = T(0.5) * (s0 + s1);
  out.sigma2 = T(0.5) * (s0 + s2);
  out.gap = s0 - s1;
  const T nq = T(1) / sqrt(e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3);
  const T qw = e0 * nq, qx = e1 * nq, qy = e2 * nq, qz = e3 * nq;
  out.R[0] = qw * qw + qx * qx - qy * qy - qz * qz;
  out.R[1] = T(2) * (qx * qy - qw * qz);
  out.R[2] = T(2) * (qx * qz + qw * qy);
  out.R[3] = T(2) * (qx * qy + qw * qz);
  out.R[4] = qw * qw - qx * qx + qy * qy - qz * qz;
  out.R[5] = T(2) * (qy * qz - qw * qx);
  out.R[6] = T(2) * (qx * qz - qw * qy);
  out.R[7] = T(2) * (qy * qz + qw * qx);
  out.R[8] = qw * qw - qx * qx - qy * qy + qz * qz;
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
VD_HD int fit_or_keep(const T (&M)[9], const T (&R_prev)[9], T (&R)[9]);

template <>
VD_HD int fit_or_keep<double>(const double (&M)[9], const double (&R_prev)[9],
                                                   double (&R)[9]) {
  Fit<double> f;
  double q0[4];
  rot_to_quat<double>(R_prev, q0);
  fit_rotation<double, 10>(M, q0, f);
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
VD_HD int fit_or_keep<float>(const float (&M)[9], const float (&R_prev)[9],
                                                  float (&R)[9]) {
  Fit<float> f;
  float q0[4];
  rot_to_quat<float>(R_prev, q0);
  fit_rotation<float, 6>(M, q0, f);
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
