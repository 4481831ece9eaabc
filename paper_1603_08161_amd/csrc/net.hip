// Learned warm start: the 3-D convolutional encoder-decoder of vd_net.h on
// the gfx950 matrix cores, its training (loss, backward, Adam) and the input
// feature build from a lattice's constraint rows.
//
// Every convolution is an implicit GEMM on channels-last bfloat16 tensors:
// rows are output voxels, columns output channels, and the reduction index
// k = tap * c_in + channel runs over the 27 taps and the input channels.  A
// wavefront issues v_mfma_f32_16x16x32_bf16 on 16-voxel x 16-channel tiles:
// each lane gathers 8 consecutive k of one voxel (8 channels of one tap, a
// single 16-byte load, since every channel count is a multiple of 8) and the
// matching 8 k of one output channel from the pre-packed weights.  The same
// kernel runs the backward data pass (flipped, transposed weights; a stride-2
// layer reads its output gradient at (o + tap - 1) / 2 where that is even).
// Weight gradients are a split-K GEMM over voxels with both operands staged
// transposed in LDS, followed by a fixed-order reduction of the partials.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/vd_net.h"
#include "net_kernels.h"
#include "vd_device.h"

namespace vd {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf2f(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

__device__ inline bool bf_pos(uint16_t b) { return !(b & 0x8000u) && (b & 0x7fffu); }

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Source coordinate of output coordinate o at tap t along one axis; false
// where the tap falls into the zero padding.
__device__ inline bool src_coord(int mode, int stride, int o, int t, int n_src, int n_out,
                                 int& q) {
  if (mode == kGatherPlain) {
    q = stride * o + t - 1;
    return q >= 0 && q < n_src;
  }
  q = o + t - 1;
  if (mode == kGatherUp) {
    const bool ok = q >= 0 && q < n_out;
    q >>= 1;
    return ok;
  }
  // kGatherTransposed2: input gradient of a stride-2 convolution
  const bool ok = q >= 0 && !(q & 1) && (q >> 1) < n_src;
  q >>= 1;
  return ok;
}

// 8 consecutive k (one tap, 8 channels) of output voxel (b, z, y, x).
__device__ inline uint4 gather8(const ConvArgs& A, int b, int z, int y, int x, int k0) {
  uint4 zero = {0u, 0u, 0u, 0u};
  if (k0 >= A.ktot) return zero;
  const int t = k0 >> A.lcin;
  int c = k0 & (A.cin - 1);
  const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
  int qz, qy, qx;
  if (!src_coord(A.mode, A.stride, z, tz, A.sd, A.od, qz)) return zero;
  if (!src_coord(A.mode, A.stride, y, ty, A.sh, A.oh, qy)) return zero;
  if (!src_coord(A.mode, A.stride, x, tx, A.sw, A.ow, qx)) return zero;
  const uint16_t* base = A.a;
  int C = A.ca;
  if (c >= A.ca) {
    base = A.b;
    C = A.cb;
    c -= A.ca;
  }
  const size_t v = (((size_t)b * A.sd + qz) * A.sh + qy) * A.sw + qx;
  return *reinterpret_cast<const uint4*>(base + v * C + c);
}

// ---------------------------------------------------------------------------
// convolution (forward and backward data)
// ---------------------------------------------------------------------------

// Epilogue of a 16 x (16 NB) tile pair: bias, skip addend, ReLU / ReLU mask,
// bfloat16 stores split over the concatenated outputs, or float32 output.
template <int MB, int NB>
__device__ __forceinline__ void conv_epilogue(const ConvArgs& A, const f32x4 (&acc)[MB][NB],
                                              int64_t mbase, int lane) {
  const int64_t M = (int64_t)A.batch * A.od * A.oh * A.ow;
  // result tile: lane holds rows 4*(lane/16) + r, column lane % 16
#pragma unroll
  for (int i = 0; i < MB; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = mbase + i * 16 + 4 * (lane >> 4) + r;
      if (m >= M) continue;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int co = j * 16 + (lane & 15);
        float v = acc[i][j][r];
        if (A.out_f32) {
          if (co < A.cout) {
            if (A.bias) v += A.bias[co];
            const int64_t npb = (int64_t)A.od * A.oh * A.ow;
            const int64_t b = m / npb, n = m - b * npb;
            A.out_f32[(b * A.cout + co) * npb + n] = v;
          }
          continue;
        }
        if (co < A.c0) {
          const size_t e = (size_t)m * A.c0 + co;
          if (A.bias) v += A.bias[co];
          if (A.add0) v += bf2f(A.add0[e]);
          if (A.relu) v = fmaxf(v, 0.f);
          if (A.mask0 && !bf_pos(A.mask0[e])) v = 0.f;
          A.dst0[e] = f2bf(v);
        } else if (co < A.c0 + A.c1) {
          const size_t e = (size_t)m * A.c1 + (co - A.c0);
          if (A.bias) v += A.bias[co];
          if (A.add1) v += bf2f(A.add1[e]);
          if (A.relu) v = fmaxf(v, 0.f);
          if (A.mask1 && !bf_pos(A.mask1[e])) v = 0.f;
          A.dst1[e] = f2bf(v);
        }
      }
    }
  }
}

template <int MB, int NB>
__global__ __launch_bounds__(kBlock) void k_conv(ConvArgs A) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t M = (int64_t)A.batch * A.od * A.oh * A.ow;
  const int64_t mbase = ((int64_t)blockIdx.x * (kBlock / kWave) + wave) * (16 * MB);
  if (mbase >= M) return;
  int vb[MB], vz[MB], vy[MB], vx[MB];
  bool vok[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int64_t m = mbase + i * 16 + (lane & 15);
    vok[i] = m < M;
    int64_t r = vok[i] ? m : 0;
    vx[i] = (int)(r % A.ow);
    r /= A.ow;
    vy[i] = (int)(r % A.oh);
    r /= A.oh;
    vz[i] = (int)(r % A.od);
    vb[i] = (int)(r / A.od);
  }
  f32x4 acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  const uint4* __restrict__ W = A.w;
  for (int ch = 0; ch < A.nchunk; ++ch) {
    bf16x8 af[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const uint4 v = vok[i] ? gather8(A, vb[i], vz[i], vy[i], vx[i], ch * 32 + kq)
                             : uint4{0u, 0u, 0u, 0u};
      af[i] = as_bf16x8(v);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bf16x8 bw = as_bf16x8(W[((size_t)ch * NB + j) * kWave + lane]);
#pragma unroll
      for (int i = 0; i < MB; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bw, acc[i][j], 0, 0, 0);
    }
  }
  conv_epilogue<MB, NB>(A, acc, mbase, lane);
}

// Stride-1 convolutions whose workgroup block (64 MB voxels: 4 waves of MB
// 16-voxel tiles) is R = 64 MB / ow whole rows of one (batch, z) plane: the
// block's input (3 planes x (R + 2) rows x
// (ow + 2) voxels x cin channels, zero outside the grid) is staged in LDS once,
// and the 27 taps of every output voxel read it there instead of gathering
// from global memory.  The fragments and the matrix ops, in their order, are
// those of k_conv, so the results are the same bits.
template <int MB, int NB>
__global__ __launch_bounds__(kBlock) void k_conv_lds(ConvArgs A) {
  constexpr int kConvBlockVox = (kBlock / kWave) * 16 * MB;
  extern __shared__ uint4 s_in[];  // [voxel][cin / 8]
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int ow = A.ow, R = kConvBlockVox / ow, W2 = ow + 2, H2 = R + 2;
  const int cg = A.cin >> 3;  // 16-byte channel groups per voxel
  const int64_t blk0 = (int64_t)blockIdx.x * kConvBlockVox;
  int64_t r = blk0 / ow;
  const int y0 = (int)(r % A.oh);
  r /= A.oh;
  const int z = (int)(r % A.od), b = (int)(r / A.od);
  const int nq = 3 * H2 * W2 * cg;
  for (int q = threadIdx.x; q < nq; q += kBlock) {
    const int v = q / cg, g = q - v * cg;
    const int lx = v % W2, ly = (v / W2) % H2, lz = v / (W2 * H2);
    const int sz = z + lz - 1, sy = y0 + ly - 1, sx = lx - 1;
    uint4 val = {0u, 0u, 0u, 0u};
    if (sz >= 0 && sz < A.sd && sy >= 0 && sy < A.sh && sx >= 0 && sx < A.sw) {
      int c = g * 8;
      const uint16_t* base = A.a;
      int C = A.ca;
      if (c >= A.ca) {
        base = A.b;
        C = A.cb;
        c -= A.ca;
      }
      const size_t sv = (((size_t)b * A.sd + sz) * A.sh + sy) * A.sw + sx;
      val = *reinterpret_cast<const uint4*>(base + sv * C + c);
    }
    s_in[q] = val;
  }
  __syncthreads();
  const int64_t mbase = blk0 + wave * (16 * MB);
  int vy[MB], vx[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int ml = wave * (16 * MB) + i * 16 + (lane & 15);
    vy[i] = ml / ow;
    vx[i] = ml - vy[i] * ow;
  }
  f32x4 acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  const uint4* __restrict__ W = A.w;
  for (int ch = 0; ch < A.nchunk; ++ch) {
    const int k0 = ch * 32 + kq;
    const bool kin = k0 < A.ktot;
    const int t = kin ? (k0 >> A.lcin) : 0, g = (k0 & (A.cin - 1)) >> 3;
    const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
    bf16x8 af[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const uint4 v = kin ? s_in[((tz * H2 + vy[i] + ty) * W2 + vx[i] + tx) * cg + g]
                          : uint4{0u, 0u, 0u, 0u};
      af[i] = as_bf16x8(v);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bf16x8 bw = as_bf16x8(W[((size_t)ch * NB + j) * kWave + lane]);
#pragma unroll
      for (int i = 0; i < MB; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bw, acc[i][j], 0, 0, 0);
    }
  }
  conv_epilogue<MB, NB>(A, acc, mbase, lane);
}

// LDS bytes k_conv_lds<MB, *> needs for A, or 0 where it does not apply.
inline size_t conv_lds_bytes(const ConvArgs& A, int MB) {
  const int block = (kBlock / kWave) * 16 * MB;
  if (A.mode != kGatherPlain || A.stride != 1 || A.ow <= 0 || block % A.ow != 0) return 0;
  const int R = block / A.ow;
  if (A.oh % R != 0 || A.sd != A.od || A.sh != A.oh || A.sw != A.ow) return 0;
  const size_t bytes = (size_t)3 * (R + 2) * (A.ow + 2) * (A.cin / 8) * 16;
  return bytes <= 65536 ? bytes : 0;
}

// ---------------------------------------------------------------------------
// weight gradients: dW[k][co] = sum_v X[v][k] dY[v][co], plus the bias row
// k = 27 c_in (X = 1).  Workgroup (mtile, chunk) sums the voxels of its chunk
// for 64 rows k and all columns; partials [chunk][mpad][npad].
// ---------------------------------------------------------------------------

constexpr int kWgVox = 32;          // voxels per LDS stage (one MFMA K step)
constexpr int kWgPitch = kWgVox + 8;  // bf16 per LDS row (80 bytes, 16-aligned)

template <int NB>
__global__ __launch_bounds__(kBlock) void k_wgrad(ConvArgs A, WgradArgs G) {
  __shared__ __attribute__((aligned(16))) uint16_t xt[64 * kWgPitch];
  __shared__ __attribute__((aligned(16))) uint16_t gt[64 * kWgPitch];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int mtile = blockIdx.x, chunk = blockIdx.y;
  const int64_t M = (int64_t)A.batch * A.od * A.oh * A.ow;
  const int64_t v_begin = (int64_t)chunk * G.vox_per_chunk;
  int64_t v_end = v_begin + G.vox_per_chunk;
  if (v_end > M) v_end = M;
  f32x4 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int sv = threadIdx.x & (kWgVox - 1);  // staging: voxel within the stage
  const int sg = threadIdx.x / kWgVox;        // staging: group of 8 rows / columns
  const int row0 = mtile * 64 + 8 * sg;
  for (int64_t v0 = v_begin; v0 < v_end; v0 += kWgVox) {
    const int64_t m = v0 + sv;
    uint4 xv = {0u, 0u, 0u, 0u}, gv = {0u, 0u, 0u, 0u};
    if (m < v_end) {
      int64_t r = m;
      const int x = (int)(r % A.ow);
      r /= A.ow;
      const int y = (int)(r % A.oh);
      r /= A.oh;
      const int z = (int)(r % A.od);
      const int b = (int)(r / A.od);
      if (row0 < A.ktot)
        xv = gather8(A, b, z, y, x, row0);
      else if (row0 == A.ktot)
        xv.x = 0x3f80u;  // bfloat16 1.0 in element 0: the bias row
      if (8 * sg < G.cdy) gv = *reinterpret_cast<const uint4*>(G.dy + (size_t)m * G.cdy + 8 * sg);
    }
    const uint16_t* xe = reinterpret_cast<const uint16_t*>(&xv);
    const uint16_t* ge = reinterpret_cast<const uint16_t*>(&gv);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      xt[(8 * sg + e) * kWgPitch + sv] = xe[e];
      gt[(8 * sg + e) * kWgPitch + sv] = ge[e];
    }
    __syncthreads();
    const bf16x8 af =
        as_bf16x8(*reinterpret_cast<const uint4*>(&xt[(wave * 16 + (lane & 15)) * kWgPitch +
                                                       8 * (lane >> 4)]));
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bf16x8 bf = as_bf16x8(
          *reinterpret_cast<const uint4*>(&gt[(j * 16 + (lane & 15)) * kWgPitch + 8 * (lane >> 4)]));
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* out = G.partial + (size_t)chunk * G.mpad * G.npad;
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mtile * 64 + wave * 16 + 4 * (lane >> 4) + r;
      out[(size_t)row * G.npad + j * 16 + (lane & 15)] = acc[j][r];
    }
}

// grad[off + p] = sum over chunks (fixed order) of the partial at (row, co).
__global__ __launch_bounds__(kBlock) void k_wgrad_reduce(const float* __restrict__ partial,
                                                         int nchunks, int mpad, int npad,
                                                         int cin, int cout, float* grad) {
  const int nw = cout * cin * 27;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= nw + cout) return;
  int row, co;
  if (p < nw) {
    co = p / (cin * 27);
    const int rem = p - co * cin * 27;
    const int ci = rem / 27, t = rem - ci * 27;
    row = t * cin + ci;
  } else {
    co = p - nw;
    row = 27 * cin;
  }
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += partial[((size_t)c * mpad + row) * npad + co];
  grad[p] = s;
}

// ---------------------------------------------------------------------------
// weight packing: float32 master -> MFMA operand order [chunk][nb][lane][8]
// ---------------------------------------------------------------------------

// Forward: k = t * cin + ci, column co; W[co][ci][t].
__global__ __launch_bounds__(kBlock) void k_pack_fwd(const float* __restrict__ W, int cin, int cout,
                                                     int nchunk, int nb, uint16_t* out) {
  const int total = nchunk * nb * kWave * 8;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const int e = i & 7, lane = (i >> 3) & (kWave - 1);
  const int rest = i / (8 * kWave);
  const int j = rest % nb, ch = rest / nb;
  const int k = ch * 32 + 8 * (lane >> 4) + e;
  const int co = j * 16 + (lane & 15);
  float v = 0.f;
  if (k < 27 * cin && co < cout) {
    const int t = k / cin, ci = k - t * cin;
    v = W[((size_t)co * cin + ci) * 27 + t];
  }
  out[i] = f2bf(v);
}

// Backward data: a convolution of the output gradient (cdy channels, cout of
// them real) producing the cin input channels, taps flipped: W[co][ci][26 - t].
__global__ __launch_bounds__(kBlock) void k_pack_dgrad(const float* __restrict__ W, int cin,
                                                       int cout, int cdy, int nchunk, int nb,
                                                       uint16_t* out) {
  const int total = nchunk * nb * kWave * 8;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const int e = i & 7, lane = (i >> 3) & (kWave - 1);
  const int rest = i / (8 * kWave);
  const int j = rest % nb, ch = rest / nb;
  const int k = ch * 32 + 8 * (lane >> 4) + e;
  const int n = j * 16 + (lane & 15);
  float v = 0.f;
  if (k < 27 * cdy && n < cin) {
    const int t = k / cdy, co = k - t * cdy;
    if (co < cout) v = W[((size_t)co * cin + n) * 27 + (26 - t)];
  }
  out[i] = f2bf(v);
}

// ---------------------------------------------------------------------------
// up-sampling backward, loss, Adam
// ---------------------------------------------------------------------------

// g[w][c] = (src[w][c] > 0) * sum of dup over the fine voxels v with v/2 = w.
__global__ __launch_bounds__(kBlock) void k_upsum(const uint16_t* __restrict__ dup, int fd, int fh,
                                                  int fw, const uint16_t* __restrict__ src, int cd,
                                                  int chh, int cw, int C, int batch, uint16_t* g) {
  const int64_t total = (int64_t)batch * cd * chh * cw * C;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % C);
  int64_t r = i / C;
  const int x = (int)(r % cw);
  r /= cw;
  const int y = (int)(r % chh);
  r /= chh;
  const int z = (int)(r % cd);
  const int b = (int)(r / cd);
  float s = 0.f;
  for (int dz = 0; dz < 2; ++dz) {
    const int fz = 2 * z + dz;
    if (fz >= fd) continue;
    for (int dy = 0; dy < 2; ++dy) {
      const int fy = 2 * y + dy;
      if (fy >= fh) continue;
      for (int dx = 0; dx < 2; ++dx) {
        const int fx = 2 * x + dx;
        if (fx >= fw) continue;
        s += bf2f(dup[((((size_t)b * fd + fz) * fh + fy) * fw + fx) * C + c]);
      }
    }
  }
  g[i] = bf_pos(src[i]) ? f2bf(s) : (uint16_t)0;
}

// dout[m][0..7] = 2 (out - target) / M for the 3 real channels, 0 otherwise;
// block partials of sum (out - target)^2.
__global__ __launch_bounds__(kBlock) void k_mse(const float* __restrict__ out,
                                                const float* __restrict__ target, int64_t npb,
                                                int batch, uint16_t* dout, double* part) {
  const int64_t M = npb * batch;
  const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v[1] = {0.0};
  if (m < M) {
    const int64_t b = m / npb, n = m - b * npb;
    uint4 w = {0u, 0u, 0u, 0u};
    uint16_t* we = reinterpret_cast<uint16_t*>(&w);
    const float scale = (float)(2.0 / (double)M);
    for (int c = 0; c < 3; ++c) {
      const size_t e = (size_t)(b * 3 + c) * npb + n;
      const float d = out[e] - target[e];
      v[0] += (double)d * d;
      we[c] = f2bf(scale * d);
    }
    *reinterpret_cast<uint4*>(dout + (size_t)m * 8) = w;
  }
  write_block_partials<1>(v, part, 0);
}

__global__ void k_mse_finalize(const double* part, int n, double inv_m, double* loss) {
  const double s = sum_partials(part, n);
  if (threadIdx.x == 0) *loss = s * inv_m;
}

// One Adam step.  ob1 = 1 - beta1 and ob2 = 1 - beta2 arrive rounded from
// their float64 values: 1.f - 0.999f would lose four digits to cancellation
// (a 1.3e-5 relative error in every second-moment update).
__global__ __launch_bounds__(kBlock) void k_adam(float* p, const float* __restrict__ g, float* m1,
                                                 float* m2, int64_t n, float lr, float b1,
                                                 float ob1, float b2, float ob2, float eps,
                                                 float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + ob1 * gi;
  const float b = b2 * m2[i] + ob2 * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ __launch_bounds__(kBlock) void k_check_finite_f(const float* v, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && !(fabsf(v[i]) <= 3.0e38f)) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// features (channels of vd_net.h) from a lattice's finest level
// ---------------------------------------------------------------------------

// Per dense row: sqrt(w) * (w-weighted residual) pieces: a = |sn| * r',
// b = |sn|^2 with r' = sn . sum_k alpha_k d_k - rho.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_row_residual(LevelView<T> L, int rows, int n_dense,
                                                         float* ra, float* rb) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_dense) return;
  const int cell = L.row_cell[i];
  const int cnx = L.nx - 1, cny = L.ny - 1;
  const int cx = cell % cnx, cy = (cell / cnx) % cny, cz = cell / (cnx * cny);
  const T f[3] = {L.row_f[i], L.row_f[(size_t)rows + i], L.row_f[2 * (size_t)rows + i]};
  const T sn[3] = {L.row_sn[i], L.row_sn[(size_t)rows + i], L.row_sn[2 * (size_t)rows + i]};
  T s[3] = {0, 0, 0};
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
    const T a = (dx ? f[0] : 1 - f[0]) * (dy ? f[1] : 1 - f[1]) * (dz ? f[2] : 1 - f[2]);
    const size_t node = (size_t)(cx + dx) + L.nx * ((size_t)(cy + dy) + (size_t)L.ny * (cz + dz));
    for (int c = 0; c < 3; ++c) s[c] += a * L.d[(size_t)c * L.N + node];
  }
  const T r = sn[0] * s[0] + sn[1] * s[1] + sn[2] * s[2] - L.row_rho[i];
  const T w2 = sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2];
  ra[i] = (float)(sqrt(w2) * r);
  rb[i] = (float)w2;
}

// One thread per node: gathers the rows of the (up to) 8 cells around it in
// cell order, then the rows of each cell in sorted order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_features(LevelView<T> L, RowView<T> R,
                                                     const float* __restrict__ ra,
                                                     const float* __restrict__ rb,
                                                     const float* __restrict__ prev2, int n_dense,
                                                     uint16_t* x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
  const int cnx = nx - 1, cny = ny - 1, cnz = nz - 1;
  const int rows = R.rows;
  double num = 0.0, den = 0.0;
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;  // corner of node i in the cell
    const int cx = ix - dx, cy = iy - dy, cz = iz - dz;
    if (cx < 0 || cy < 0 || cz < 0 || cx >= cnx || cy >= cny || cz >= cnz) continue;
    const int a = L.cell_map[cx + cnx * (cy + cny * cz)];
    if (a < 0) continue;
    for (int s = R.seg_start[a]; s < R.seg_start[a + 1]; ++s) {
      const int row = R.sorted[s];
      if (row >= n_dense) continue;
      const T fx = R.f[row], fy = R.f[(size_t)rows + row], fz = R.f[2 * (size_t)rows + row];
      const double al = (double)((dx ? fx : 1 - fx) * (dy ? fy : 1 - fy) * (dz ? fz : 1 - fz));
      num += al * ra[row];
      den += al * rb[row];
    }
  }
  const double inv_h = 1.0 / (double)L.h;
  float ch[8];
  for (int c = 0; c < 3; ++c) {
    const double d1 = (double)L.d[(size_t)c * L.N + i];
    ch[c] = (float)(d1 * inv_h);
    ch[3 + c] = prev2 ? (float)((d1 - (double)prev2[(size_t)c * L.N + i]) * inv_h) : 0.f;
  }
  ch[6] = den > 0.0 ? (float)(num / den * inv_h) : 0.f;
  ch[7] = den > 0.0 ? 1.f : 0.f;
  uint4 w;
  uint16_t* we = reinterpret_cast<uint16_t*>(&w);
  for (int c = 0; c < 8; ++c) we[c] = f2bf(ch[c]);
  *reinterpret_cast<uint4*>(x + (size_t)i * 8) = w;
}

template <typename T>
hipError_t launch_features(const LevelView<T>& L, const RowView<T>& R, const float* prev2,
                           float* scratch, uint16_t* x, hipStream_t s) {
  float* ra = scratch;
  float* rb = scratch + (R.n_dense > 0 ? R.n_dense : 1);
  if (R.n_dense > 0)
    k_row_residual<T><<<(R.n_dense + kBlock - 1) / kBlock, kBlock, 0, s>>>(L, R.rows, R.n_dense,
                                                                          ra, rb);
  k_features<T><<<(L.N + kBlock - 1) / kBlock, kBlock, 0, s>>>(L, R, ra, rb, prev2, R.n_dense, x);
  return hipGetLastError();
}

template hipError_t launch_features<float>(const LevelView<float>&, const RowView<float>&,
                                           const float*, float*, uint16_t*, hipStream_t);
template hipError_t launch_features<double>(const LevelView<double>&, const RowView<double>&,
                                            const float*, float*, uint16_t*, hipStream_t);

// ---------------------------------------------------------------------------
// host side: the network handle
// ---------------------------------------------------------------------------

namespace {

struct LayerDef {
  int ca, cb, cout, stride, up, relu;
};

// The 11 layers of vd_net.h in parameter order.
constexpr LayerDef kLayers[kNumLayers] = {
    {8, 0, 16, 1, 0, 1},   {16, 0, 16, 1, 0, 1},  {16, 0, 32, 2, 0, 1}, {32, 0, 32, 1, 0, 1},
    {32, 0, 64, 2, 0, 1},  {64, 0, 64, 1, 0, 1},  {64, 0, 32, 1, 1, 1}, {32, 32, 32, 1, 0, 1},
    {32, 0, 16, 1, 1, 1},  {16, 16, 16, 1, 0, 1}, {16, 0, 3, 1, 0, 0}};
enum { E0A, E0, E1A, E1, E2A, E2, U1, D1, U0, D0, HEAD };

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
int round_up(int v, int m) { return (v + m - 1) / m * m; }
int64_t layer_params(const LayerDef& d) { return (int64_t)d.cout * (d.ca + d.cb) * 27 + d.cout; }

struct Dims {
  int d, h, w;
  int64_t n() const { return (int64_t)d * h * w; }
};

}  // namespace

class Net {
 public:
  Net(int nx, int ny, int nz, int max_batch, hipStream_t s)
      : max_batch_(max_batch), stream_(s) {
    dims_[0] = Dims{nz, ny, nx};
    dims_[1] = Dims{(nz + 1) / 2, (ny + 1) / 2, (nx + 1) / 2};
    dims_[2] = Dims{(dims_[1].d + 1) / 2, (dims_[1].h + 1) / 2, (dims_[1].w + 1) / 2};
  }
  ~Net() {
    for (void* p : ptrs_) (void)hipFree(p);
  }

  static int64_t param_count() {
    int64_t n = 0;
    for (const LayerDef& d : kLayers) n += layer_params(d);
    return n;
  }

  int init() {
    const int64_t P = param_count();
    int64_t off = 0;
    for (int l = 0; l < kNumLayers; ++l) {
      off_[l] = off;
      off += layer_params(kLayers[l]);
    }
    VD_NET_CHECK(alloc(&params_, P));
    VD_NET_CHECK(alloc(&grad_, P));
    VD_NET_CHECK(alloc(&m1_, P));
    VD_NET_CHECK(alloc(&m2_, P));
    VD_NET_CHECK(alloc(&flag_, 1));
    if (hipMemsetAsync(params_, 0, P * sizeof(float), stream_) != hipSuccess ||
        hipMemsetAsync(m1_, 0, P * sizeof(float), stream_) != hipSuccess ||
        hipMemsetAsync(m2_, 0, P * sizeof(float), stream_) != hipSuccess)
      return VD_EHIP;
    // packed weights
    for (int l = 0; l < kNumLayers; ++l) {
      const LayerDef& d = kLayers[l];
      const int cin = d.ca + d.cb;
      const int nchunk = (27 * cin + 31) / 32, nb = (d.cout + 15) / 16;
      wf_n_[l] = (size_t)nchunk * nb * kWave * 8;
      VD_NET_CHECK(alloc(&wf_[l], wf_n_[l]));
      const int cdy = round_up(d.cout, 8);
      const int nchunk_b = (27 * cdy + 31) / 32, nb_b = (cin + 15) / 16;
      wb_n_[l] = (size_t)nchunk_b * nb_b * kWave * 8;
      VD_NET_CHECK(alloc(&wb_[l], wb_n_[l]));
    }
    // activations and gradients
    const int B = max_batch_;
    const int64_t n0 = dims_[0].n() * B, n1 = dims_[1].n() * B, n2 = dims_[2].n() * B;
    struct Want {
      uint16_t** p;
      int64_t n;
    } want[] = {
        {&x_, n0 * 8},      {&a_[E0A], n0 * 16}, {&a_[E0], n0 * 16}, {&a_[E1A], n1 * 32},
        {&a_[E1], n1 * 32}, {&a_[E2A], n2 * 64}, {&a_[E2], n2 * 64}, {&a_[U1], n1 * 32},
        {&a_[D1], n1 * 32}, {&a_[U0], n0 * 16},  {&a_[D0], n0 * 16},
        // gradients w.r.t. pre-activations, skip parts and up-sampled inputs
        {&dout_, n0 * 8},   {&g_[D0], n0 * 16},  {&g_[U0], n0 * 16}, {&skip0_, n0 * 16},
        {&dup0_, n0 * 32},  {&g_[D1], n1 * 32},  {&g_[U1], n1 * 32}, {&skip1_, n1 * 32},
        {&dup1_, n1 * 64},  {&g_[E2], n2 * 64},  {&g_[E2A], n2 * 64}, {&g_[E1], n1 * 32},
        {&g_[E1A], n1 * 32}, {&g_[E0], n0 * 16}, {&g_[E0A], n0 * 16},
    };
    for (const Want& w : want) VD_NET_CHECK(alloc(w.p, w.n));
    VD_NET_CHECK(alloc(&out_, n0 * 3));
    VD_NET_CHECK(alloc(&tgt_, n0 * 3));
    mse_blocks_ = (int)((n0 + kBlock - 1) / kBlock);
    VD_NET_CHECK(alloc(&mse_part_, mse_blocks_));
    VD_NET_CHECK(alloc(&loss_, 1));
    // weight-gradient partials: the largest layer's need
    size_t need = 1;
    for (int l = 0; l < kNumLayers; ++l) {
      const WgPlan p = wg_plan(l, B);
      need = std::max(need, (size_t)p.nchunks * p.mpad * p.npad);
    }
    VD_NET_CHECK(alloc(&wpart_, need));
    return pack() == hipSuccess ? VD_OK : VD_EHIP;
  }

  int set_params(const float* p, int mem) {
    const int64_t P = param_count();
    if (mem == VD_MEM_HOST) {
      if (hipMemcpyAsync(params_, p, P * 4, hipMemcpyHostToDevice, stream_) != hipSuccess)
        return VD_EHIP;
    } else {
      if (hipMemcpyAsync(params_, p, P * 4, hipMemcpyDeviceToDevice, stream_) != hipSuccess)
        return VD_EHIP;
    }
    if (hipMemsetAsync(flag_, 0, sizeof(int), stream_) != hipSuccess) return VD_EHIP;
    k_check_finite_f<<<(unsigned)((P + kBlock - 1) / kBlock), kBlock, 0, stream_>>>(params_, P,
                                                                                   flag_);
    int h = 0;
    if (hipMemcpyAsync(&h, flag_, sizeof(int), hipMemcpyDeviceToHost, stream_) != hipSuccess ||
        hipStreamSynchronize(stream_) != hipSuccess)
      return VD_EHIP;
    if (h) return VD_EINVAL;
    if (hipMemsetAsync(m1_, 0, P * 4, stream_) != hipSuccess) return VD_EHIP;
    if (hipMemsetAsync(m2_, 0, P * 4, stream_) != hipSuccess) return VD_EHIP;
    step_ = 0;
    return pack() == hipSuccess ? VD_OK : VD_EHIP;
  }

  int get_params(float* p, int mem) {
    const int64_t P = param_count();
    const hipMemcpyKind kind = mem == VD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(p, params_, P * 4, kind, stream_) != hipSuccess) return VD_EHIP;
    return hipStreamSynchronize(stream_) == hipSuccess ? VD_OK : VD_EHIP;
  }

  // Copies (host) or aliases (device) the input, runs the forward pass.
  int forward(const uint16_t* x, int batch, float* out, int mem) {
    VD_NET_CHECK(check_batch(batch));
    const uint16_t* xd = x;
    if (mem == VD_MEM_HOST) {
      if (hipMemcpyAsync(x_, x, dims_[0].n() * batch * 16, hipMemcpyHostToDevice, stream_) !=
          hipSuccess)
        return VD_EHIP;
      xd = x_;
    }
    float* od = mem == VD_MEM_HOST ? out_ : out;
    if (run_forward(xd, batch, od) != hipSuccess) return VD_EHIP;
    if (mem == VD_MEM_HOST) {
      if (hipMemcpyAsync(out, out_, dims_[0].n() * batch * 12, hipMemcpyDeviceToHost, stream_) !=
          hipSuccess)
        return VD_EHIP;
      if (hipStreamSynchronize(stream_) != hipSuccess) return VD_EHIP;
    }
    return VD_OK;
  }

  // Forward + loss + backward; the gradient lands in grad_.
  int gradients(const uint16_t* x, const float* target, int batch, int mem) {
    VD_NET_CHECK(check_batch(batch));
    const uint16_t* xd = x;
    const float* td = target;
    if (mem == VD_MEM_HOST) {
      const int64_t n = dims_[0].n() * batch;
      if (hipMemcpyAsync(x_, x, n * 16, hipMemcpyHostToDevice, stream_) != hipSuccess ||
          hipMemcpyAsync(tgt_, target, n * 12, hipMemcpyHostToDevice, stream_) != hipSuccess)
        return VD_EHIP;
      xd = x_;
      td = tgt_;
    }
    if (run_forward(xd, batch, out_) != hipSuccess) return VD_EHIP;
    if (run_backward(xd, td, batch) != hipSuccess) return VD_EHIP;
    return VD_OK;
  }

  int copy_grad(float* g, int mem) {
    const int64_t P = param_count();
    const hipMemcpyKind kind = mem == VD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(g, grad_, P * 4, kind, stream_) != hipSuccess) return VD_EHIP;
    return hipStreamSynchronize(stream_) == hipSuccess ? VD_OK : VD_EHIP;
  }

  int read_loss(double* loss) {
    if (hipMemcpyAsync(loss, loss_, sizeof(double), hipMemcpyDeviceToHost, stream_) != hipSuccess)
      return VD_EHIP;
    return hipStreamSynchronize(stream_) == hipSuccess ? VD_OK : VD_EHIP;
  }

  int adam(float lr) {
    ++step_;
    const double b1 = 0.9, b2 = 0.999;
    const float eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(b1, (double)step_));
    const float c2 = (float)(1.0 - std::pow(b2, (double)step_));
    const int64_t P = param_count();
    k_adam<<<(unsigned)((P + kBlock - 1) / kBlock), kBlock, 0, stream_>>>(
        params_, grad_, m1_, m2_, P, lr, (float)b1, (float)(1.0 - b1), (float)b2,
        (float)(1.0 - b2), eps, c1, c2);
    if (hipGetLastError() != hipSuccess) return VD_EHIP;
    return pack() == hipSuccess ? VD_OK : VD_EHIP;
  }

 private:
  struct WgPlan {
    int mpad, npad, nb, mtiles, nchunks;
    int64_t vox_per_chunk;
  };

  template <typename P>
  int alloc(P** p, int64_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max<int64_t>(count, 1) * sizeof(P)) != hipSuccess) {
      (void)hipGetLastError();
      return VD_ENOMEM;
    }
    ptrs_.push_back(q);
    *p = static_cast<P*>(q);
    return VD_OK;
  }

  int check_batch(int batch) const {
    return (batch >= 1 && batch <= max_batch_) ? VD_OK : VD_EINVAL;
  }

  int level_in(int l) const {  // grid level of a layer's input
    static const int lv[kNumLayers] = {0, 0, 0, 1, 1, 2, 2, 1, 1, 0, 0};
    return lv[l];
  }
  int level_out(int l) const {
    static const int lv[kNumLayers] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0};
    return lv[l];
  }

  WgPlan wg_plan(int l, int batch) const {
    const LayerDef& d = kLayers[l];
    const int cin = d.ca + d.cb;
    WgPlan p;
    p.mpad = round_up(27 * cin + 1, 64);
    p.nb = (d.cout + 15) / 16;
    p.npad = 16 * p.nb;
    p.mtiles = p.mpad / 64;
    const int64_t M = dims_[level_out(l)].n() * batch;
    const int64_t steps = (M + kWgVox - 1) / kWgVox;
    int64_t nch = (512 + p.mtiles - 1) / p.mtiles;
    if (nch > steps) nch = steps;
    if (nch < 1) nch = 1;
    p.vox_per_chunk = (steps + nch - 1) / nch * kWgVox;
    p.nchunks = (int)((M + p.vox_per_chunk - 1) / p.vox_per_chunk);
    return p;
  }

  // Geometry and sources of layer l's forward convolution.
  ConvArgs fwd_args(int l, const uint16_t* x, int batch) const {
    const LayerDef& d = kLayers[l];
    ConvArgs A{};
    static const int src_a[kNumLayers] = {-1, E0A, E0, E1A, E1, E2A, E2, U1, D1, U0, D0};
    static const int src_b[kNumLayers] = {-1, -1, -1, -1, -1, -1, -1, E1, -1, E0, -1};
    A.a = src_a[l] < 0 ? x : a_[src_a[l]];
    A.ca = d.ca;
    A.b = src_b[l] < 0 ? nullptr : a_[src_b[l]];
    A.cb = d.cb;
    A.cin = d.ca + d.cb;
    A.lcin = log2i(A.cin);
    A.ktot = 27 * A.cin;
    A.nchunk = (A.ktot + 31) / 32;
    A.mode = d.up ? kGatherUp : kGatherPlain;
    A.stride = d.stride;
    const Dims& si = dims_[level_in(l)];
    const Dims& so = dims_[level_out(l)];
    A.sd = si.d; A.sh = si.h; A.sw = si.w;
    A.od = so.d; A.oh = so.h; A.ow = so.w;
    A.batch = batch;
    A.cout = d.cout;
    A.nb = (d.cout + 15) / 16;
    A.w = reinterpret_cast<const uint4*>(wf_[l]);
    A.bias = params_ + off_[l] + (int64_t)d.cout * A.cin * 27;
    A.relu = d.relu;
    if (l == HEAD) {
      A.out_f32 = nullptr;  // set by the caller
    } else {
      A.dst0 = const_cast<uint16_t*>(a_[l]);
      A.c0 = d.cout;
    }
    return A;
  }

  hipError_t launch_conv(const ConvArgs& A) {
    const int64_t M = (int64_t)A.batch * A.od * A.oh * A.ow;
    const unsigned blocks = (unsigned)((M + 127) / 128);
    // (4 tiles per wave, 256-voxel blocks, measured no faster than k_conv)
    if (const size_t lds = conv_lds_bytes(A, 2)) {
      switch (A.nb) {
        case 1: k_conv_lds<2, 1><<<blocks, kBlock, lds, stream_>>>(A); break;
        case 2: k_conv_lds<2, 2><<<blocks, kBlock, lds, stream_>>>(A); break;
        case 4: k_conv_lds<2, 4><<<blocks, kBlock, lds, stream_>>>(A); break;
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
    switch (A.nb) {
      case 1: k_conv<2, 1><<<blocks, kBlock, 0, stream_>>>(A); break;
      case 2: k_conv<2, 2><<<blocks, kBlock, 0, stream_>>>(A); break;
      case 4: k_conv<2, 4><<<blocks, kBlock, 0, stream_>>>(A); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }

  hipError_t run_forward(const uint16_t* x, int batch, float* out) {
    for (int l = 0; l < kNumLayers; ++l) {
      ConvArgs A = fwd_args(l, x, batch);
      if (l == HEAD) A.out_f32 = out;
      const hipError_t e = launch_conv(A);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // Input gradient of layer l as a convolution of its output gradient gy
  // (cdy channels) over grid `out_level`.
  ConvArgs dgrad_args(int l, const uint16_t* gy, int batch) const {
    const LayerDef& d = kLayers[l];
    ConvArgs A{};
    const int cdy = round_up(d.cout, 8);
    A.a = gy;
    A.ca = cdy;
    A.cin = cdy;
    A.lcin = log2i(cdy);
    A.ktot = 27 * cdy;
    A.nchunk = (A.ktot + 31) / 32;
    A.stride = 1;
    const Dims& gd = dims_[level_out(l)];
    // the data gradient lives on the forward input grid (the up-sampled one
    // for the up layers)
    const Dims& xd = d.up ? dims_[level_out(l)] : dims_[level_in(l)];
    A.mode = d.stride == 2 ? kGatherTransposed2 : kGatherPlain;
    A.sd = gd.d; A.sh = gd.h; A.sw = gd.w;
    A.od = xd.d; A.oh = xd.h; A.ow = xd.w;
    A.batch = batch;
    A.cout = d.ca + d.cb;
    A.nb = (A.cout + 15) / 16;
    A.w = reinterpret_cast<const uint4*>(wb_[l]);
    return A;
  }

  hipError_t launch_wgrad(int l, const uint16_t* x, const uint16_t* gy, int batch) {
    const WgPlan p = wg_plan(l, batch);
    const ConvArgs A = fwd_args(l, x, batch);
    WgradArgs G{};
    G.dy = gy;
    G.cdy = round_up(kLayers[l].cout, 8);
    G.mpad = p.mpad;
    G.npad = p.npad;
    G.vox_per_chunk = p.vox_per_chunk;
    G.partial = wpart_;
    const dim3 grid(p.mtiles, p.nchunks);
    switch (p.nb) {
      case 1: k_wgrad<1><<<grid, kBlock, 0, stream_>>>(A, G); break;
      case 2: k_wgrad<2><<<grid, kBlock, 0, stream_>>>(A, G); break;
      case 4: k_wgrad<4><<<grid, kBlock, 0, stream_>>>(A, G); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const LayerDef& d = kLayers[l];
    const int64_t np = layer_params(d);
    k_wgrad_reduce<<<(unsigned)((np + kBlock - 1) / kBlock), kBlock, 0, stream_>>>(
        wpart_, p.nchunks, p.mpad, p.npad, d.ca + d.cb, d.cout, grad_ + off_[l]);
    return hipGetLastError();
  }

  hipError_t launch_upsum(const uint16_t* dup, int fine_level, const uint16_t* src, int level,
                          int C, int batch, uint16_t* g) {
    const Dims& f = dims_[fine_level];
    const Dims& c = dims_[level];
    const int64_t total = c.n() * batch * C;
    k_upsum<<<(unsigned)((total + kBlock - 1) / kBlock), kBlock, 0, stream_>>>(
        dup, f.d, f.h, f.w, src, c.d, c.h, c.w, C, batch, g);
    return hipGetLastError();
  }

#define VD_NET_HIP(expr)                 \
  do {                                   \
    const hipError_t e_ = (expr);        \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

  hipError_t run_backward(const uint16_t* x, const float* target, int batch) {
    const int64_t npb = dims_[0].n();
    const int64_t M = npb * batch;
    const unsigned mb = (unsigned)((M + kBlock - 1) / kBlock);
    k_mse<<<mb, kBlock, 0, stream_>>>(out_, target, npb, batch, dout_, mse_part_);
    VD_NET_HIP(hipGetLastError());
    k_mse_finalize<<<1, kBlock, 0, stream_>>>(mse_part_, (int)mb, 1.0 / (double)M, loss_);
    VD_NET_HIP(hipGetLastError());
    ConvArgs A;
    // head
    VD_NET_HIP(launch_wgrad(HEAD, x, dout_, batch));
    A = dgrad_args(HEAD, dout_, batch);
    A.dst0 = g_[D0]; A.c0 = 16; A.mask0 = a_[D0];
    VD_NET_HIP(launch_conv(A));
    // d0 = relu(conv([u0, e0]))
    VD_NET_HIP(launch_wgrad(D0, x, g_[D0], batch));
    A = dgrad_args(D0, g_[D0], batch);
    A.dst0 = g_[U0]; A.c0 = 16; A.mask0 = a_[U0];
    A.dst1 = skip0_; A.c1 = 16;
    VD_NET_HIP(launch_conv(A));
    // u0 = relu(conv(up(d1)))
    VD_NET_HIP(launch_wgrad(U0, x, g_[U0], batch));
    A = dgrad_args(U0, g_[U0], batch);
    A.dst0 = dup0_; A.c0 = 32;
    VD_NET_HIP(launch_conv(A));
    VD_NET_HIP(launch_upsum(dup0_, 0, a_[D1], 1, 32, batch, g_[D1]));
    // d1 = relu(conv([u1, e1]))
    VD_NET_HIP(launch_wgrad(D1, x, g_[D1], batch));
    A = dgrad_args(D1, g_[D1], batch);
    A.dst0 = g_[U1]; A.c0 = 32; A.mask0 = a_[U1];
    A.dst1 = skip1_; A.c1 = 32;
    VD_NET_HIP(launch_conv(A));
    // u1 = relu(conv(up(e2)))
    VD_NET_HIP(launch_wgrad(U1, x, g_[U1], batch));
    A = dgrad_args(U1, g_[U1], batch);
    A.dst0 = dup1_; A.c0 = 64;
    VD_NET_HIP(launch_conv(A));
    VD_NET_HIP(launch_upsum(dup1_, 1, a_[E2], 2, 64, batch, g_[E2]));
    // e2
    VD_NET_HIP(launch_wgrad(E2, x, g_[E2], batch));
    A = dgrad_args(E2, g_[E2], batch);
    A.dst0 = g_[E2A]; A.c0 = 64; A.mask0 = a_[E2A];
    VD_NET_HIP(launch_conv(A));
    // e2a (stride 2): its input e1 also feeds d1 through the skip
    VD_NET_HIP(launch_wgrad(E2A, x, g_[E2A], batch));
    A = dgrad_args(E2A, g_[E2A], batch);
    A.dst0 = g_[E1]; A.c0 = 32; A.mask0 = a_[E1]; A.add0 = skip1_;
    VD_NET_HIP(launch_conv(A));
    // e1
    VD_NET_HIP(launch_wgrad(E1, x, g_[E1], batch));
    A = dgrad_args(E1, g_[E1], batch);
    A.dst0 = g_[E1A]; A.c0 = 32; A.mask0 = a_[E1A];
    VD_NET_HIP(launch_conv(A));
    // e1a (stride 2): its input e0 also feeds d0 through the skip
    VD_NET_HIP(launch_wgrad(E1A, x, g_[E1A], batch));
    A = dgrad_args(E1A, g_[E1A], batch);
    A.dst0 = g_[E0]; A.c0 = 16; A.mask0 = a_[E0]; A.add0 = skip0_;
    VD_NET_HIP(launch_conv(A));
    // e0
    VD_NET_HIP(launch_wgrad(E0, x, g_[E0], batch));
    A = dgrad_args(E0, g_[E0], batch);
    A.dst0 = g_[E0A]; A.c0 = 16; A.mask0 = a_[E0A];
    VD_NET_HIP(launch_conv(A));
    // e0a (the input needs no gradient)
    VD_NET_HIP(launch_wgrad(E0A, x, g_[E0A], batch));
    return hipSuccess;
  }

  hipError_t pack() {
    for (int l = 0; l < kNumLayers; ++l) {
      const LayerDef& d = kLayers[l];
      const int cin = d.ca + d.cb;
      const float* W = params_ + off_[l];
      const int nchunk = (27 * cin + 31) / 32, nb = (d.cout + 15) / 16;
      k_pack_fwd<<<(unsigned)((wf_n_[l] + kBlock - 1) / kBlock), kBlock, 0, stream_>>>(
          W, cin, d.cout, nchunk, nb, wf_[l]);
      VD_NET_HIP(hipGetLastError());
      const int cdy = round_up(d.cout, 8);
      const int nchunk_b = (27 * cdy + 31) / 32, nb_b = (cin + 15) / 16;
      k_pack_dgrad<<<(unsigned)((wb_n_[l] + kBlock - 1) / kBlock), kBlock, 0, stream_>>>(
          W, cin, d.cout, cdy, nchunk_b, nb_b, wb_[l]);
      VD_NET_HIP(hipGetLastError());
    }
    return hipSuccess;
  }

  Dims dims_[3];
  int max_batch_;
  hipStream_t stream_;
  std::vector<void*> ptrs_;
  int64_t off_[kNumLayers] = {};
  float *params_ = nullptr, *grad_ = nullptr, *m1_ = nullptr, *m2_ = nullptr;
  int* flag_ = nullptr;
  uint16_t* wf_[kNumLayers] = {};
  uint16_t* wb_[kNumLayers] = {};
  size_t wf_n_[kNumLayers] = {}, wb_n_[kNumLayers] = {};
  uint16_t* x_ = nullptr;
  uint16_t* a_[kNumLayers] = {};
  uint16_t* g_[kNumLayers] = {};
  uint16_t *dout_ = nullptr, *skip0_ = nullptr, *skip1_ = nullptr, *dup0_ = nullptr,
           *dup1_ = nullptr;
  float *out_ = nullptr, *tgt_ = nullptr, *wpart_ = nullptr;
  double *mse_part_ = nullptr, *loss_ = nullptr;
  int mse_blocks_ = 0;
  int64_t step_ = 0;
};

}  // namespace net
}  // namespace vd

struct vd_net {
  vd::net::Net* impl;
};

extern "C" {

int64_t vd_net_param_count(void) { return vd::net::Net::param_count(); }

int vd_net_create(int32_t nx, int32_t ny, int32_t nz, int32_t max_batch, void* stream,
                  vd_net** out) {
  if (!out) return VD_EINVAL;
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1 || max_batch < 1) return VD_EINVAL;
  if ((int64_t)nx * ny * nz * max_batch > (int64_t)1 << 28) return VD_EINVAL;
  vd::net::Net* impl =
      new (std::nothrow) vd::net::Net(nx, ny, nz, max_batch, static_cast<hipStream_t>(stream));
  if (!impl) return VD_ENOMEM;
  const int rc = impl->init();
  if (rc != VD_OK) {
    delete impl;
    return rc;
  }
  vd_net* h = new (std::nothrow) vd_net{impl};
  if (!h) {
    delete impl;
    return VD_ENOMEM;
  }
  *out = h;
  return VD_OK;
}

int vd_net_destroy(vd_net* n) {
  if (!n) return VD_OK;
  delete n->impl;
  delete n;
  return VD_OK;
}

int vd_net_set_params(vd_net* n, const float* params, int32_t mem) {
  if (!n || !params || (mem != VD_MEM_HOST && mem != VD_MEM_DEVICE)) return VD_EINVAL;
  return n->impl->set_params(params, mem);
}

int vd_net_get_params(vd_net* n, float* params, int32_t mem) {
  if (!n || !params || (mem != VD_MEM_HOST && mem != VD_MEM_DEVICE)) return VD_EINVAL;
  return n->impl->get_params(params, mem);
}

int vd_net_forward(vd_net* n, const uint16_t* x, int32_t batch, float* out, int32_t mem) {
  if (!n || !x || !out || (mem != VD_MEM_HOST && mem != VD_MEM_DEVICE)) return VD_EINVAL;
  return n->impl->forward(x, batch, out, mem);
}

int vd_net_gradients(vd_net* n, const uint16_t* x, const float* target, int32_t batch, float* grad,
                     double* loss, int32_t mem) {
  if (!n || !x || !target || !grad || (mem != VD_MEM_HOST && mem != VD_MEM_DEVICE))
    return VD_EINVAL;
  int rc = n->impl->gradients(x, target, batch, mem);
  if (rc != VD_OK) return rc;
  rc = n->impl->copy_grad(grad, mem);
  if (rc != VD_OK) return rc;
  return loss ? n->impl->read_loss(loss) : VD_OK;
}

int vd_net_train_step(vd_net* n, const uint16_t* x, const float* target, int32_t batch, float lr,
                      int32_t mem, double* loss) {
  if (!n || !x || !target || (mem != VD_MEM_HOST && mem != VD_MEM_DEVICE)) return VD_EINVAL;
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return VD_EINVAL;
  int rc = n->impl->gradients(x, target, batch, mem);
  if (rc != VD_OK) return rc;
  if (loss) {
    rc = n->impl->read_loss(loss);
    if (rc != VD_OK) return rc;
  }
  return n->impl->adam(lr);
}

}  // extern "C"
