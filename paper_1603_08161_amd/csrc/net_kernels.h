// Device-side argument blocks of the warm-start network kernels (net.hip)
// and the feature launcher used by the lattice handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "vd_kernels.h"

namespace vd {
namespace net {

constexpr int kNumLayers = 11;

// How a convolution reads its source along each axis at output coordinate o
// and tap t (0..2):
enum {
  kGatherPlain = 0,        // stride * o + t - 1
  kGatherUp = 1,           // nearest x2 up-sampled source: (o + t - 1) / 2
  kGatherTransposed2 = 2,  // input gradient of a stride-2 layer: (o + t - 1) / 2 if even
};

// One convolution launch (forward, or backward data with packed transposed
// weights).  Tensors are channels-last bfloat16 bits, [batch][d][h][w][C].
struct ConvArgs {
  const uint16_t* a;  // first source (channels [0, ca) of the reduction)
  const uint16_t* b;  // second source of a concatenation, or nullptr
  int ca, cb;         // channels of a and b (multiples of 8)
  int cin, lcin;      // ca + cb (a power of two) and its log2
  int ktot, nchunk;   // 27 * cin and ceil(ktot / 32)
  int mode, stride;
  int sd, sh, sw;     // source grid
  int od, oh, ow;     // output grid
  int batch;
  int cout, nb;       // output channels and 16-channel blocks (nb * 16 >= cout)
  const uint4* w;     // packed weights [nchunk][nb][64 lanes][8 bf16]
  const float* bias;  // nullptr or [cout]
  int relu;
  // epilogue: channels [0, c0) -> dst0 ([M][c0]), [c0, c0 + c1) -> dst1
  // ([M][c1]); v = acc + bias + add, relu, then zeroed where mask <= 0
  uint16_t* dst0;
  int c0;
  const uint16_t* mask0;
  const uint16_t* add0;
  uint16_t* dst1;
  int c1;
  const uint16_t* mask1;
  const uint16_t* add1;
  float* out_f32;  // if set: float32 output [batch][cout][d*h*w] instead
};

// Weight-gradient launch: the forward geometry (ConvArgs) plus the output
// gradient and the partial-sum buffer.
struct WgradArgs {
  const uint16_t* dy;  // [M][cdy] gradient w.r.t. the layer's pre-activation
  int cdy;             // cout rounded up to 8
  int mpad, npad;      // partial tile: rows 27 cin + 1 rounded to 64, columns
  int64_t vox_per_chunk;
  float* partial;      // [chunks][mpad][npad]
};

// Features of vd_net.h from a lattice level: `scratch` holds 2 * max(C, 1)
// floats, x receives [N][8] bfloat16 bits.
template <typename T>
hipError_t launch_features(const LevelView<T>& L, const RowView<T>& R, const float* prev2,
                           float* scratch, uint16_t* x, hipStream_t s);

}  // namespace net
}  // namespace vd

#define VD_NET_CHECK(expr)        \
  do {                            \
    const int rc_ = (expr);       \
    if (rc_ != VD_OK) return rc_; \
  } while (0)
