// The per-frame solve kernels (Sec. 7): gradient, fused CG iterations,
// rotation fits, energy and level transfers.  Every launch takes a Dispatch:
// one lattice by value, or a device table of lattices that are all at the
// same schedule step (the batched solve), with workgroup g belonging to the
// lattice b for which starts[b] <= g < starts[b + 1].
//
// Unknowns are displacements d = t - t_hat; node vectors are SoA [3][N] in
// x-fastest order (rotations [9][N]).

#include "vd_device.h"
#include "vd_kernels.h"

namespace vd {

namespace {

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ bool in_box(int x, int y, int z, int nx, int ny, int nz) {
  return x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
}

__device__ __forceinline__ size_t rot_at(int row, int col, size_t N, size_t i) {
  return (size_t)(row * 3 + col) * N + i;
}

// The lattice of workgroup g, its local workgroup index and count.
template <typename T>
struct Where {
  LevelView<T> L;
  int b, local, count;
};

// The lattice is the number of b in 1..n-1 with starts[b] <= g (starts is
// non-decreasing): one wave-wide vector load and ballot per 64 lattices
// instead of a binary search's chain of dependent loads.
template <typename T>
__device__ __forceinline__ Where<T> locate(const Dispatch<T>& D, int g) {
  Where<T> w;
  if (D.n == 1) {
    w.L = D.one;
    w.b = 0;
    w.local = g;
    w.count = D.blocks;
    return w;
  }
  const int lane = threadIdx.x & (kWave - 1);
  int lo = 0;
  for (int base = 1; base < D.n; base += kWave) {
    const int idx = base + lane;
    lo += __popcll(__ballot(idx < D.n && glob<const int>(D.starts)[idx] <= g));
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  w.L = D.views[lo];
  w.b = lo;
  w.local = g - D.starts[lo];
  w.count = D.starts[lo + 1] - D.starts[lo];
  return w;
}

// A guarded launch (energy-target mode) returns at entry once the target
// was reached: the flag is uniform, so every workgroup leaves before any
// barrier or store.
template <typename T>
__device__ __forceinline__ bool skipped(const Dispatch<T>& D) {
  return D.stop != nullptr && *D.stop != 0;
}

template <typename T>
__device__ __forceinline__ LevelView<T> view_of(const Dispatch<T>& D, int b) {
  return D.n == 1 ? D.one : D.views[b];
}

template <typename T>
__device__ __forceinline__ int energy_blocks_dev(const LevelView<T>& L) {
  return L.rblocks + (L.N + kBlock - 1) / kBlock;
}

// Block sums of K values written to out[k * stride + local]: wave sums, then
// thread k adds the waves' k-th sums in wave order and stores the result.
template <int K, int NT = kBlock>
__device__ __forceinline__ void write_partials(double (&v)[K], double* out, int stride,
                                               int local) {
  constexpr int NW = NT / kWave;
  __shared__ double lds[K * NW];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * NW + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += lds[threadIdx.x * NW + w];
    glob(out)[(size_t)threadIdx.x * stride + local] = s;
  }
}

}  // namespace

// ===========================================================================
// tiles
// ===========================================================================

int tile_blocks(int kind, int nx, int ny, int nz) {
  auto nb = [&](int tx, int ty, int tz) {
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz);
  };
  switch (kind) {
    case 1: return nb(TileM::TX, TileM::TY, TileM::TZ);
    case 2: return nb(TileW::TX, TileW::TY, TileW::TZ);
    case 3: return nb(TileX::TX, TileX::TY, TileX::TZ);
    case 4: return nb(TileZ::TX, TileZ::TY, TileZ::TZ);
    case 5: return nb(TileY::TX, TileY::TY, TileY::TZ);
    case 6: return nb(TileH::TX, TileH::TY, TileH::TZ);
    case 7: return nb(TileC::TX, TileC::TY, TileC::TZ);
    default: return nb(TileS::TX, TileS::TY, TileS::TZ);
  }
}

int default_tile(int nx, int ny, int nz) { return tile_blocks(1, nx, ny, nz) >= 512 ? 1 : 0; }
int node_blocks(int N) { return blocks_for(N); }
int energy_blocks(int rblocks, int N) { return rblocks + blocks_for(N); }

template <typename TL>
struct TilePos {
  int x0, y0, z0;  // lattice coordinates of LDS index (0,0,0) (tile origin - 1)
  __device__ __forceinline__ TilePos(int nx, int ny, int local) {
    const int ntx = (nx + TL::TX - 1) / TL::TX, nty = (ny + TL::TY - 1) / TL::TY;
    const int tx = local % ntx, ty = (local / ntx) % nty, tz = local / (ntx * nty);
    x0 = tx * TL::TX - 1;
    y0 = ty * TL::TY - 1;
    z0 = tz * TL::TZ - 1;
  }
  // whether this thread owns nodes (tiles with more threads than nodes leave
  // the last threads without; they stage the halo and evaluate data blocks)
  __device__ __forceinline__ static bool owner() {
    return TL::OWNERS == TL::NT || (int)threadIdx.x < TL::OWNERS;
  }
  // LDS index of the k-th node owned by this thread
  __device__ __forceinline__ static int own(int k) {
    const int t = owner() ? (int)threadIdx.x : 0;
    const int lx = t % TL::TX + 1, ly = (t / TL::TX) % TL::TY + 1;
    const int lz = (t / (TL::TX * TL::TY)) * TL::NPT + k + 1;
    return lx + TL::HX * (ly + TL::HY * lz);
  }
};

// ===========================================================================
// the normal-equation stencil (Sec. 7.1): A p = J^T J p
// ===========================================================================
//
// A p at node i = 2 w_r sum_{j in N_i} (p_i - p_j)                (ARAP part)
//               + sum_{delta in {-1,0,1}^3} A27_i[delta] p_{i+delta}  (data part)
//
// One workgroup per tile; the tile plus a one-node halo of p is staged in LDS
// (all 27 stencil neighbours of a tile node are in it; nodes outside the
// lattice hold 0 and have zero blocks).

// ARAP part of A p at own node c (tile-local) / i (global) from the tile's p
// in LDS: 2 w_r times the 6-neighbour Laplacian.  The data part is added by
// the caller (eval_data_nodes).  With the optimised set M (sm: the tile's
// membership in LDS) only the edges inside M count: node c couples to the
// neighbours q in M.
template <typename T, typename TL>
__device__ __forceinline__ void arap_at(const LevelView<T>& L, const T (*sp)[TL::HALO], int c,
                                        int gx, int gy, int gz, T& o0, T& o1, T& o2,
                                        const unsigned char* sm = nullptr) {
  const T p0 = sp[0][c], p1 = sp[1][c], p2 = sp[2][c];
  T l0 = T(0), l1 = T(0), l2 = T(0);
  const int off[3] = {1, TL::HX, TL::HX * TL::HY};
  const int pos[3] = {gx, gy, gz};
  const int lim[3] = {L.nx, L.ny, L.nz};
  if (sm) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        if (sgn < 0 ? pos[ax] == 0 : pos[ax] == lim[ax] - 1) continue;
        const int q = sgn < 0 ? c - off[ax] : c + off[ax];
        if (!sm[q]) continue;
        l0 += p0 - sp[0][q];
        l1 += p1 - sp[1][q];
        l2 += p2 - sp[2][q];
      }
    }
    const T w2 = T(2) * L.wr;
    o0 = w2 * l0;
    o1 = w2 * l1;
    o2 = w2 * l2;
    return;
  }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (pos[ax] > 0) {
      const int q = c - off[ax];
      l0 += p0 - sp[0][q];
      l1 += p1 - sp[1][q];
      l2 += p2 - sp[2][q];
    }
    if (pos[ax] < lim[ax] - 1) {
      const int q = c + off[ax];
      l0 += p0 - sp[0][q];
      l1 += p1 - sp[1][q];
      l2 += p2 - sp[2][q];
    }
  }
  const T w2 = T(2) * L.wr;
  o0 = w2 * l0;
  o1 = w2 * l1;
  o2 = w2 * l2;
}

// ---------------------------------------------------------------------------
// data part of A p, shared by the workgroup (CG iteration and gradient pass)
// ---------------------------------------------------------------------------
//
// Only nodes near the observed surface carry data blocks, and they cluster in
// a few waves.  Evaluated by its owner, a node's 27 blocks are a long chain of
// row loads in one lane while most lanes idle, and the workgroup waits for its
// busiest wave.  Instead every wave lists its own such nodes in LDS (a segment
// per wave, in (k, lane) order) and, once the tile is staged, the workgroup's
// lanes take (node, part) items: per wave and round 21 nodes, lanes 3n, 3n+1
// and 3n+2 evaluating the blocks of dz = -1, 0, +1 of node n from that part of
// the node's row (14 16-byte loads; the row interleaves the three parts'
// chunks, so the three lanes of a node read one contiguous 48-byte span per
// load).  Lane 3n adds the three sums in fixed order and leaves the result in
// LDS for the owner.  A node's sum does not
// depend on which lane or round evaluates it, so the gradient pass and the CG
// iteration give the same bits with every tile shape.

constexpr int kPartsPerNode = 3;
constexpr int kNodesPerWave = kWave / kPartsPerNode;  // 21; lane 63 idles

template <typename T, typename TL>
struct DataShare {
  static constexpr int SEG = kWave * TL::NPT;  // list entries per wave
  static constexpr int NW = TL::NT / kWave;
  int slot[NW * SEG];
  int node[NW * SEG];  // LDS tile index of the node
  int cnt[NW];
  T d[3][NW * SEG];    // data part of A p of list entry e
};

// List the calling wave's own nodes that carry data blocks; rank[k]: entry of
// the thread's k-th node in the wave's segment (-1: none).
template <typename T, typename TL>
__device__ __forceinline__ void list_data_nodes(const int (&slot)[TL::NPT],
                                                DataShare<T, TL>& ds, int (&rank)[TL::NPT]) {
  using DS = DataShare<T, TL>;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const unsigned long long below = (1ull << lane) - 1ull;
  int base = 0;
#pragma unroll
  for (int k = 0; k < TL::NPT; ++k) {
    const unsigned long long m = __ballot(slot[k] >= 0);
    rank[k] = -1;
    if (slot[k] >= 0) {
      rank[k] = base + __popcll(m & below);
      const int e = wv * DS::SEG + rank[k];
      ds.slot[e] = slot[k];
      ds.node[e] = TilePos<TL>::own(k);
    }
    base += __popcll(m);
  }
  if (lane == 0) ds.cnt[wv] = base;
}

// Data part of A p for every listed node of the workgroup (after the barrier
// that publishes the lists and the tile's p); results in ds.d.
template <typename T, typename TL>
__device__ __forceinline__ void eval_data_nodes(const LevelView<T>& L,
                                                const T (*sp)[TL::HALO],
                                                DataShare<T, TL>& ds) {
  using DS = DataShare<T, TL>;
  constexpr int CW = 16 / (int)sizeof(T);  // entries per 16-byte chunk
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int part = lane % kPartsPerNode, nl = lane / kPartsPerNode;
  // first list position of every wave's segment (uniform: scalar registers)
  int pre[DS::NW + 1];
  pre[0] = 0;
#pragma unroll
  for (int w = 0; w < DS::NW; ++w) pre[w + 1] = pre[w] + __builtin_amdgcn_readfirstlane(ds.cnt[w]);
  const int total = pre[DS::NW];
  for (int r0 = 0; r0 < total; r0 += DS::NW * kNodesPerWave) {
    const int v = r0 + wv * kNodesPerWave + nl;
    T o0 = T(0), o1 = T(0), o2 = T(0);
    int e = -1;
    if (nl < kNodesPerWave && v < total) {
      // the segment holding list position v: the last one starting at or
      // before it (segments are in wave order)
      int u = 0, before = 0;
#pragma unroll
      for (int x = 1; x < DS::NW; ++x)
        if (v >= pre[x]) {
          u = x;
          before = pre[x];
        }
      e = u * DS::SEG + (v - before);
      const int cz = ds.node[e] + TL::HX * TL::HY * (part - 1);
      // entry x of the part: chunk 3 (x / CW) + part of the row
      const gptr<const T> __restrict__ A = glob<const T>(static_cast<const T*>(
          __builtin_assume_aligned(L.A27r + (size_t)ds.slot[e] * kA27Row + part * CW, 16)));
      auto entry = [&](int x) { return A[kPartsPerNode * CW * (x / CW) + x % CW]; };
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int q = cz + (j % 3 - 1) + TL::HX * (j / 3 - 1);
        const T s0 = entry(6 * j), s1 = entry(6 * j + 1), s2 = entry(6 * j + 2),
                s3 = entry(6 * j + 3), s4 = entry(6 * j + 4), s5 = entry(6 * j + 5);
        const T q0 = sp[0][q], q1 = sp[1][q], q2 = sp[2][q];
        o0 += s0 * q0 + s1 * q1 + s2 * q2;
        o1 += s1 * q0 + s3 * q1 + s4 * q2;
        o2 += s2 * q0 + s4 * q1 + s5 * q2;
      }
    }
    const T a0 = __shfl_down(o0, 1, kWave), a1 = __shfl_down(o1, 1, kWave),
            a2 = __shfl_down(o2, 1, kWave);
    const T b0 = __shfl_down(o0, 2, kWave), b1 = __shfl_down(o1, 2, kWave),
            b2 = __shfl_down(o2, 2, kWave);
    if (part == 0 && e >= 0) {
      ds.d[0][e] = (o0 + a0) + b0;
      ds.d[1][e] = (o1 + a1) + b1;
      ds.d[2][e] = (o2 + a2) + b2;
    }
  }
}

// kModeRhs : p = d; g = A d - b + w_r sum_j (2I - R_i - R_j) e_ij is the
//            gradient J^T r; r = -g is stored (the CG residual r_0).
// kModeApply / kModeGrad : A p or g written to `out` (test entry points).
template <typename T, typename TL, int MODE, bool MASK>
__global__ __launch_bounds__(TL::NT) void k_stencil(Dispatch<T> D, const T* __restrict__ pin,
                                                    T* __restrict__ out) {
  if (skipped(D)) return;
  __shared__ T sp[3][TL::HALO];
  __shared__ unsigned char sm[TL::HALO];
  __shared__ DataShare<T, TL> ds;
  const Where<T> w = locate(D, xcd_remap(blockIdx.x, gridDim.x));
  const LevelView<T>& L = w.L;
  const TilePos<TL> t(L.nx, L.ny, w.local);
  const size_t N = L.N;
  const gptr<const T> __restrict__ src = glob<const T>((MODE == kModeRhs) ? L.d : pin);
  // the CG solve that follows a gradient pass counts its grid barrier from 0
  if (MODE == kModeRhs && w.local == 0 && threadIdx.x == 0) L.sc->bar = 0u;
  // MASK: the optimised set M (a lattice of the launch may still have none)
  const gptr<const unsigned char> __restrict__ act =
      MASK ? glob<const unsigned char>(L.act) : nullptr;
  const gptr<T> __restrict__ dst_out = glob<T>((MODE == kModeRhs) ? L.r : out);
  if (MODE == kModeRhs && act) {
    // a tile without points of M has no unknowns (its r is never read)
    int any = 0;
#pragma unroll
    for (int kk = 0; kk < TL::NPT; ++kk) {
      const int c = TilePos<TL>::own(kk);
      const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
      const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
      if ((TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz)))
        any |= act[gx + (size_t)L.nx * (gy + (size_t)L.ny * gz)];
    }
    if (!__syncthreads_or(any)) return;
  }
  // own nodes' data-block slots (loaded with the tile)
  int own_slot[TL::NPT];
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    own_slot[kk] = (TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz))
                       ? glob<const int>(L.node_slot)[gx + (size_t)L.nx * (gy + (size_t)L.ny * gz)]
                       : -1;
  }
  for (int k = threadIdx.x; k < TL::HALO; k += TL::NT) {
    const int lx = k % TL::HX, ly = (k / TL::HX) % TL::HY, lz = k / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    T v0 = T(0), v1 = T(0), v2 = T(0);
    unsigned char m = 0;
    if (in_box(gx, gy, gz, L.nx, L.ny, L.nz)) {
      const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
      m = act ? act[i] : 1;
      // A p acts on the unknowns of M only; the gradient reads the stored
      // displacement of every point
      if (MODE != kModeApply || m) {
        v0 = src[i];
        v1 = src[N + i];
        v2 = src[2 * N + i];
      }
    }
    sp[0][k] = v0;
    sp[1][k] = v1;
    sp[2][k] = v2;
    if (MASK) sm[k] = m;
  }
  int rank[TL::NPT];
  list_data_nodes<T, TL>(own_slot, ds, rank);
  __syncthreads();
  eval_data_nodes<T, TL>(L, sp, ds);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    if (!(TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz))) continue;
    const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
    if (act && !act[i]) {
      // not an unknown: zero gradient / product
      dst_out[i] = T(0);
      dst_out[N + i] = T(0);
      dst_out[2 * N + i] = T(0);
      continue;
    }
    T o0, o1, o2;
    arap_at<T, TL>(L, sp, c, gx, gy, gz, o0, o1, o2, act ? sm : nullptr);
    if (rank[kk] >= 0) {
      const int e = (threadIdx.x / kWave) * DataShare<T, TL>::SEG + rank[kk];
      o0 += ds.d[0][e];
      o1 += ds.d[1][e];
      o2 += ds.d[2][e];
    }
    if (MODE == kModeApply) {
      dst_out[i] = o0;
      dst_out[N + i] = o1;
      dst_out[2 * N + i] = o2;
      continue;
    }
    // rotation part of the ARAP gradient: for neighbour j = i + s*axis,
    // e_ij = -s h axis and (2I - R_i - R_j) e_ij = -s h (2 axis - R_i[:,k] - R_j[:,k]).
    const gptr<const T> __restrict__ rot = glob<const T>(L.rot);
    const gptr<const T> __restrict__ bnode = glob<const T>(L.bnode);
    T q0 = T(0), q1 = T(0), q2 = T(0);
    const int pos[3] = {gx, gy, gz};
    const int lim[3] = {L.nx, L.ny, L.nz};
    const size_t stride[3] = {1, (size_t)L.nx, (size_t)L.nx * L.ny};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T ci0 = rot[rot_at(0, ax, N, i)], ci1 = rot[rot_at(1, ax, N, i)],
              ci2 = rot[rot_at(2, ax, N, i)];
#pragma unroll
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int pj = pos[ax] + sgn;
        if (pj < 0 || pj >= lim[ax]) continue;
        const size_t j = sgn > 0 ? i + stride[ax] : i - stride[ax];
        const T cj0 = rot[rot_at(0, ax, N, j)], cj1 = rot[rot_at(1, ax, N, j)],
                cj2 = rot[rot_at(2, ax, N, j)];
        if (act && !act[j]) continue;  // only the edges inside M
        const T s = -T(sgn) * L.h;
        T u0 = -ci0 - cj0, u1 = -ci1 - cj1, u2 = -ci2 - cj2;
        if (ax == 0) u0 += T(2);
        if (ax == 1) u1 += T(2);
        if (ax == 2) u2 += T(2);
        q0 += s * u0;
        q1 += s * u1;
        q2 += s * u2;
      }
    }
    const T g0 = o0 - bnode[i] + L.wr * q0;
    const T g1 = o1 - bnode[N + i] + L.wr * q1;
    const T g2 = o2 - bnode[2 * N + i] + L.wr * q2;
    const T sg = (MODE == kModeGrad) ? T(1) : T(-1);
    dst_out[i] = sg * g0;
    dst_out[N + i] = sg * g1;
    dst_out[2 * N + i] = sg * g2;
  }
}

template <typename T, typename TL, bool MASK>
void launch_stencil_m(int mode, const Dispatch<T>& D, const T* pin, T* out, hipStream_t s) {
  switch (mode) {
    case kModeRhs:
      k_stencil<T, TL, kModeRhs, MASK><<<D.blocks, TL::NT, 0, s>>>(D, pin, out);
      break;
    case kModeApply:
      k_stencil<T, TL, kModeApply, MASK><<<D.blocks, TL::NT, 0, s>>>(D, pin, out);
      break;
    default: k_stencil<T, TL, kModeGrad, MASK><<<D.blocks, TL::NT, 0, s>>>(D, pin, out); break;
  }
}

template <typename T, typename TL>
void launch_stencil_t(int mode, const Dispatch<T>& D, const T* pin, T* out, hipStream_t s) {
  if (D.masked) launch_stencil_m<T, TL, true>(mode, D, pin, out, s);
  else launch_stencil_m<T, TL, false>(mode, D, pin, out, s);
}

// The tile kind is common to all lattices of a launch.
template <typename T>
hipError_t launch_stencil(int mode, const Dispatch<T>& D, const T* pin, T* out, hipStream_t s) {
  if (mode != kModeRhs && mode != kModeApply && mode != kModeGrad) return hipErrorInvalidValue;
  if (D.blocks <= 0) return hipSuccess;
  switch (D.one.tile) {
    case 1: launch_stencil_t<T, TileM>(mode, D, pin, out, s); break;
    case 2: launch_stencil_t<T, TileW>(mode, D, pin, out, s); break;
    case 3: launch_stencil_t<T, TileX>(mode, D, pin, out, s); break;
    case 4: launch_stencil_t<T, TileZ>(mode, D, pin, out, s); break;
    case 5: launch_stencil_t<T, TileY>(mode, D, pin, out, s); break;
    case 6: launch_stencil_t<T, TileH>(mode, D, pin, out, s); break;
    case 7: launch_stencil_t<T, TileC>(mode, D, pin, out, s); break;
    default: launch_stencil_t<T, TileS>(mode, D, pin, out, s); break;
  }
  return hipGetLastError();
}

// ===========================================================================
// one Jacobi-preconditioned CG iteration per launch (Sec. 7.1, position step)
// ===========================================================================
//
// Iteration m (FIRST: m = 0) reads the block partials S_{m-1} of the
// previous launch: r^T D^-1 r, p^T A p, (Ap)^T D^-1 r and (Ap)^T D^-1 Ap of
// iterate m-1.  From them
//   alpha_{m-1} = rz_{m-1} / p^T A p                    (zero if p^T A p <= 0)
//   rz_m        = rz_{m-1} - 2 alpha (Ap)^T D^-1 r + alpha^2 (Ap)^T D^-1 Ap
//   beta_m      = rz_m / rz_{m-1}                       (zero if rz_{m-1} <= 0)
// (rz_m is r_m^T D^-1 r_m expanded through r_m = r_{m-1} - alpha Ap_{m-1}, so
// one reduction phase per iteration suffices).  While staging the tile it
// forms r_m = r_{m-1} - alpha Ap_{m-1}, p_m = D^-1 r_m + beta p_{m-1}, applies
// d += alpha p_{m-1} to its own nodes, computes Ap_m and writes S_m.  Iterate
// m keeps r, p, Ap and S in buffer m % 2 of each pair (r_0 in L.r).  The
// halo inputs are loaded before the scalar reduction so that both latencies
// overlap.  The last iteration's step is applied by k_cg_final.

// A CG scalar as the sum hi + lo of two T values (lo = 0 for float64).  The
// step sizes are computed in float64 and applied to float32 vectors through
// both parts, x + s y = fma(lo, y, fma(hi, y, x)): a step size rounded to
// float32 would perturb the iterate coherently along p, and truncated CG
// amplifies such perturbations by about an order of magnitude per iteration
// once its Ritz values settle.
template <typename T>
struct Step {
  T hi, lo;
  __device__ __forceinline__ static Step of(double s) {
    Step r;
    r.hi = (T)s;
    r.lo = (T)(s - (double)r.hi);
    return r;
  }
  __device__ __forceinline__ T axpy(T x, T y) const { return fma(lo, y, fma(hi, y, x)); }
};

template <typename T, int NT = kBlock>
__device__ __forceinline__ void cg_scalars(const double* s, int n, Step<T>& alpha, Step<T>& beta,
                                           Scalars* sc, bool count_guard) {
  double v[4];
  sum_partials_k<4, NT>(s, n, v);
  const double rz = v[0], pap = v[1], apdr = v[2], apdap = v[3];
  const double a = pap > 0.0 ? rz / pap : 0.0;
  double rz_new = rz - 2.0 * a * apdr + a * a * apdap;
  if (rz_new < 0.0) rz_new = 0.0;
  alpha = Step<T>::of(a);
  beta = Step<T>::of(rz > 0.0 ? rz_new / rz : 0.0);
  if (count_guard && threadIdx.x == 0 && !(pap > 0.0)) sc->guard_hits += 1;
}

// One CG iteration m on the tile of workgroup w (body of k_cg and of the
// persistent k_cg_loop).  The own nodes' data-block slot, preconditioner,
// displacement and previous direction are loaded together with the halo,
// before the CG scalars, so that every workgroup pays one memory round trip
// before it stages the tile (a form that loaded them at their use, for more
// resident waves, was slower also on grids of several rounds of workgroups).
template <typename T, typename TL, bool FIRST, bool MASK = false>
__device__ __forceinline__ void cg_body(const Where<T>& w, int m, T (&sp)[3][TL::HALO],
                                        T (&sr)[3][TL::HALO], unsigned char (&sm)[TL::HALO],
                                        DataShare<T, TL>& ds) {
  const LevelView<T>& L = w.L;
  const TilePos<TL> t(L.nx, L.ny, w.local);
  const size_t N = L.N;
  const bool odd = (m & 1) != 0;
  const gptr<const T> __restrict__ r_in = glob<const T>((FIRST || odd) ? L.r : L.r2);
  const gptr<T> __restrict__ r_out = glob<T>(odd ? L.r2 : L.r);
  const gptr<const T> __restrict__ p_in = glob<const T>(odd ? L.pa : L.pb);
  const gptr<T> __restrict__ p_out = glob<T>(odd ? L.pb : L.pa);
  const gptr<const T> __restrict__ ap_in = glob<const T>(odd ? L.ap : L.ap2);
  const gptr<T> __restrict__ ap_out = glob<T>(odd ? L.ap2 : L.ap);
  const double* s_in = odd ? L.scg0 : L.scg1;
  double* s_out = odd ? L.scg1 : L.scg0;
  const gptr<const T> __restrict__ dinv = glob<const T>(L.dinv);
  const gptr<T> __restrict__ dvec = glob<T>(L.d);
  const gptr<const int> __restrict__ node_slot = glob<const int>(L.node_slot);
  // MASK: the optimised set M (a lattice of the launch may still have none)
  const gptr<const unsigned char> __restrict__ act =
      MASK ? glob<const unsigned char>(L.act) : nullptr;
  if (act) {
    // restricted to M: a tile without points of M has no unknowns; its
    // partials are zero.  Points outside M are read as 0 below and their
    // vectors never written.
    int any = 0;
#pragma unroll
    for (int kk = 0; kk < TL::NPT; ++kk) {
      const int c = TilePos<TL>::own(kk);
      const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
      const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
      if ((TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz)))
        any |= act[gx + (size_t)L.nx * (gy + (size_t)L.ny * gz)];
    }
    if (!__syncthreads_or(any)) {
      if (!FIRST && w.local == 0) {
        Step<T> a0, b0;
        cg_scalars<T, TL::NT>(s_in, L.ntiles, a0, b0, L.sc, true);
      }
      double zero[4] = {0.0, 0.0, 0.0, 0.0};
      write_partials<4, TL::NT>(zero, s_out, w.count, w.local);
      return;
    }
  }
  // 1. halo inputs into registers
  T hr[TL::HPT][3], hq[TL::HPT][3], hp[TL::HPT][3], ha[TL::HPT][3];
  size_t hi[TL::HPT];
  bool hin[TL::HPT];
  unsigned char hm[TL::HPT];
#pragma unroll
  for (int h = 0; h < TL::HPT; ++h) {
    const int k = threadIdx.x + h * TL::NT;
    const int lx = k % TL::HX, ly = (k / TL::HX) % TL::HY, lz = k / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    hin[h] = k < TL::HALO && in_box(gx, gy, gz, L.nx, L.ny, L.nz);
    hi[h] = hin[h] ? gx + (size_t)L.nx * (gy + (size_t)L.ny * gz) : 0;
    hm[h] = hin[h] ? (act ? act[hi[h]] : 1) : 0;
    hin[h] = hin[h] && hm[h];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      hr[h][a] = T(0);
      hq[h][a] = T(0);
      hp[h][a] = T(0);
      ha[h][a] = T(0);
    }
    if (hin[h]) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = a * N + hi[h];
        hr[h][a] = r_in[j];
        hq[h][a] = dinv[j];
        if (!FIRST) {
          hp[h][a] = p_in[j];
          ha[h][a] = ap_in[j];
        }
      }
    }
  }
  // own nodes' data-block slot, preconditioner and displacement, loaded with
  // the halo so they are off the dependent chain of steps 3 and 4
  int own_slot[TL::NPT];
  T own_q[TL::NPT][3];
  T own_d[TL::NPT][3];
  T own_pp[TL::NPT][3];  // p of the previous iterate (the step d += alpha p)
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    own_slot[kk] = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      own_q[kk][a] = T(0);
      own_d[kk][a] = T(0);
      own_pp[kk][a] = T(0);
    }
    if ((TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz)) &&
        (!act || act[gx + (size_t)L.nx * (gy + (size_t)L.ny * gz)])) {
      const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
      own_slot[kk] = node_slot[i];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        own_q[kk][a] = dinv[a * N + i];
        if (!FIRST) {
          own_d[kk][a] = dvec[a * N + i];
          own_pp[kk][a] = p_in[a * N + i];
        }
      }
    }
  }
  // 2. CG scalars of the previous iterate
  Step<T> alpha = Step<T>::of(0.0), beta = Step<T>::of(0.0);
  if (!FIRST) cg_scalars<T, TL::NT>(s_in, L.ntiles, alpha, beta, L.sc, w.local == 0);
  int rank[TL::NPT];
  list_data_nodes<T, TL>(own_slot, ds, rank);
  // 3. r_m, p_m into LDS; own nodes also store r_m, p_m and step d
#pragma unroll
  for (int h = 0; h < TL::HPT; ++h) {
    const int k = threadIdx.x + h * TL::NT;
    if (k >= TL::HALO) continue;
    T p3[3], r3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T r = hr[h][a];
      if (!FIRST) r = alpha.axpy(r, -ha[h][a]);
      T p = hq[h][a] * r;
      if (!FIRST) p = beta.axpy(p, hp[h][a]);
      r3[a] = r;
      p3[a] = p;
      sp[a][k] = p;
      sr[a][k] = r;
    }
    if (MASK) sm[k] = hm[h];
    const int lx = k % TL::HX, ly = (k / TL::HX) % TL::HY, lz = k / (TL::HX * TL::HY);
    if (hin[h] && lx >= 1 && lx <= TL::TX && ly >= 1 && ly <= TL::TY && lz >= 1 &&
        lz <= TL::TZ) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = a * N + hi[h];
        p_out[j] = p3[a];
        if (!FIRST) r_out[j] = r3[a];
      }
    }
  }
  __syncthreads();
  // 4. A p_m on own nodes and the block partials of S_m
  eval_data_nodes<T, TL>(L, sp, ds);
  __syncthreads();
  double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    if (!(TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz)) || (act && !sm[c])) continue;
    const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
    T o[3];
    arap_at<T, TL>(L, sp, c, gx, gy, gz, o[0], o[1], o[2], act ? sm : nullptr);
    const int e = (threadIdx.x / kWave) * DataShare<T, TL>::SEG + rank[kk];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (rank[kk] >= 0) o[a] += ds.d[a][e];
      const size_t j = a * N + i;
      ap_out[j] = o[a];
      if (!FIRST) dvec[j] = alpha.axpy(own_d[kk][a], own_pp[kk][a]);
      const double q = (double)own_q[kk][a], r = (double)sr[a][c],
                   p = (double)sp[a][c];
      const double ap = (double)o[a];
      part[0] += r * q * r;
      part[1] += p * ap;
      part[2] += ap * q * r;
      part[3] += ap * q * ap;
    }
  }
  write_partials<4, TL::NT>(part, s_out, w.count, w.local);
}

// Clock stamp of a launch's first workgroup at its start (graph timing).
__device__ __forceinline__ void entry_stamp(unsigned long long* stamp) {
  if (stamp != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
    *stamp = (unsigned long long)wall_clock64();
}

template <typename T, typename TL, bool FIRST, bool MASK>
__global__ __launch_bounds__(TL::NT) void k_cg(Dispatch<T> D, int m, unsigned long long* stamp) {
  if (skipped(D)) return;
  __shared__ T sp[3][TL::HALO];
  __shared__ T sr[3][TL::HALO];
  __shared__ unsigned char sm[TL::HALO];
  __shared__ DataShare<T, TL> ds;
  entry_stamp(stamp);
  const Where<T> w = locate(D, xcd_remap(blockIdx.x, gridDim.x));
  cg_body<T, TL, FIRST, MASK>(w, m, sp, sr, sm, ds);
}

// Grid barrier of a launch whose workgroups are all resident: every
// workgroup publishes its writes (agent-scope release), counts itself in,
// waits for `target` arrivals and then acquires.  The wait is bounded: after
// kSpinLimit polls it gives up and counts a timeout, so the kernel always
// ends (the result of such a frame is then reported as unreliable).
constexpr unsigned kSpinLimit = 1u << 18;

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, int* timeouts) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1u);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        atomicAdd(timeouts, 1);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

// The last step d += alpha p of CG iterate `last` on the tile's own nodes.
template <typename T, typename TL>
__device__ __forceinline__ void cg_final_tile(const Where<T>& w, int last) {
  const LevelView<T>& L = w.L;
  const TilePos<TL> t(L.nx, L.ny, w.local);
  const bool odd = (last & 1) != 0;
  Step<T> alpha, beta;
  cg_scalars<T, TL::NT>(odd ? L.scg1 : L.scg0, L.ntiles, alpha, beta, L.sc, w.local == 0);
  const size_t N = L.N;
  const gptr<const T> __restrict__ p = glob<const T>(odd ? L.pb : L.pa);
  const gptr<T> __restrict__ d = glob<T>(L.d);
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    if (!(TilePos<TL>::owner() && in_box(gx, gy, gz, L.nx, L.ny, L.nz))) continue;
    const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
    if (L.act && !L.act[i]) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a * N + i] = alpha.axpy(d[a * N + i], p[a * N + i]);
  }
}

// All iterations of one CG solve (single lattice, every tile resident).
template <typename T, typename TL, bool MASK>
__global__ __launch_bounds__(TL::NT) void k_cg_loop(Dispatch<T> D, int iters) {
  if (skipped(D)) return;
  __shared__ T sp[3][TL::HALO];
  __shared__ T sr[3][TL::HALO];
  __shared__ unsigned char sm[TL::HALO];
  __shared__ DataShare<T, TL> ds;
  const Where<T> w = locate(D, xcd_remap(blockIdx.x, gridDim.x));
  Scalars* sc = w.L.sc;
  for (int m = 0; m < iters; ++m) {
    if (m == 0)
      cg_body<T, TL, true, MASK>(w, m, sp, sr, sm, ds);
    else
      cg_body<T, TL, false, MASK>(w, m, sp, sr, sm, ds);
    grid_barrier(&sc->bar, (unsigned)(m + 1) * gridDim.x, &sc->bar_timeouts);
  }
  cg_final_tile<T, TL>(w, iters - 1);
}

// d += alpha p of the last CG iterate (node workgroups).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_final(Dispatch<T> D, int last,
                                                     unsigned long long* stamp) {
  if (skipped(D)) return;
  entry_stamp(stamp);
  const Where<T> w = locate(D, blockIdx.x);
  const LevelView<T>& L = w.L;
  const bool odd = (last & 1) != 0;
  Step<T> alpha, beta;
  cg_scalars<T>(odd ? L.scg1 : L.scg0, L.ntiles, alpha, beta, L.sc, w.local == 0);
  const int i = w.local * kBlock + threadIdx.x;
  if (i >= L.N || (L.act && !L.act[i])) return;
  const size_t N = L.N;
  const gptr<const T> __restrict__ p = glob<const T>(odd ? L.pb : L.pa);
  const gptr<T> __restrict__ d = glob<T>(L.d);
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a * N + i] = alpha.axpy(d[a * N + i], p[a * N + i]);
}

template <typename T, typename TL>
void launch_cg_t(int m, const Dispatch<T>& D, hipStream_t s, unsigned long long* stamp) {
  if (D.masked) {
    if (m == 0) k_cg<T, TL, true, true><<<D.blocks, TL::NT, 0, s>>>(D, m, stamp);
    else k_cg<T, TL, false, true><<<D.blocks, TL::NT, 0, s>>>(D, m, stamp);
  } else {
    if (m == 0) k_cg<T, TL, true, false><<<D.blocks, TL::NT, 0, s>>>(D, m, stamp);
    else k_cg<T, TL, false, false><<<D.blocks, TL::NT, 0, s>>>(D, m, stamp);
  }
}

template <typename T>
hipError_t launch_cg(int m, const Dispatch<T>& D, hipStream_t s, unsigned long long* stamp) {
  if (D.blocks <= 0) return hipSuccess;
  switch (D.one.tile) {
    case 1: launch_cg_t<T, TileM>(m, D, s, stamp); break;
    case 2: launch_cg_t<T, TileW>(m, D, s, stamp); break;
    case 3: launch_cg_t<T, TileX>(m, D, s, stamp); break;
    case 4: launch_cg_t<T, TileZ>(m, D, s, stamp); break;
    case 5: launch_cg_t<T, TileY>(m, D, s, stamp); break;
    case 6: launch_cg_t<T, TileH>(m, D, s, stamp); break;
    case 7: launch_cg_t<T, TileC>(m, D, s, stamp); break;
    default: launch_cg_t<T, TileS>(m, D, s, stamp); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_final(int last, const Dispatch<T>& D, hipStream_t s,
                           unsigned long long* stamp) {
  if (D.blocks <= 0) return hipSuccess;
  k_cg_final<T><<<D.blocks, kBlock, 0, s>>>(D, last, stamp);
  return hipGetLastError();
}

template <typename T, bool MASK>
void launch_cg_loop_t(int iters, const Dispatch<T>& D, hipStream_t s) {
  switch (D.one.tile) {
    case 1: k_cg_loop<T, TileM, MASK><<<D.blocks, TileM::NT, 0, s>>>(D, iters); break;
    case 2: k_cg_loop<T, TileW, MASK><<<D.blocks, TileW::NT, 0, s>>>(D, iters); break;
    case 3: k_cg_loop<T, TileX, MASK><<<D.blocks, TileX::NT, 0, s>>>(D, iters); break;
    case 4: k_cg_loop<T, TileZ, MASK><<<D.blocks, TileZ::NT, 0, s>>>(D, iters); break;
    case 5: k_cg_loop<T, TileY, MASK><<<D.blocks, TileY::NT, 0, s>>>(D, iters); break;
    case 6: k_cg_loop<T, TileH, MASK><<<D.blocks, TileH::NT, 0, s>>>(D, iters); break;
    case 7: k_cg_loop<T, TileC, MASK><<<D.blocks, TileC::NT, 0, s>>>(D, iters); break;
    default: k_cg_loop<T, TileS, MASK><<<D.blocks, TileS::NT, 0, s>>>(D, iters); break;
  }
}

template <typename T>
hipError_t launch_cg_loop(int iters, const Dispatch<T>& D, hipStream_t s) {
  if (D.blocks <= 0 || iters <= 0) return hipSuccess;
  if (D.n != 1 || D.blocks > kPersistMaxTiles || D.blocks != D.one.ntiles)
    return hipErrorInvalidValue;
  if (D.masked) launch_cg_loop_t<T, true>(iters, D, s);
  else launch_cg_loop_t<T, false>(iters, D, s);
  return hipGetLastError();
}

// ===========================================================================
// energy, eq. (1): rows (dense and sparse) and ARAP edges, float64 sums
// ===========================================================================

template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy(Dispatch<T> D) {
  if (skipped(D)) return;
  const Where<T> w = locate(D, blockIdx.x);
  const LevelView<T>& L = w.L;
  double part[3] = {0.0, 0.0, 0.0};
  const size_t N = L.N;
  const T* __restrict__ d = L.d;
  if (w.local < L.rblocks) {
    const int row = w.local * kBlock + threadIdx.x;
    const int rows = L.sc->rows;
    if (row < rows) {
      const int cell = L.row_cell[row];
      const int cnx = L.nx - 1, cny = L.ny - 1;
      const int cx = cell % cnx, cy = (cell / cnx) % cny, cz = cell / (cnx * cny);
      const T* __restrict__ f = L.row_f;
      const T* __restrict__ sn = L.row_sn;
      const T fx = f[row], fy = f[(size_t)rows + row], fz = f[2 * (size_t)rows + row];
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t m = (cx + (k & 1)) + (size_t)L.nx * ((cy + ((k >> 1) & 1)) +
                                                          (size_t)L.ny * (cz + (k >> 2)));
        const T wk = corner_weight<T>(k, fx, fy, fz);
        s0 += wk * d[m];
        s1 += wk * d[N + m];
        s2 += wk * d[2 * N + m];
      }
      const T res = sn[row] * s0 + sn[(size_t)rows + row] * s1 + sn[2 * (size_t)rows + row] * s2 -
                    L.row_rho[row];
      const double e = (double)res * (double)res;
      if (row < L.sc->n_dense) part[0] = e; else part[1] = e;
    }
  } else {
    const int i = (w.local - L.rblocks) * kBlock + threadIdx.x;
    // E_reg sums the edges inside M (all of them when the whole lattice is
    // optimised)
    if (i < L.N && (!L.act || L.act[i])) {
      const T* __restrict__ rot = L.rot;
      const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
      const int pos[3] = {x, y, z};
      const int lim[3] = {L.nx, L.ny, L.nz};
      const size_t stride[3] = {1, (size_t)L.nx, (size_t)L.nx * L.ny};
      double acc = 0.0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        // (I - R_i) e_ij with e_ij = -s h axis
        T c0 = -rot[rot_at(0, ax, N, i)], c1 = -rot[rot_at(1, ax, N, i)],
          c2 = -rot[rot_at(2, ax, N, i)];
        if (ax == 0) c0 += T(1);
        if (ax == 1) c1 += T(1);
        if (ax == 2) c2 += T(1);
#pragma unroll
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          const int pj = pos[ax] + sgn;
          if (pj < 0 || pj >= lim[ax]) continue;
          const size_t j = sgn > 0 ? i + stride[ax] : i - stride[ax];
          if (L.act && !L.act[j]) continue;
          const T s = -T(sgn) * L.h;
          const T e0 = d[i] - d[j] + s * c0;
          const T e1 = d[N + i] - d[N + j] + s * c1;
          const T e2 = d[2 * N + i] - d[2 * N + j] + s * c2;
          acc += (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
        }
      }
      part[2] = (double)L.wr * acc;
    }
  }
  write_partials<3>(part, L.pe, w.count, w.local);
}

// One workgroup per lattice: sums its energy partials into sc->energy.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy_finalize(Dispatch<T> D1, int record_trace) {
  if (skipped(D1)) return;
  const LevelView<T> L = view_of(D1, blockIdx.x);
  const int n = energy_blocks_dev(L);
  double v[3];
  sum_partials_k<3>(L.pe, n, v);
  if (threadIdx.x == 0) {
    Scalars* sc = L.sc;
    sc->energy[0] = v[0] + v[1] + v[2];
    sc->energy[1] = v[0];
    sc->energy[2] = v[1];
    sc->energy[3] = v[2];
    if (record_trace && sc->n_trace < VD_MAX_TRACE) {
      sc->trace[sc->n_trace] = sc->energy[0];
      sc->n_trace += 1;
    }
  }
}

template <typename T>
hipError_t launch_energy(const Dispatch<T>& De, const Dispatch<T>& D1, int record_trace,
                         hipStream_t s) {
  if (De.blocks <= 0) return hipSuccess;
  k_energy<T><<<De.blocks, kBlock, 0, s>>>(De);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_energy_finalize<T><<<D1.blocks, kBlock, 0, s>>>(D1, record_trace);
  return hipGetLastError();
}

template <typename T>
__global__ void k_reset_counters(Dispatch<T> D1) {
  if (threadIdx.x != 0) return;
  Scalars* sc = view_of(D1, blockIdx.x).sc;
  sc->guard_hits = 0;
  sc->polar_fp64 = 0;
  sc->polar_keep = 0;
  sc->n_trace = 0;
  sc->bar_timeouts = 0;
}

__global__ void k_target_begin(Scalars* sc, double target) {
  if (threadIdx.x != 0) return;
  sc->target = target;
  sc->gn_done = 0;
  sc->stop = sc->energy[0] <= target ? 1 : 0;
}

__global__ void k_target_step(Scalars* sc) {
  if (threadIdx.x != 0 || sc->stop) return;
  sc->gn_done += 1;
  if (sc->energy[0] <= sc->target) sc->stop = 1;
}

hipError_t launch_target_begin(Scalars* sc, double target, hipStream_t s) {
  k_target_begin<<<1, 64, 0, s>>>(sc, target);
  return hipGetLastError();
}

hipError_t launch_target_step(Scalars* sc, hipStream_t s) {
  k_target_step<<<1, 64, 0, s>>>(sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reset_counters(const Dispatch<T>& D1, hipStream_t s) {
  k_reset_counters<T><<<D1.blocks, 64, 0, s>>>(D1);
  return hipGetLastError();
}

// ===========================================================================
// rotation step (Sec. 7.1): M_i = sum_j (t_i - t_j)(t_hat_i - t_hat_j)^T
// ===========================================================================

template <typename T>
__global__ __launch_bounds__(kBlock) void k_polar(Dispatch<T> D) {
  if (skipped(D)) return;
  const Where<T> w = locate(D, blockIdx.x);
  const LevelView<T>& L = w.L;
  const int i = w.local * kBlock + threadIdx.x;
  if (i >= L.N || (L.act && !L.act[i])) return;  // points outside M keep R
  const size_t N = L.N;
  const T* __restrict__ d = L.d;
  T* rot = L.rot;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const int pos[3] = {x, y, z};
  const int lim[3] = {L.nx, L.ny, L.nz};
  const size_t stride[3] = {1, (size_t)L.nx, (size_t)L.nx * L.ny};
  const T di0 = d[i], di1 = d[N + i], di2 = d[2 * N + i];
  T M[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = T(0);
  const T h2 = L.h * L.h;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      const int pj = pos[ax] + sgn;
      if (pj < 0 || pj >= lim[ax]) continue;
      const size_t j = sgn > 0 ? i + stride[ax] : i - stride[ax];
      if (L.act && !L.act[j]) continue;  // the terms of eq. (4) inside M
      // (d_i - d_j + e_ij) e_ij^T with e_ij = -s h axis: column ax gets
      // -s h (d_i - d_j) + h^2 axis
      const T s = -T(sgn) * L.h;
      M[0 * 3 + ax] += s * (di0 - d[j]);
      M[1 * 3 + ax] += s * (di1 - d[N + j]);
      M[2 * 3 + ax] += s * (di2 - d[2 * N + j]);
      M[ax * 3 + ax] += h2;
    }
  }
  T Rp[9], R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rp[k] = rot[(size_t)k * N + i];
  const int code = fit_or_keep<T>(M, Rp, R);
#pragma unroll
  for (int k = 0; k < 9; ++k) rot[(size_t)k * N + i] = R[k];
  if (code == kFitFp64) atomicAdd(&L.sc->polar_fp64, 1);
  if (code == kFitKeep) atomicAdd(&L.sc->polar_keep, 1);
}

template <typename T>
hipError_t launch_polar(const Dispatch<T>& D, hipStream_t s) {
  if (D.blocks <= 0) return hipSuccess;
  k_polar<T><<<D.blocks, kBlock, 0, s>>>(D);
  return hipGetLastError();
}

// ===========================================================================
// level transfers (Sec. 7.2)
// ===========================================================================

// Level node (a,b,c) takes the finest node stride*(a,b,c): d, base and R.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inject(Dispatch<T> D, Dispatch<T> F, int stride) {
  const Where<T> w = locate(D, blockIdx.x);
  const LevelView<T>& Lv = w.L;
  const int i = w.local * kBlock + threadIdx.x;
  if (i >= Lv.N) return;
  const LevelView<T> Fv = view_of(F, w.b);
  const int x = i % Lv.nx, y = (i / Lv.nx) % Lv.ny, z = i / (Lv.nx * Lv.ny);
  const size_t f = (size_t)x * stride + (size_t)Fv.nx * ((size_t)y * stride + (size_t)Fv.ny * z * stride);
  const size_t N = Lv.N, NF = Fv.N;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T v = Fv.d[k * NF + f];
    Lv.d[k * N + i] = v;
    Lv.base[k * N + i] = v;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Lv.rot[k * N + i] = Fv.rot[k * NF + f];
}

template <typename T>
hipError_t launch_inject(const Dispatch<T>& D, const Dispatch<T>& F, int stride, hipStream_t s) {
  if (D.blocks <= 0) return hipSuccess;
  k_inject<T><<<D.blocks, kBlock, 0, s>>>(D, F, stride);
  return hipGetLastError();
}

// fine.d (+)= trilinear evaluation of (coarse.d - coarse.base) at the fine
// rest positions: fine node a sits at coarse coordinate a/2; its cell is
// clamped to the last coarse cell, so the last fine plane of an even-sized
// axis is linearly extrapolated (f = 1.5).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(Dispatch<T> D, Dispatch<T> C, int add) {
  const Where<T> w = locate(D, blockIdx.x);
  const LevelView<T>& Fl = w.L;
  const int i = w.local * kBlock + threadIdx.x;
  if (i >= Fl.N) return;
  if (add && Fl.act && !Fl.act[i]) return;  // the increment reaches M only
  const LevelView<T> Cv = view_of(C, w.b);
  const int x = i % Fl.nx, y = (i / Fl.nx) % Fl.ny, z = i / (Fl.nx * Fl.ny);
  const int p[3] = {x, y, z};
  const int nc[3] = {Cv.nx, Cv.ny, Cv.nz};
  int cc[3];
  T f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int c = p[k] >> 1;
    if (c > nc[k] - 2) c = nc[k] - 2;
    cc[k] = c;
    f[k] = T(0.5) * T(p[k]) - T(c);
  }
  const size_t NC = Cv.N, NF = Fl.N;
  const T* __restrict__ cin = Cv.d;
  const T* __restrict__ cbase = Cv.base;
  T v[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const size_t m = (cc[0] + (k & 1)) +
                     (size_t)Cv.nx * ((cc[1] + ((k >> 1) & 1)) + (size_t)Cv.ny * (cc[2] + (k >> 2)));
    const T wk = corner_weight<T>(k, f[0], f[1], f[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T inc = cbase ? cin[a * NC + m] - cbase[a * NC + m] : cin[a * NC + m];
      v[a] += wk * inc;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (add) Fl.d[a * NF + i] += v[a];
    else Fl.d[a * NF + i] = v[a];
  }
}

template <typename T>
hipError_t launch_prolong(const Dispatch<T>& Dfine, const Dispatch<T>& C, int add, hipStream_t s) {
  if (Dfine.blocks <= 0) return hipSuccess;
  k_prolong<T><<<Dfine.blocks, kBlock, 0, s>>>(Dfine, C, add);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_rest(Dispatch<T> D) {
  const Where<T> w = locate(D, blockIdx.x);
  const LevelView<T>& L = w.L;
  const int i = w.local * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const size_t N = L.N;
#pragma unroll
  for (int k = 0; k < 3; ++k) L.d[k * N + i] = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) L.rot[k * N + i] = (k % 4 == 0) ? T(1) : T(0);
}

template <typename T>
hipError_t launch_set_rest(const Dispatch<T>& D, hipStream_t s) {
  if (D.blocks <= 0) return hipSuccess;
  k_set_rest<T><<<D.blocks, kBlock, 0, s>>>(D);
  return hipGetLastError();
}

#define VD_INSTANTIATE_SOLVE(T)                                                                  \
  template hipError_t launch_stencil<T>(int, const Dispatch<T>&, const T*, T*, hipStream_t);    \
  template hipError_t launch_cg<T>(int, const Dispatch<T>&, hipStream_t, unsigned long long*);   \
  template hipError_t launch_cg_final<T>(int, const Dispatch<T>&, hipStream_t,                   \
                                          unsigned long long*);                                 \
  template hipError_t launch_energy<T>(const Dispatch<T>&, const Dispatch<T>&, int, hipStream_t); \
  template hipError_t launch_reset_counters<T>(const Dispatch<T>&, hipStream_t);                 \
  template hipError_t launch_cg_loop<T>(int, const Dispatch<T>&, hipStream_t);                   \
  template hipError_t launch_polar<T>(const Dispatch<T>&, hipStream_t);                          \
  template hipError_t launch_inject<T>(const Dispatch<T>&, const Dispatch<T>&, int, hipStream_t); \
  template hipError_t launch_prolong<T>(const Dispatch<T>&, const Dispatch<T>&, int, hipStream_t); \
  template hipError_t launch_set_rest<T>(const Dispatch<T>&, hipStream_t);

VD_INSTANTIATE_SOLVE(float)
VD_INSTANTIATE_SOLVE(double)

}  // namespace vd
