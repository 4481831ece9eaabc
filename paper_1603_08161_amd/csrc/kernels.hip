// HIP kernels of the lattice solver (gfx950).
//
// Unknowns are stored as displacements d_i = t_i - t_hat_i (float32 by
// default): the residuals of eqs. (2)-(4) are then differences of small
// numbers, which keeps float32 accurate even when the lattice sits far from
// the world origin.  Every node vector is SoA [3][N] in x-fastest node order.

#include "vd_device.h"
#include "vd_kernels.h"

namespace vd {

namespace {

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ bool in_box(int x, int y, int z, int nx, int ny, int nz) {
  return x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
}

// Row-major index of rotation entry (row, col) in the [9][N] SoA array.
__device__ __forceinline__ size_t rot_at(int row, int col, size_t N, size_t i) {
  return (size_t)(row * 3 + col) * N + i;
}

// Unique (a <= b) corner pairs of a cell and the six components of a
// symmetric 3x3 block.
__constant__ unsigned char c_pair_a[36] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2,
                                           2, 2, 2, 3, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5, 5, 6, 6, 7};
__constant__ unsigned char c_pair_b[36] = {0, 1, 2, 3, 4, 5, 6, 7, 1, 2, 3, 4, 5, 6, 7, 2, 3, 4,
                                           5, 6, 7, 3, 4, 5, 6, 7, 4, 5, 6, 7, 5, 6, 7, 6, 7, 7};
__constant__ unsigned char c_comp_i[6] = {0, 0, 0, 1, 1, 2};
__constant__ unsigned char c_comp_j[6] = {0, 1, 2, 1, 2, 2};

}  // namespace

// ===========================================================================
// constraint validation and per-level rows
// ===========================================================================

__global__ __launch_bounds__(kBlock) void k_validate(RawConstraints c, int nx0, int ny0, int nz0,
                                                     double h0, double ox, double oy, double oz,
                                                     int* flags) {
  const int total = c.n_dense + c.n_sparse;
  int f = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    const float* pc;
    const float* pt;
    if (i < c.n_dense) {
      pc = c.canon + 3 * (size_t)i;
      pt = c.target + 3 * (size_t)i;
      const float* pn = c.normal + 3 * (size_t)i;
      for (int k = 0; k < 3; ++k)
        if (!isfinite(pn[k])) f |= 1;
      if (c.weight) {
        const float w = c.weight[i];
        if (!isfinite(w) || w < 0.0f) f |= 1;
      }
    } else {
      const int s = i - c.n_dense;
      pc = c.sparse_canon + 3 * (size_t)s;
      pt = c.sparse_target + 3 * (size_t)s;
    }
    for (int k = 0; k < 3; ++k)
      if (!isfinite(pc[k]) || !isfinite(pt[k])) f |= 1;
    const double o[3] = {ox, oy, oz};
    const int n[3] = {nx0, ny0, nz0};
    for (int k = 0; k < 3; ++k) {
      const double u = ((double)pc[k] - o[k]) / h0;
      if (!(u >= 0.0 && u <= (double)(n[k] - 1))) f |= 2;
    }
  }
  if (f) atomicOr(flags, f);
}

hipError_t launch_validate(const RawConstraints& c, int nx0, int ny0, int nz0, double h0,
                           const double* o, int* flags, hipStream_t s) {
  const int total = c.n_dense + c.n_sparse;
  if (total == 0) return hipSuccess;
  int grid = blocks_for(total);
  if (grid > 4096) grid = 4096;
  k_validate<<<grid, kBlock, 0, s>>>(c, nx0, ny0, nz0, h0, o[0], o[1], o[2], flags);
  return hipGetLastError();
}

// One row per dense correspondence (eq. (2)) and three per sparse pair
// (eq. (3): a point-to-point term is the sum of three axis-aligned
// point-to-plane terms).  Row value: sn . sum_k alpha_k d_k - rho, with
// sn = sqrt(w) * normal and rho = sn . (target - canonical).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rows(RawConstraints c, LevelView<T> L, RowView<T> R,
                                                 double ox, double oy, double oz, double wd,
                                                 double ws, unsigned* keys, int* vals) {
  const int rows = R.rows;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < rows; i += gridDim.x * kBlock) {
    double x[3], sn[3], rho;
    if (i < c.n_dense) {
      const size_t b = 3 * (size_t)i;
      double n[3], tp[3];
      for (int k = 0; k < 3; ++k) {
        x[k] = c.canon[b + k];
        tp[k] = c.target[b + k];
        n[k] = c.normal[b + k];
      }
      const double ln = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      double w = c.weight ? (double)c.weight[i] : 1.0;
      if (ln > 0.0) {
        for (int k = 0; k < 3; ++k) n[k] /= ln;
      } else {
        w = 0.0;
        n[0] = n[1] = n[2] = 0.0;
      }
      const double s = sqrt(wd * w);
      rho = 0.0;
      for (int k = 0; k < 3; ++k) {
        sn[k] = s * n[k];
        rho += sn[k] * (tp[k] - x[k]);
      }
    } else {
      const int j = i - c.n_dense;
      const int sidx = j / 3, axis = j % 3;
      const size_t b = 3 * (size_t)sidx;
      for (int k = 0; k < 3; ++k) x[k] = c.sparse_canon[b + k];
      const double s = sqrt(ws);
      sn[0] = sn[1] = sn[2] = 0.0;
      sn[axis] = s;
      rho = s * ((double)c.sparse_target[b + axis] - x[axis]);
    }
    const double o[3] = {ox, oy, oz};
    const int n[3] = {L.nx, L.ny, L.nz};
    int cc[3];
    for (int k = 0; k < 3; ++k) {
      const double u = (x[k] - o[k]) / (double)L.h;
      double fl = floor(u);
      if (fl < 0.0) fl = 0.0;
      if (fl > (double)(n[k] - 2)) fl = (double)(n[k] - 2);
      cc[k] = (int)fl;
      R.f[(size_t)k * rows + i] = (T)(u - fl);
      R.sn[(size_t)k * rows + i] = (T)sn[k];
    }
    const int cell = cc[0] + (L.nx - 1) * (cc[1] + (L.ny - 1) * cc[2]);
    R.cell[i] = cell;
    R.rho[i] = (T)rho;
    keys[i] = (unsigned)cell;
    vals[i] = i;
  }
}

template <typename T>
hipError_t launch_rows(const RawConstraints& c, const LevelView<T>& L, const RowView<T>& R,
                       const double* o, double wd, double ws, unsigned* keys, int* vals,
                       hipStream_t s) {
  if (R.rows == 0) return hipSuccess;
  int grid = blocks_for(R.rows);
  if (grid > 4096) grid = 4096;
  k_rows<T><<<grid, kBlock, 0, s>>>(c, L, R, o[0], o[1], o[2], wd, ws, keys, vals);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_heads(const unsigned* skeys, int n, int* heads) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    heads[i] = (i == 0 || skeys[i] != skeys[i - 1]) ? 1 : 0;
}

hipError_t launch_heads(const unsigned* skeys, int n, int* heads, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = blocks_for(n);
  if (grid > 4096) grid = 4096;
  k_heads<<<grid, kBlock, 0, s>>>(skeys, n, heads);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_fill_int(int* p, int v, int n) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = v;
}

// Active cells = distinct keys of the sorted rows.  `scan` is the exclusive
// prefix sum of the head flags, i.e. the active index of each head.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_segments(RowView<T> R, const unsigned* skeys,
                                                     const int* scan, int* cell_map, Scalars* sc) {
  const int n = R.rows;
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->n_active = 0;
      R.seg_start[0] = 0;
    }
    return;
  }
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const bool head = (i == 0 || skeys[i] != skeys[i - 1]);
    if (head) {
      const int a = scan[i];
      R.seg_start[a] = i;
      R.active_cell[a] = (int)skeys[i];
      cell_map[skeys[i]] = a;
    }
    if (i == n - 1) {
      const int total = scan[i] + (head ? 1 : 0);
      R.seg_start[total] = n;
      sc->n_active = total;
    }
  }
}

template <typename T>
hipError_t launch_segments(const LevelView<T>& L, const RowView<T>& R, const unsigned* skeys,
                           const int* scan, int* cell_map_w, int ncell, hipStream_t s) {
  int g = blocks_for(ncell);
  if (g > 4096) g = 4096;
  k_fill_int<<<g, kBlock, 0, s>>>(cell_map_w, -1, ncell);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int grid = blocks_for(R.rows > 0 ? R.rows : 1);
  if (grid > 4096) grid = 4096;
  k_segments<T><<<grid, kBlock, 0, s>>>(R, skeys, scan, cell_map_w, L.sc);
  return hipGetLastError();
}

// B^T B and B^T b cached per active cell (Sec. 7.1: "pre-compute and cache").
// Block for corners (a, b): sum over the cell's rows of
// alpha_a alpha_b sn sn^T (symmetric 3x3); rhs block of corner a:
// sum alpha_a sn rho.  One workgroup per cell; rows are staged through LDS
// in chunks of 256 (corner weights computed once per row); each thread owns
// one output entry and accumulates it in float64 over the rows in sorted
// order (deterministic).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_build_cells(RowView<T> R, T* K, const Scalars* sc) {
  constexpr int P = kBlock + 1;  // padded rows: conflict-free column reads
  __shared__ T s_w[8 * P];
  __shared__ T s_sn[3 * P];
  __shared__ T s_rho[kBlock];
  const int n_active = sc->n_active;
  const int rows = R.rows;
  const int j = threadIdx.x;
  int ca = 0, cb = 0, ci = 0, cj = 0, kind = 2;
  if (j < 216) {
    const int p = j / 6, comp = j % 6;
    ca = c_pair_a[p];
    cb = c_pair_b[p];
    ci = c_comp_i[comp];
    cj = c_comp_j[comp];
    kind = 0;
  } else if (j < 240) {
    ca = (j - 216) / 3;
    ci = (j - 216) % 3;
    kind = 1;
  }
  for (int a = blockIdx.x; a < n_active; a += gridDim.x) {
    const int s0 = R.seg_start[a], s1 = R.seg_start[a + 1];
    double acc = 0.0;
    for (int base = s0; base < s1; base += kBlock) {
      const int cnt = min(kBlock, s1 - base);
      __syncthreads();
      if (j < cnt) {
        const int row = R.sorted[base + j];
        const T fx = R.f[row], fy = R.f[(size_t)rows + row], fz = R.f[2 * (size_t)rows + row];
#pragma unroll
        for (int k = 0; k < 8; ++k) s_w[k * P + j] = corner_weight<T>(k, fx, fy, fz);
#pragma unroll
        for (int k = 0; k < 3; ++k) s_sn[k * P + j] = R.sn[(size_t)k * rows + row];
        s_rho[j] = R.rho[row];
      }
      __syncthreads();
      // four independent accumulators keep several LDS reads in flight
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (kind == 0) {
        auto term = [&](int q) {
          return (double)s_w[ca * P + q] * (double)s_w[cb * P + q] *
                 ((double)s_sn[ci * P + q] * (double)s_sn[cj * P + q]);
        };
        int q = 0;
        for (; q + 4 <= cnt; q += 4) {
          a0 += term(q);
          a1 += term(q + 1);
          a2 += term(q + 2);
          a3 += term(q + 3);
        }
        for (; q < cnt; ++q) a0 += term(q);
      } else if (kind == 1) {
        auto term = [&](int q) {
          return (double)s_w[ca * P + q] * ((double)s_sn[ci * P + q] * (double)s_rho[q]);
        };
        int q = 0;
        for (; q + 4 <= cnt; q += 4) {
          a0 += term(q);
          a1 += term(q + 1);
          a2 += term(q + 2);
          a3 += term(q + 3);
        }
        for (; q < cnt; ++q) a0 += term(q);
      }
      acc += (a0 + a1) + (a2 + a3);
    }
    if (kind == 0) {
      const int comp = j % 6;
      K[((size_t)a * 64 + ca * 8 + cb) * 6 + comp] = (T)acc;
      if (ca != cb) K[((size_t)a * 64 + cb * 8 + ca) * 6 + comp] = (T)acc;
    } else if (kind == 1) {
      R.bcell[((size_t)a * 8 + ca) * 3 + ci] = (T)acc;
    }
  }
}

template <typename T>
hipError_t launch_build_cells(const LevelView<T>& L, const RowView<T>& R, T* K, int grid,
                              hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  k_build_cells<T><<<grid, kBlock, 0, s>>>(R, K, L.sc);
  return hipGetLastError();
}

// flags[i] = 1 when node i is a corner of at least one active cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_node_flags(LevelView<T> L, int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const int cnx = L.nx - 1, cny = L.ny - 1, cnz = L.nz - 1;
  int f = 0;
  for (int a = 0; a < 8; ++a) {
    const int cx = x - (a & 1), cy = y - ((a >> 1) & 1), cz = z - (a >> 2);
    if (in_box(cx, cy, cz, cnx, cny, cnz) && L.cell_map[cx + cnx * (cy + cny * cz)] >= 0) f = 1;
  }
  flags[i] = f;
}

template <typename T>
hipError_t launch_node_flags(const LevelView<T>& L, int* flags, hipStream_t s) {
  k_node_flags<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, flags);
  return hipGetLastError();
}

// Per node: the data part of row i of A as a 27-point block stencil,
// A27[delta] = sum over adjacent active cells c (i = corner a of c, neighbour
// = corner b, delta = b - a) of K_c[a][b]; stored SoA [27*6][capA] at the
// node's compact slot.  Also the Jacobi diagonal 2 w_r |N_i| + diag(A27[0]),
// and the data right-hand side b_i gathered from the cells.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_assemble_nodes(LevelView<T> L, RowView<T> R,
                                                           const int* flags, const int* scan,
                                                           int* node_slot, T* A27) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const int nb = (x > 0) + (x < L.nx - 1) + (y > 0) + (y < L.ny - 1) + (z > 0) + (z < L.nz - 1);
  const int cnx = L.nx - 1, cny = L.ny - 1, cnz = L.nz - 1;
  int cells[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int cx = x - (a & 1), cy = y - ((a >> 1) & 1), cz = z - (a >> 2);
    cells[a] = in_box(cx, cy, cz, cnx, cny, cnz) ? L.cell_map[cx + cnx * (cy + cny * cz)] : -1;
  }
  const int slot = flags[i] ? scan[i] : -1;
  node_slot[i] = slot;
  T dg[3] = {T(0), T(0), T(0)};
  T b[3] = {T(0), T(0), T(0)};
  if (slot >= 0) {
    // each adjacent cell's block row K_c[a][*] is read once and scattered
    // into the 27 offsets delta = b - a (summed over a in ascending order)
    T acc[27][6];
#pragma unroll
    for (int dl = 0; dl < 27; ++dl)
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[dl][k] = T(0);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (cells[a] < 0) continue;
      const T* __restrict__ row = L.K + ((size_t)cells[a] * 64 + a * 8) * 6;
#pragma unroll
      for (int bb = 0; bb < 8; ++bb) {
        const int dl = ((bb & 1) - (a & 1) + 1) + 3 * ((((bb >> 1) & 1) - ((a >> 1) & 1) + 1) +
                                                      3 * ((bb >> 2) - (a >> 2) + 1));
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[dl][k] += row[bb * 6 + k];
      }
      const T* bc = R.bcell + ((size_t)cells[a] * 8 + a) * 3;
      b[0] += bc[0];
      b[1] += bc[1];
      b[2] += bc[2];
    }
    const size_t cap = L.capA;
#pragma unroll
    for (int dl = 0; dl < 27; ++dl)
#pragma unroll
      for (int k = 0; k < 6; ++k) A27[(size_t)(dl * 6 + k) * cap + slot] = acc[dl][k];
    dg[0] = acc[13][0];
    dg[1] = acc[13][3];
    dg[2] = acc[13][5];
  }
  const size_t N = L.N;
  const T arap = T(2) * L.wr * T(nb);
  for (int k = 0; k < 3; ++k) {
    const T dk = arap + dg[k];
    L.dinv[k * N + i] = dk > T(0) ? T(1) / dk : T(0);
    L.bnode[k * N + i] = b[k];
  }
}

template <typename T>
hipError_t launch_assemble_nodes(const LevelView<T>& L, const RowView<T>& R, const int* flags,
                                 const int* scan, int* node_slot, T* A27, hipStream_t s) {
  k_assemble_nodes<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, R, flags, scan, node_slot, A27);
  return hipGetLastError();
}

// ===========================================================================
// the normal-equation stencil (Sec. 7.1): A p = J^T J p
// ===========================================================================
//
// A p at node i = 2 w_r sum_{j in N_i} (p_i - p_j)                (ARAP part)
//               + sum_{delta in {-1,0,1}^3} A27_i[delta] p_{i+delta}  (data part)
//
// One workgroup per tile; the tile plus a one-node halo of p is staged in LDS
// (all 27 stencil neighbours of a tile node are in it; nodes outside the
// lattice hold 0 and have zero blocks).  Levels with enough nodes to give
// >= 256 wide tiles use TileW (32x8x4, 4 nodes per thread), others TileS.

int tile_blocks(int kind, int nx, int ny, int nz) {
  auto nb = [&](int tx, int ty, int tz) {
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz);
  };
  switch (kind) {
    case 1: return nb(TileM::TX, TileM::TY, TileM::TZ);
    case 2: return nb(TileW::TX, TileW::TY, TileW::TZ);
    default: return nb(TileS::TX, TileS::TY, TileS::TZ);
  }
}

int default_tile(int nx, int ny, int nz) {
  return tile_blocks(1, nx, ny, nz) >= 512 ? 1 : 0;
}

int update_blocks(int N) { return blocks_for(N); }
int energy_blocks(int cap_rows, int N) { return blocks_for(cap_rows) + blocks_for(N); }

template <typename TL>
struct TilePos {
  int x0, y0, z0;  // lattice coordinates of LDS index (0,0,0) (tile origin - 1)
  __device__ __forceinline__ TilePos(int nx, int ny) {
    const int ntx = (nx + TL::TX - 1) / TL::TX, nty = (ny + TL::TY - 1) / TL::TY;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    x0 = tx * TL::TX - 1;
    y0 = ty * TL::TY - 1;
    z0 = tz * TL::TZ - 1;
  }
  // LDS index of the k-th node owned by this thread
  __device__ __forceinline__ static int own(int k) {
    const int t = threadIdx.x;
    const int lx = t % TL::TX + 1, ly = (t / TL::TX) % TL::TY + 1;
    const int lz = (t / (TL::TX * TL::TY)) * TL::NPT + k + 1;
    return lx + TL::HX * (ly + TL::HY * lz);
  }
};

// A p at the tile node with LDS index c and lattice coordinates (gx,gy,gz).
template <typename T, typename TL>
__device__ __forceinline__ void apply_at(const LevelView<T>& L, const T (*sp)[TL::HALO], int c,
                                         int gx, int gy, int gz, size_t i, T& o0, T& o1,
                                         T& o2) {
  const T p0 = sp[0][c], p1 = sp[1][c], p2 = sp[2][c];
  T l0 = T(0), l1 = T(0), l2 = T(0);
  const int off[3] = {1, TL::HX, TL::HX * TL::HY};
  const int pos[3] = {gx, gy, gz};
  const int lim[3] = {L.nx, L.ny, L.nz};
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
  const int slot = L.node_slot[i];
  if (slot >= 0) {
    const size_t cap = L.capA;
    const T* __restrict__ A = L.A27 + slot;
#pragma unroll
    for (int dl = 0; dl < 27; ++dl) {
      const int ddx = dl % 3 - 1, ddy = (dl / 3) % 3 - 1, ddz = dl / 9 - 1;
      const int q = c + ddx + TL::HX * (ddy + TL::HY * ddz);
      const T* __restrict__ blk = A + (size_t)dl * 6 * cap;
      const T s0 = blk[0], s1 = blk[cap], s2 = blk[2 * cap], s3 = blk[3 * cap],
              s4 = blk[4 * cap], s5 = blk[5 * cap];
      const T q0 = sp[0][q], q1 = sp[1][q], q2 = sp[2][q];
      o0 += s0 * q0 + s1 * q1 + s2 * q2;
      o1 += s1 * q0 + s3 * q1 + s4 * q2;
      o2 += s2 * q0 + s4 * q1 + s5 * q2;
    }
  }
}

// kModeRhs : p = d; g = A d - b + w_r sum_j (2I - R_i - R_j) e_ij is the
//            gradient J^T r; r = -g is stored (the CG residual r_0).
// kModeApply / kModeGrad : A p or g written to `out` (test entry points).
template <typename T, typename TL, int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil(LevelView<T> L, const T* __restrict__ pin,
                                                    T* __restrict__ out) {
  __shared__ T sp[3][TL::HALO];
  const TilePos<TL> t(L.nx, L.ny);
  const size_t N = L.N;
  const T* __restrict__ src = (MODE == kModeRhs) ? L.d : pin;
  for (int k = threadIdx.x; k < TL::HALO; k += kBlock) {
    const int lx = k % TL::HX, ly = (k / TL::HX) % TL::HY, lz = k / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    T v0 = T(0), v1 = T(0), v2 = T(0);
    if (in_box(gx, gy, gz, L.nx, L.ny, L.nz)) {
      const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
      v0 = src[i];
      v1 = src[N + i];
      v2 = src[2 * N + i];
    }
    sp[0][k] = v0;
    sp[1][k] = v1;
    sp[2][k] = v2;
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    if (!in_box(gx, gy, gz, L.nx, L.ny, L.nz)) continue;
    const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
    T o0, o1, o2;
    apply_at<T, TL>(L, sp, c, gx, gy, gz, i, o0, o1, o2);
    if (MODE == kModeApply) {
      out[i] = o0;
      out[N + i] = o1;
      out[2 * N + i] = o2;
      continue;
    }
    // rotation part of the ARAP gradient: for neighbour j = i + s*axis,
    // e_ij = -s h axis and (2I - R_i - R_j) e_ij = -s h (2 axis - R_i[:,k] - R_j[:,k]).
    const T* __restrict__ rot = L.rot;
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
    const T g0 = o0 - L.bnode[i] + L.wr * q0;
    const T g1 = o1 - L.bnode[N + i] + L.wr * q1;
    const T g2 = o2 - L.bnode[2 * N + i] + L.wr * q2;
    T* __restrict__ dst = (MODE == kModeGrad) ? out : L.r;
    const T sg = (MODE == kModeGrad) ? T(1) : T(-1);
    dst[i] = sg * g0;
    dst[N + i] = sg * g1;
    dst[2 * N + i] = sg * g2;
  }
}

template <typename T, typename TL>
hipError_t launch_stencil_t(int mode, const LevelView<T>& L, const T* pin, T* out, hipStream_t s) {
  const int grid = tile_blocks(L.tile, L.nx, L.ny, L.nz);
  switch (mode) {
    case kModeRhs:
      k_stencil<T, TL, kModeRhs><<<grid, kBlock, 0, s>>>(L, pin, out);
      break;
    case kModeApply:
      k_stencil<T, TL, kModeApply><<<grid, kBlock, 0, s>>>(L, pin, out);
      break;
    case kModeGrad:
      k_stencil<T, TL, kModeGrad><<<grid, kBlock, 0, s>>>(L, pin, out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(int mode, const LevelView<T>& L, const T* pin, T* out, hipStream_t s) {
  switch (L.tile) {
    case 1: return launch_stencil_t<T, TileM>(mode, L, pin, out, s);
    case 2: return launch_stencil_t<T, TileW>(mode, L, pin, out, s);
    default: return launch_stencil_t<T, TileS>(mode, L, pin, out, s);
  }
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
// d += alpha p_{m-1} to its own nodes, computes Ap_m and writes S_m.  The
// last iteration's step is applied by k_cg_final.  The halo inputs are
// loaded before the scalar reduction so that both latencies overlap.

template <typename T>
__device__ __forceinline__ void cg_scalars(const double* s, int n, T& alpha, T& beta,
                                           Scalars* sc) {
  double v[4];
  sum_partials_k<4>(s, n, v);
  const double rz = v[0], pap = v[1], apdr = v[2], apdap = v[3];
  const double a = pap > 0.0 ? rz / pap : 0.0;
  double rz_new = rz - 2.0 * a * apdr + a * a * apdap;
  if (rz_new < 0.0) rz_new = 0.0;
  alpha = (T)a;
  beta = rz > 0.0 ? (T)(rz_new / rz) : T(0);
  if (blockIdx.x == 0 && threadIdx.x == 0 && !(pap > 0.0)) sc->guard_hits += 1;
}

template <typename T, typename TL, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_cg(LevelView<T> L, CgIo<T> io) {
  __shared__ T sp[3][TL::HALO];
  __shared__ T sr[3][TL::HALO];
  const TilePos<TL> t(L.nx, L.ny);
  const size_t N = L.N;
  const T* __restrict__ r_in = io.r_in;
  const T* __restrict__ p_in = io.p_in;
  const T* __restrict__ ap_in = io.ap_in;
  const T* __restrict__ dinv = L.dinv;
  // 1. halo inputs into registers
  T hr[TL::HPT][3], hq[TL::HPT][3], hp[TL::HPT][3], ha[TL::HPT][3];
  size_t hi[TL::HPT];
  bool hin[TL::HPT];
#pragma unroll
  for (int h = 0; h < TL::HPT; ++h) {
    const int k = threadIdx.x + h * kBlock;
    const int lx = k % TL::HX, ly = (k / TL::HX) % TL::HY, lz = k / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    hin[h] = k < TL::HALO && in_box(gx, gy, gz, L.nx, L.ny, L.nz);
    hi[h] = hin[h] ? gx + (size_t)L.nx * (gy + (size_t)L.ny * gz) : 0;
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
  // 2. CG scalars of the previous iterate
  T alpha = T(0), beta = T(0);
  if (!FIRST) cg_scalars<T>(io.s_in, io.n_in, alpha, beta, L.sc);
  // 3. r_m, p_m into LDS; own nodes also store r_m, p_m and step d
#pragma unroll
  for (int h = 0; h < TL::HPT; ++h) {
    const int k = threadIdx.x + h * kBlock;
    if (k >= TL::HALO) continue;
    T p3[3], r3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T r = hr[h][a];
      if (!FIRST) r -= alpha * ha[h][a];
      T p = hq[h][a] * r;
      if (!FIRST) p += beta * hp[h][a];
      r3[a] = r;
      p3[a] = p;
      sp[a][k] = p;
      sr[a][k] = r;
    }
    const int lx = k % TL::HX, ly = (k / TL::HX) % TL::HY, lz = k / (TL::HX * TL::HY);
    if (hin[h] && lx >= 1 && lx <= TL::TX && ly >= 1 && ly <= TL::TY && lz >= 1 &&
        lz <= TL::TZ) {
      T* __restrict__ d = L.d;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = a * N + hi[h];
        io.p_out[j] = p3[a];
        if (!FIRST) {
          io.r_out[j] = r3[a];
          d[j] += alpha * hp[h][a];
        }
      }
    }
  }
  __syncthreads();
  // 4. A p_m on own nodes and the block partials of S_m
  double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < TL::NPT; ++kk) {
    const int c = TilePos<TL>::own(kk);
    const int lx = c % TL::HX, ly = (c / TL::HX) % TL::HY, lz = c / (TL::HX * TL::HY);
    const int gx = t.x0 + lx, gy = t.y0 + ly, gz = t.z0 + lz;
    if (!in_box(gx, gy, gz, L.nx, L.ny, L.nz)) continue;
    const size_t i = gx + (size_t)L.nx * (gy + (size_t)L.ny * gz);
    T o[3];
    apply_at<T, TL>(L, sp, c, gx, gy, gz, i, o[0], o[1], o[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t j = a * N + i;
      io.ap_out[j] = o[a];
      const double q = (double)dinv[j], r = (double)sr[a][c], p = (double)sp[a][c];
      const double ap = (double)o[a];
      part[0] += r * q * r;
      part[1] += p * ap;
      part[2] += ap * q * r;
      part[3] += ap * q * ap;
    }
  }
  write_block_partials<4>(part, io.s_out, gridDim.x);
}

// d += alpha p of the last CG iterate.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_final(LevelView<T> L, const T* __restrict__ p,
                                                     const double* s, int n) {
  T alpha, beta;
  cg_scalars<T>(s, n, alpha, beta, L.sc);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const size_t N = L.N;
  T* __restrict__ d = L.d;
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a * N + i] += alpha * p[a * N + i];
}

template <typename T, typename TL>
void launch_cg_t(bool first, const LevelView<T>& L, const CgIo<T>& io, hipStream_t s) {
  const int grid = tile_blocks(L.tile, L.nx, L.ny, L.nz);
  if (first) k_cg<T, TL, true><<<grid, kBlock, 0, s>>>(L, io);
  else k_cg<T, TL, false><<<grid, kBlock, 0, s>>>(L, io);
}

template <typename T>
hipError_t launch_cg(bool first, const LevelView<T>& L, const CgIo<T>& io, hipStream_t s) {
  switch (L.tile) {
    case 1: launch_cg_t<T, TileM>(first, L, io, s); break;
    case 2: launch_cg_t<T, TileW>(first, L, io, s); break;
    default: launch_cg_t<T, TileS>(first, L, io, s); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_final(const LevelView<T>& L, const T* p, const double* s_last, int n,
                           hipStream_t st) {
  k_cg_final<T><<<blocks_for(L.N), kBlock, 0, st>>>(L, p, s_last, n);
  return hipGetLastError();
}

// ===========================================================================
// energy, eq. (1): rows (dense and sparse) and ARAP edges, float64 sums
// ===========================================================================

template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy(LevelView<T> L, RowView<T> R, int row_blocks,
                                                   double* part_out) {
  double part[3] = {0.0, 0.0, 0.0};
  const size_t N = L.N;
  const T* __restrict__ d = L.d;
  if ((int)blockIdx.x < row_blocks) {
    const int row = blockIdx.x * kBlock + threadIdx.x;
    const int rows = L.sc->rows;
    if (row < rows) {
      const int cell = R.cell[row];
      const int cnx = L.nx - 1, cny = L.ny - 1;
      const int cx = cell % cnx, cy = (cell / cnx) % cny, cz = cell / (cnx * cny);
      const T fx = R.f[row], fy = R.f[(size_t)rows + row], fz = R.f[2 * (size_t)rows + row];
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t m = (cx + (k & 1)) + (size_t)L.nx * ((cy + ((k >> 1) & 1)) +
                                                          (size_t)L.ny * (cz + (k >> 2)));
        const T w = corner_weight<T>(k, fx, fy, fz);
        s0 += w * d[m];
        s1 += w * d[N + m];
        s2 += w * d[2 * N + m];
      }
      const T res = R.sn[row] * s0 + R.sn[(size_t)rows + row] * s1 +
                    R.sn[2 * (size_t)rows + row] * s2 - R.rho[row];
      const double e = (double)res * (double)res;
      if (row < L.sc->n_dense) part[0] = e; else part[1] = e;
    }
  } else {
    const int i = (blockIdx.x - row_blocks) * kBlock + threadIdx.x;
    if (i < L.N) {
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
  write_block_partials<3>(part, part_out, gridDim.x);
}

// One block: sums the energy partials into sc->energy (and the trace).
__global__ __launch_bounds__(kBlock) void k_energy_finalize(Scalars* sc, const double* part,
                                                            int n, int record_trace) {
  const double e_dense = sum_partials(part, n);
  const double e_sparse = sum_partials(part + n, n);
  const double e_reg = sum_partials(part + 2 * (size_t)n, n);
  if (threadIdx.x == 0) {
    sc->energy[0] = e_dense + e_sparse + e_reg;
    sc->energy[1] = e_dense;
    sc->energy[2] = e_sparse;
    sc->energy[3] = e_reg;
    if (record_trace && sc->n_trace < VD_MAX_TRACE) {
      sc->trace[sc->n_trace] = sc->energy[0];
      sc->n_trace += 1;
    }
  }
}

template <typename T>
hipError_t launch_energy(const LevelView<T>& L, const RowView<T>& R, int cap_rows,
                         double* part, int record_trace, hipStream_t s) {
  const int rb = blocks_for(cap_rows);
  const int nb = energy_blocks(cap_rows, L.N);
  k_energy<T><<<nb, kBlock, 0, s>>>(L, R, rb, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_energy_finalize<<<1, kBlock, 0, s>>>(L.sc, part, nb, record_trace);
  return hipGetLastError();
}

__global__ void k_reset_counters(Scalars* sc, int rows, int n_dense, int clear_trace) {
  if (threadIdx.x != 0) return;
  sc->guard_hits = 0;
  sc->polar_fp64 = 0;
  sc->polar_keep = 0;
  if (clear_trace) sc->n_trace = 0;
  if (rows >= 0) sc->rows = rows;
  if (n_dense >= 0) sc->n_dense = n_dense;
}

hipError_t launch_reset_counters(Scalars* sc, int rows, int n_dense, int clear_trace,
                                 hipStream_t s) {
  k_reset_counters<<<1, 64, 0, s>>>(sc, rows, n_dense, clear_trace);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const float* v, int64_t n, int* flags) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    if (!isfinite(v[i])) bad = 1;
  if (bad) atomicOr(flags, 1);
}

hipError_t launch_check_finite(const float* v, int64_t n, int* flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  k_check_finite<<<(unsigned)g, kBlock, 0, s>>>(v, n, flags);
  return hipGetLastError();
}

// ===========================================================================
// rotation step (Sec. 7.1): M_i = sum_j (t_i - t_j)(t_hat_i - t_hat_j)^T
// ===========================================================================

template <typename T>
__global__ __launch_bounds__(kBlock) void k_polar(LevelView<T> L, const T* __restrict__ d,
                                                  const T* rot_prev, T* rot_out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const size_t N = L.N;
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
  for (int k = 0; k < 9; ++k) Rp[k] = rot_prev[(size_t)k * N + i];
  const int code = fit_or_keep<T>(M, Rp, R);
#pragma unroll
  for (int k = 0; k < 9; ++k) rot_out[(size_t)k * N + i] = R[k];
  if (code == kFitFp64) atomicAdd(&L.sc->polar_fp64, 1);
  if (code == kFitKeep) atomicAdd(&L.sc->polar_keep, 1);
}

template <typename T>
hipError_t launch_polar(const LevelView<T>& L, const T* d_in, const T* rot_prev, T* rot_out,
                        hipStream_t s) {
  k_polar<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, d_in, rot_prev, rot_out);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fit_batch(const float* M, const float* Rp, float* R,
                                                      int* keep, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T m[9], rp[9], r[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    m[k] = (T)M[9 * i + k];
    rp[k] = Rp ? (T)Rp[9 * i + k] : ((k % 4 == 0) ? T(1) : T(0));
  }
  const int code = fit_or_keep<T>(m, rp, r);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[9 * i + k] = (float)r[k];
  if (keep) keep[i] = code;
}

template <typename T>
hipError_t launch_fit_batch(const float* M, const float* R_prev, float* R, int* keep, int64_t n,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fit_batch<T><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(M, R_prev, R, keep, n);
  return hipGetLastError();
}

// ===========================================================================
// level transfers (Sec. 7.2)
// ===========================================================================

// Level node (a,b,c) takes the finest node stride*(a,b,c): d, base and R.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inject(LevelView<T> F, LevelView<T> Lv, int stride) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Lv.N) return;
  const int x = i % Lv.nx, y = (i / Lv.nx) % Lv.ny, z = i / (Lv.nx * Lv.ny);
  const size_t f = (size_t)x * stride + (size_t)F.nx * ((size_t)y * stride + (size_t)F.ny * z * stride);
  const size_t N = Lv.N, NF = F.N;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T v = F.d[k * NF + f];
    Lv.d[k * N + i] = v;
    Lv.base[k * N + i] = v;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Lv.rot[k * N + i] = F.rot[k * NF + f];
}

template <typename T>
hipError_t launch_inject(const LevelView<T>& fine, const LevelView<T>& lvl, int stride,
                         hipStream_t s) {
  k_inject<T><<<blocks_for(lvl.N), kBlock, 0, s>>>(fine, lvl, stride);
  return hipGetLastError();
}

// fine_out (+)= trilinear evaluation of (coarse_in - coarse_base) at the fine
// rest positions: fine node a sits at coarse coordinate a/2; its cell is
// clamped to the last coarse cell, so the last fine plane of an even-sized
// axis is linearly extrapolated (f = 1.5).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelView<T> C, LevelView<T> Fl,
                                                    const T* __restrict__ cin,
                                                    const T* __restrict__ cbase, T* fout,
                                                    int add) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Fl.N) return;
  const int x = i % Fl.nx, y = (i / Fl.nx) % Fl.ny, z = i / (Fl.nx * Fl.ny);
  const int p[3] = {x, y, z};
  const int nc[3] = {C.nx, C.ny, C.nz};
  int cc[3];
  T f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int c = p[k] >> 1;
    if (c > nc[k] - 2) c = nc[k] - 2;
    cc[k] = c;
    f[k] = T(0.5) * T(p[k]) - T(c);
  }
  const size_t NC = C.N, NF = Fl.N;
  T v[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const size_t m = (cc[0] + (k & 1)) +
                     (size_t)C.nx * ((cc[1] + ((k >> 1) & 1)) + (size_t)C.ny * (cc[2] + (k >> 2)));
    const T w = corner_weight<T>(k, f[0], f[1], f[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T inc = cbase ? cin[a * NC + m] - cbase[a * NC + m] : cin[a * NC + m];
      v[a] += w * inc;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (add) fout[a * NF + i] += v[a];
    else fout[a * NF + i] = v[a];
  }
}

template <typename T>
hipError_t launch_prolong_add(const LevelView<T>& coarse, const LevelView<T>& fine,
                              const T* coarse_in, const T* coarse_base, T* fine_out, int add,
                              hipStream_t s) {
  k_prolong<T><<<blocks_for(fine.N), kBlock, 0, s>>>(coarse, fine, coarse_in, coarse_base,
                                                      fine_out, add);
  return hipGetLastError();
}

// ===========================================================================
// state helpers
// ===========================================================================

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_rest(LevelView<T> L) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const size_t N = L.N;
#pragma unroll
  for (int k = 0; k < 3; ++k) L.d[k * N + i] = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) L.rot[k * N + i] = (k % 4 == 0) ? T(1) : T(0);
}

template <typename T>
hipError_t launch_set_rest(const LevelView<T>& L, hipStream_t s) {
  k_set_rest<T><<<blocks_for(L.N), kBlock, 0, s>>>(L);
  return hipGetLastError();
}

// dir 0: export positions t = t_hat + d (AoS float) and rotations (row-major
// AoS float); dir 1: import them (non-finite input sets flags bit 1).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_state_io(LevelView<T> L, double ox, double oy,
                                                     double oz, float* pos, float* rot,
                                                     const float* pos_in, const float* rot_in,
                                                     int dir, int* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const size_t N = L.N;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const double rest[3] = {ox + (double)L.h * x, oy + (double)L.h * y, oz + (double)L.h * z};
  if (dir == 0) {
    if (pos) {
#pragma unroll
      for (int k = 0; k < 3; ++k) pos[3 * (size_t)i + k] = (float)(rest[k] + (double)L.d[k * N + i]);
    }
    if (rot) {
#pragma unroll
      for (int k = 0; k < 9; ++k) rot[9 * (size_t)i + k] = (float)L.rot[k * N + i];
    }
  } else {
    int bad = 0;
    if (pos_in) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float v = pos_in[3 * (size_t)i + k];
        if (!isfinite(v)) bad = 1;
        L.d[k * N + i] = (T)((double)v - rest[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float v = rot_in ? rot_in[9 * (size_t)i + k] : ((k % 4 == 0) ? 1.0f : 0.0f);
      if (!isfinite(v)) bad = 1;
      L.rot[k * N + i] = (T)v;
    }
    if (bad) atomicOr(flags, 1);
  }
}

template <typename T>
hipError_t launch_state_io(const LevelView<T>& L, const double* o, float* pos, float* rot,
                           const float* pos_in, const float* rot_in, int dir, int* flags,
                           hipStream_t s) {
  k_state_io<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, o[0], o[1], o[2], pos, rot, pos_in, rot_in,
                                                    dir, flags);
  return hipGetLastError();
}

// AoS float xyz <-> SoA T (used by the test entry points)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_convert(const float* in, T* out, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) out[(size_t)k * n + i] = (T)in[3 * (size_t)i + k];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_convert_back(const T* in, float* out, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) out[3 * (size_t)i + k] = (float)in[(size_t)k * n + i];
}
template <typename T>
hipError_t launch_convert(const float* in, T* out, int n, hipStream_t s) {
  k_convert<T><<<blocks_for(n), kBlock, 0, s>>>(in, out, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_convert_back(const T* in, float* out, int n, hipStream_t s) {
  k_convert_back<T><<<blocks_for(n), kBlock, 0, s>>>(in, out, n);
  return hipGetLastError();
}

// ---- explicit instantiations -----------------------------------------------
#define VD_INSTANTIATE(T)                                                                        \
  template hipError_t launch_rows<T>(const RawConstraints&, const LevelView<T>&,                \
                                     const RowView<T>&, const double*, double, double,          \
                                     unsigned*, int*, hipStream_t);                             \
  template hipError_t launch_segments<T>(const LevelView<T>&, const RowView<T>&,                \
                                         const unsigned*, const int*, int*, int, hipStream_t);  \
  template hipError_t launch_build_cells<T>(const LevelView<T>&, const RowView<T>&, T*, int,    \
                                            hipStream_t);                                       \
  template hipError_t launch_assemble_nodes<T>(const LevelView<T>&, const RowView<T>&,          \
                                               const int*, const int*, int*, T*, hipStream_t);  \
  template hipError_t launch_node_flags<T>(const LevelView<T>&, int*, hipStream_t);             \
  template hipError_t launch_stencil<T>(int, const LevelView<T>&, const T*, T*, hipStream_t);   \
  template hipError_t launch_cg<T>(bool, const LevelView<T>&, const CgIo<T>&, hipStream_t);     \
  template hipError_t launch_cg_final<T>(const LevelView<T>&, const T*, const double*, int,     \
                                         hipStream_t);                                          \
  template hipError_t launch_energy<T>(const LevelView<T>&, const RowView<T>&, int, double*,    \
                                       int, hipStream_t);                                       \
  template hipError_t launch_polar<T>(const LevelView<T>&, const T*, const T*, T*, hipStream_t); \
  template hipError_t launch_inject<T>(const LevelView<T>&, const LevelView<T>&, int,           \
                                       hipStream_t);                                            \
  template hipError_t launch_prolong_add<T>(const LevelView<T>&, const LevelView<T>&,           \
                                            const T*, const T*, T*, int, hipStream_t);          \
  template hipError_t launch_set_rest<T>(const LevelView<T>&, hipStream_t);                     \
  template hipError_t launch_state_io<T>(const LevelView<T>&, const double*, float*, float*,    \
                                         const float*, const float*, int, int*, hipStream_t);   \
  template hipError_t launch_convert<T>(const float*, T*, int, hipStream_t);                    \
  template hipError_t launch_convert_back<T>(const T*, float*, int, hipStream_t);               \
  template hipError_t launch_fit_batch<T>(const float*, const float*, float*, int*, int64_t,    \
                                          hipStream_t);

VD_INSTANTIATE(float)
VD_INSTANTIATE(double)

}  // namespace vd
