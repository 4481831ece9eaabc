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

// B^T B and B^T b cached per active cell (the per-voxel cache of Sec. 7.1).
// Block for corners (a, b): sum over the cell's rows of
// alpha_a alpha_b sn sn^T (symmetric 3x3); rhs block of corner a:
// sum alpha_a sn rho.  One workgroup per cell; rows are staged through LDS in
// chunks of 256 as the float64 products u[3a + i] = alpha_a sn_i and rho (a
// product of two floats is exact in float64, so u_ai u_bj is the same number
// as (alpha_a alpha_b)(sn_i sn_j)); each thread owns one output entry and
// accumulates it in float64 over the rows in sorted order (deterministic).
// While a chunk is accumulated, the next chunk's rows and the row indices of
// the one after are already being loaded (cells of coarse levels hold
// thousands of rows).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_build_cells(RowView<T> R, T* K, const Scalars* sc) {
  constexpr int P = kBlock + 1;  // padded rows: conflict-free column reads
  __shared__ double s_u[25 * P];  // 24 products alpha_a sn_i, then rho
  const int n_active = sc->n_active;
  const int rows = R.rows;
  const int j = threadIdx.x;
  int ka = 0, kb = 0, ca = 0, ci = 0, kind = 2;
  if (j < 216) {
    const int p = j / 6, comp = j % 6;
    ca = c_pair_a[p];
    ci = c_comp_i[comp];
    ka = ca * 3 + ci;
    kb = c_pair_b[p] * 3 + c_comp_j[comp];
    kind = 0;
  } else if (j < 240) {
    ca = (j - 216) / 3;
    ci = (j - 216) % 3;
    ka = ca * 3 + ci;
    kb = 24;
    kind = 1;
  }
  for (int a = blockIdx.x; a < n_active; a += gridDim.x) {
    const int s0 = R.seg_start[a], s1 = R.seg_start[a + 1];
    // row of this thread in the chunk being staged (f, sn, rho) and the row
    // index of the following chunk
    int row_next = (s0 + kBlock + j < s1) ? R.sorted[s0 + kBlock + j] : 0;
    T f3[3] = {T(0), T(0), T(0)}, n3[3] = {T(0), T(0), T(0)}, rho = T(0);
    if (s0 + j < s1) {
      const int row = R.sorted[s0 + j];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        f3[k] = R.f[(size_t)k * rows + row];
        n3[k] = R.sn[(size_t)k * rows + row];
      }
      rho = R.rho[row];
    }
    double acc = 0.0;
    for (int base = s0; base < s1; base += kBlock) {
      const int cnt = min(kBlock, s1 - base);
      __syncthreads();  // the previous chunk's reads are done
      if (j < cnt) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const double w = (double)corner_weight<T>(c, f3[0], f3[1], f3[2]);
#pragma unroll
          for (int k = 0; k < 3; ++k) s_u[(c * 3 + k) * P + j] = w * (double)n3[k];
        }
        s_u[24 * P + j] = (double)rho;
      }
      __syncthreads();
      // next chunk's rows (index loaded one chunk ago), and the index after
      if (base + kBlock + j < s1) {
        const int row = row_next;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          f3[k] = R.f[(size_t)k * rows + row];
          n3[k] = R.sn[(size_t)k * rows + row];
        }
        rho = R.rho[row];
      }
      row_next = (base + 2 * kBlock + j < s1) ? R.sorted[base + 2 * kBlock + j] : 0;
      // four independent accumulators keep several LDS reads in flight
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (kind < 2) {
        const double* __restrict__ ua = s_u + ka * P;
        const double* __restrict__ ub = s_u + kb * P;
        int q = 0;
        // unrolled so that 16 rows' LDS reads are in flight at once (one wave
        // per SIMD: nothing else hides their latency); each accumulator still
        // adds its rows in row order
#pragma unroll 4
        for (; q + 4 <= cnt; q += 4) {
          a0 += ua[q] * ub[q];
          a1 += ua[q + 1] * ub[q + 1];
          a2 += ua[q + 2] * ub[q + 2];
          a3 += ua[q + 3] * ub[q + 3];
        }
        for (; q < cnt; ++q) a0 += ua[q] * ub[q];
      }
      acc += (a0 + a1) + (a2 + a3);
    }
    if (kind == 0) {
      const int comp = j % 6, cb = c_pair_b[j / 6];
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
// = corner b, delta = b - a) of K_c[a][b]; stored at the node's compact slot
// as a row A27r[slot][kA27Row]: three parts by dz (one part is one lane's
// share of the node in the stencil and CG kernels), interleaved by 16-byte
// chunks.  Also the
// Jacobi diagonal 2 w_r |N_i| + diag(A27[0]), and the data right-hand side
// b_i gathered from the cells.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_assemble_nodes(LevelView<T> L, RowView<T> R,
                                                           const int* flags, const int* scan,
                                                           int* node_slot, T* A27r) {
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
    // entry q of part m (block (dx, dy) of dz = m - 1, zero padded) at chunk
    // 3 (q / CW) + m, position q % CW
    constexpr int CW = 16 / (int)sizeof(T);
    T* __restrict__ row_out = A27r + (size_t)slot * kA27Row;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int q = 0; q < kA27Part; ++q)
        row_out[(3 * (q / CW) + m) * CW + q % CW] = q < 54 ? acc[m * 9 + q / 6][q % 6] : T(0);
    dg[0] = acc[13][0];
    dg[1] = acc[13][3];
    dg[2] = acc[13][5];
  }
  const size_t N = L.N;
  T arap = T(2) * L.wr * T(nb);
  bool in_set = true;
  if (L.act) {
    // restricted to M: only the edges inside M count, so the ARAP diagonal
    // is 2 w_r |N_i and M|; points outside M are not unknowns (D^-1 = 0)
    in_set = L.act[i] != 0;
    int w = 0;
    const size_t st[3] = {1, (size_t)L.nx, (size_t)L.nx * L.ny};
    const int pos[3] = {x, y, z};
    const int lim[3] = {L.nx, L.ny, L.nz};
    for (int ax = 0; ax < 3; ++ax) {
      if (pos[ax] > 0) w += L.act[i - st[ax]];
      if (pos[ax] < lim[ax] - 1) w += L.act[i + st[ax]];
    }
    arap = T(2) * L.wr * T(w);
  }
  for (int k = 0; k < 3; ++k) {
    const T dk = arap + dg[k];
    L.dinv[k * N + i] = (in_set && dk > T(0)) ? T(1) / dk : T(0);
    L.bnode[k * N + i] = b[k];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dilate(LevelView<T> L, const int* flags,
                                                   unsigned char* act) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const size_t st[3] = {1, (size_t)L.nx, (size_t)L.nx * L.ny};
  const int pos[3] = {x, y, z};
  const int lim[3] = {L.nx, L.ny, L.nz};
  int f = flags[i];
  for (int ax = 0; ax < 3; ++ax) {
    if (pos[ax] > 0) f |= flags[i - st[ax]];
    if (pos[ax] < lim[ax] - 1) f |= flags[i + st[ax]];
  }
  act[i] = f ? 1 : 0;
}

template <typename T>
hipError_t launch_dilate(const LevelView<T>& L, const int* flags, unsigned char* act,
                         hipStream_t s) {
  k_dilate<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, flags, act);
  return hipGetLastError();
}

// Grid growth, one layer (Sec. 8: points that join M for the first time are
// initialised by extrapolating the deformation field).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_grow_layer(LevelView<T> L, const unsigned char* act,
                                                       const unsigned char* known, T* tmp_d,
                                                       T* tmp_r, unsigned char* fresh,
                                                       int* count) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  fresh[i] = 0;
  if (!act[i] || known[i]) return;
  const size_t N = L.N;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const size_t st[3] = {1, (size_t)L.nx, (size_t)L.nx * L.ny};
  const int pos[3] = {x, y, z};
  const int lim[3] = {L.nx, L.ny, L.nz};
  double acc[3] = {0.0, 0.0, 0.0};
  int cnt = 0;
  long first = -1;
  for (int ax = 0; ax < 3; ++ax) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      const int pj = pos[ax] + sgn;
      if (pj < 0 || pj >= lim[ax]) continue;
      const size_t j = sgn > 0 ? i + st[ax] : i - st[ax];
      if (!known[j]) continue;
      for (int k = 0; k < 3; ++k) acc[k] += (double)L.d[k * N + j];
      ++cnt;
      if (first < 0) first = (long)j;
    }
  }
  if (!cnt) return;
  for (int k = 0; k < 3; ++k) tmp_d[k * N + i] = (T)(acc[k] / cnt);
  for (int k = 0; k < 9; ++k) tmp_r[k * N + i] = L.rot[k * N + (size_t)first];
  fresh[i] = 1;
  atomicAdd(count, 1);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_grow_commit(LevelView<T> L, const T* tmp_d,
                                                        const T* tmp_r, unsigned char* fresh,
                                                        unsigned char* known) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N || !fresh[i]) return;
  const size_t N = L.N;
  for (int k = 0; k < 3; ++k) L.d[k * N + i] = tmp_d[k * N + i];
  for (int k = 0; k < 9; ++k) L.rot[k * N + i] = tmp_r[k * N + i];
  known[i] = 1;
  fresh[i] = 0;
}

template <typename T>
hipError_t launch_grow_layer(const LevelView<T>& L, const unsigned char* act,
                             const unsigned char* known, T* tmp_d, T* tmp_r,
                             unsigned char* fresh, int* count, hipStream_t s) {
  k_grow_layer<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, act, known, tmp_d, tmp_r, fresh, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_grow_commit(const LevelView<T>& L, const T* tmp_d, const T* tmp_r,
                              unsigned char* fresh, unsigned char* known, hipStream_t s) {
  k_grow_commit<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, tmp_d, tmp_r, fresh, known);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_assemble_nodes(const LevelView<T>& L, const RowView<T>& R, const int* flags,
                                 const int* scan, int* node_slot, T* A27r, hipStream_t s) {
  k_assemble_nodes<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, R, flags, scan, node_slot, A27r);
  return hipGetLastError();
}

// Rows / dense-row counts of the current frame (read by the energy kernel).
__global__ void k_set_counts(Scalars* sc, int rows, int n_dense) {
  if (threadIdx.x == 0) {
    sc->rows = rows;
    sc->n_dense = n_dense;
  }
}

hipError_t launch_set_counts(Scalars* sc, int rows, int n_dense, hipStream_t s) {
  k_set_counts<<<1, 64, 0, s>>>(sc, rows, n_dense);
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
// batched rotation fit of raw matrices (test entry point)
// ===========================================================================

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
// state helpers
// ===========================================================================

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

// Finest state as float64 AoS: positions t_hat + d, rotations row-major.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_state_out64(LevelView<T> L, double ox, double oy,
                                                        double oz, double* pos, double* rot) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  const size_t N = L.N;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const double rest[3] = {ox + (double)L.h * x, oy + (double)L.h * y, oz + (double)L.h * z};
  if (pos) {
#pragma unroll
    for (int k = 0; k < 3; ++k) pos[3 * (size_t)i + k] = rest[k] + (double)L.d[k * N + i];
  }
  if (rot) {
#pragma unroll
    for (int k = 0; k < 9; ++k) rot[9 * (size_t)i + k] = (double)L.rot[k * N + i];
  }
}

template <typename T>
hipError_t launch_state_out64(const LevelView<T>& L, const double* o, double* pos, double* rot,
                              hipStream_t s) {
  k_state_out64<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, o[0], o[1], o[2], pos, rot);
  return hipGetLastError();
}

// AoS float xyz <-> SoA T (used by the test entry points)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_delta(T* d, const float* delta, T h, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) d[i] += h * (T)delta[i];
}

template <typename T>
hipError_t launch_add_delta(T* d, const float* delta, double h, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_add_delta<T><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(d, delta, (T)h, n);
  return hipGetLastError();
}

// Exact step of a warm start along its predicted direction v (not in the
// paper): with the rotations fixed E is quadratic in the displacement,
// E(d + b v) = E(d) + 2 b g.v + b^2 v.Av with g = J^T r and A = J^T J
// (Sec. 7.1), smallest at b = -g.v / v.Av.  k_warm_dots writes the block
// partials of g.v and v.Av in float64; k_warm_step re-reduces them in every
// block in the same order and applies d += b v (b = 0 when v.Av <= 0).
constexpr int kWarmDotBlocks = 1024;  // partial pairs at most (the caller's buffer)

template <typename T>
__global__ __launch_bounds__(kBlock) void k_warm_dots(const T* __restrict__ g,
                                                      const float* __restrict__ v,
                                                      const T* __restrict__ av, int64_t n,
                                                      double* part) {
  double acc[2] = {0.0, 0.0};
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kBlock) {
    const double vk = (double)v[k];
    acc[0] += (double)g[k] * vk;
    acc[1] += (double)av[k] * vk;
  }
  write_block_partials<2>(acc, part, gridDim.x);
}

// act (null: every point): with the optimised set M only its points move.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_warm_step(T* d, const float* __restrict__ v,
                                                      int64_t n, const double* part,
                                                      int nblocks,
                                                      const unsigned char* __restrict__ act,
                                                      int64_t N) {
  double s[2];
  sum_partials_k<2>(part, nblocks, s);
  const double b = s[1] > 0.0 ? -s[0] / s[1] : 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kBlock)
    if (!act || act[k % N]) d[k] = (T)((double)d[k] + b * (double)v[k]);
}

// d += h delta on the points of the optimised set M only.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_delta_in(T* d, const float* __restrict__ delta,
                                                         T h, int64_t n,
                                                         const unsigned char* __restrict__ act,
                                                         int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && act[i % N]) d[i] += h * (T)delta[i];
}

template <typename T>
hipError_t launch_add_delta_in(T* d, const float* delta, double h, int64_t n,
                               const unsigned char* act, int64_t N, hipStream_t s) {
  if (!act) return launch_add_delta<T>(d, delta, h, n, s);
  if (n == 0) return hipSuccess;
  k_add_delta_in<T><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(d, delta, (T)h, n,
                                                                            act, N);
  return hipGetLastError();
}

// The direction as T (the A p pass reads T) and the step; `part` holds
// 2 * kWarmDotBlocks doubles.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_type(const float* __restrict__ in, T* out,
                                                    int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

template <typename T>
hipError_t launch_to_type(const float* in, T* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_to_type<T><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(in, out, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_warm_step(T* d, const T* g, const float* v, const T* av, int64_t n,
                            double* part, const unsigned char* act, int64_t N, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t want = (n + kBlock - 1) / kBlock;
  const int nb = (int)(want < kWarmDotBlocks ? want : kWarmDotBlocks);
  k_warm_dots<T><<<nb, kBlock, 0, s>>>(g, v, av, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_warm_step<T><<<nb, kBlock, 0, s>>>(d, v, n, part, nb, act, N);
  return hipGetLastError();
}

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
                                               const int*, const int*, int*, T*,             \
                                               hipStream_t);                                    \
  template hipError_t launch_node_flags<T>(const LevelView<T>&, int*, hipStream_t);             \
  template hipError_t launch_dilate<T>(const LevelView<T>&, const int*, unsigned char*,         \
                                       hipStream_t);                                             \
  template hipError_t launch_grow_layer<T>(const LevelView<T>&, const unsigned char*,           \
                                           const unsigned char*, T*, T*, unsigned char*, int*,  \
                                           hipStream_t);                                         \
  template hipError_t launch_grow_commit<T>(const LevelView<T>&, const T*, const T*,            \
                                            unsigned char*, unsigned char*, hipStream_t);       \
  template hipError_t launch_state_io<T>(const LevelView<T>&, const double*, float*, float*,    \
                                         const float*, const float*, int, int*, hipStream_t);   \
  template hipError_t launch_state_out64<T>(const LevelView<T>&, const double*, double*,        \
                                            double*, hipStream_t);                              \
  template hipError_t launch_convert<T>(const float*, T*, int, hipStream_t);                    \
  template hipError_t launch_add_delta<T>(T*, const float*, double, int64_t, hipStream_t);      \
  template hipError_t launch_to_type<T>(const float*, T*, int64_t, hipStream_t);                \
  template hipError_t launch_warm_step<T>(T*, const T*, const float*, const T*, int64_t,        \
                                          double*, const unsigned char*, int64_t, hipStream_t); \
  template hipError_t launch_add_delta_in<T>(T*, const float*, double, int64_t,                 \
                                             const unsigned char*, int64_t, hipStream_t);       \
  template hipError_t launch_convert_back<T>(const T*, float*, int, hipStream_t);               \
  template hipError_t launch_fit_batch<T>(const float*, const float*, float*, int*, int64_t,    \
                                          hipStream_t);

VD_INSTANTIATE(float)
VD_INSTANTIATE(double)

}  // namespace vd
