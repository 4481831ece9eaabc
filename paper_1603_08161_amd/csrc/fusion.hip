// Non-rigid TSDF fusion (Sec. 8) and data-parallel marching cubes (Sec. 4)
// on the finest lattice's grid (gfx950).
//
// As in the association, every decision and every stored value is computed
// in float64 from the float32 inputs in the operation order written here;
// this file is compiled without floating-point contraction.

#include <hip/hip_runtime.h>

#include <mutex>

#include "fusion_kernels.h"
#include "vd_device.h"

namespace vd {

namespace {

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// ---- the marching-cubes case table (built on the host, see build_table) ----
// Corners k = dx + 2 dy + 4 dz; edge 4 q + j joins the two corners that differ
// in bit q, j = b1 + 2 b2 from the bits of the other two axes (ascending).
struct McTable {
  unsigned char count[256];      // triangles of the case
  unsigned char edge[256][15];   // their edges, three per triangle
};
__constant__ McTable c_mc;

int edge_of(int a, int b) {
  const int x = a ^ b;
  const int q = x == 1 ? 0 : (x == 2 ? 1 : 2);
  const int o1 = q == 0 ? 1 : 0, o2 = q == 2 ? 1 : 2;
  return 4 * q + ((a >> o1) & 1) + 2 * ((a >> o2) & 1);
}

// For every case: walk each face's corners counter-clockwise as seen from
// outside; each maximal run of inside corners yields a segment from the edge
// entering the run to the edge leaving it.  Every sign-change edge starts
// one segment and ends another, so following the segments from the lowest
// unvisited edge closes loops; each loop is split into a fan of triangles
// from its first edge.
void build_table(McTable* t) {
  int faces[6][4];
  int f = 0;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const int ring[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int s = 0; s < 2; ++s) {
      for (int m = 0; m < 4; ++m) {
        const int k = s == 0 ? 3 - m : m;  // the outward normal -e_a reverses the turn
        faces[f][m] = (s << a) | (ring[k][0] << b) | (ring[k][1] << c);
      }
      ++f;
    }
  }
  for (int inside = 0; inside < 256; ++inside) {
    int next[12];
    for (int e = 0; e < 12; ++e) next[e] = -1;
    for (int fi = 0; fi < 6; ++fi) {
      int neg[4], n = 0;
      for (int m = 0; m < 4; ++m) {
        neg[m] = (inside >> faces[fi][m]) & 1;
        n += neg[m];
      }
      if (n == 0 || n == 4) continue;
      for (int m = 0; m < 4; ++m) {
        if (!neg[m] || neg[(m + 3) % 4]) continue;
        const int enter = edge_of(faces[fi][(m + 3) % 4], faces[fi][m]);
        int e = m;
        while (neg[(e + 1) % 4]) e = (e + 1) % 4;
        next[enter] = edge_of(faces[fi][e], faces[fi][(e + 1) % 4]);
      }
    }
    bool seen[12] = {false};
    int cnt = 0;
    for (int start = 0; start < 12; ++start) {
      if (next[start] < 0 || seen[start]) continue;
      int loop[12], len = 0;
      int e = start;
      do {
        loop[len++] = e;
        seen[e] = true;
        e = next[e];
      } while (e != start);
      for (int k = 1; k + 1 < len; ++k) {
        t->edge[inside][3 * cnt + 0] = (unsigned char)loop[0];
        t->edge[inside][3 * cnt + 1] = (unsigned char)loop[k];
        t->edge[inside][3 * cnt + 2] = (unsigned char)loop[k + 1];
        ++cnt;
      }
    }
    t->count[inside] = (unsigned char)cnt;
  }
}

std::mutex g_table_mutex;
bool g_table_ready[64] = {false};

__device__ __forceinline__ void apply_pose(const double* P, const double p[3], double q[3]) {
  for (int r = 0; r < 3; ++r)
    q[r] = P[3 * r] * p[0] + P[3 * r + 1] * p[1] + P[3 * r + 2] * p[2] + P[9 + r];
}

}  // namespace

int mc_table_ready() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  std::lock_guard<std::mutex> lock(g_table_mutex);
  if (!g_table_ready[dev]) {
    static McTable host;
    static bool built = false;
    if (!built) {
      build_table(&host);
      built = true;
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_mc), &host, sizeof(McTable)) != hipSuccess) return -1;
    g_table_ready[dev] = true;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// fusion
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fuse(FuseParams p, LevelView<T> L,
                                                 const float* __restrict__ depth,
                                                 const double* __restrict__ pose,
                                                 const int* __restrict__ frames, float* D,
                                                 float* W, int* n_updated) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  bool upd = false;
  if (i < L.N) {
    const bool allowed =
        p.all_points || ((!L.act || L.act[i]) && frames[i] >= p.k_min);
    if (allowed) {
      const int idx[3] = {i % L.nx, (i / L.nx) % L.ny, i / (L.nx * L.ny)};
      const double o[3] = {p.ox, p.oy, p.oz};
      const size_t N = L.N;
      double q[3], x[3];
      for (int k = 0; k < 3; ++k) q[k] = (o[k] + p.h * (double)idx[k]) + (double)L.d[k * N + i];
      double P[12];
      for (int k = 0; k < 12; ++k) P[k] = pose[k];
      apply_pose(P, q, x);
      if (x[2] > 0.0) {
        const double uf = floor(p.fx * x[0] / x[2] + p.cx);
        const double vf = floor(p.fy * x[1] / x[2] + p.cy);
        if (uf >= 0.0 && uf < (double)p.W && vf >= 0.0 && vf < (double)p.H) {
          const double z = (double)depth[(size_t)vf * p.W + (size_t)uf];
          if (z > 0.0) {
            const double eta = z - x[2];
            if (!(eta < -p.tau)) {
              const double s = fmin(1.0, eta / p.tau);
              const double w = (double)W[i];
              D[i] = (float)((w * (double)D[i] + s) / (w + 1.0));
              W[i] = (float)fmin(w + 1.0, p.w_max);
              upd = true;
            }
          }
        }
      }
    }
  }
  if (upd) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0 && cnt) atomicAdd(n_updated, cnt);
}

template <typename T>
hipError_t launch_fuse(const FuseParams& p, const LevelView<T>& L, const float* depth,
                       const double* pose, const int* frames, float* D, float* W, int* n_updated,
                       hipStream_t s) {
  k_fuse<T><<<blocks_for(L.N), kBlock, 0, s>>>(p, L, depth, pose, frames, D, W, n_updated);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_count_frames(LevelView<T> L, int* frames) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.N) return;
  frames[i] = (!L.act || L.act[i]) ? frames[i] + 1 : 0;
}

template <typename T>
hipError_t launch_count_frames(const LevelView<T>& L, int* frames, hipStream_t s) {
  k_count_frames<T><<<blocks_for(L.N), kBlock, 0, s>>>(L, frames);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// marching cubes: count, (scan), emit
// ---------------------------------------------------------------------------

__device__ __forceinline__ int mc_case(const float* __restrict__ D, const float* __restrict__ W,
                                       int nx, int ny, int cx, int cy, int cz, double v[8]) {
  int inside = 0;
  for (int k = 0; k < 8; ++k) {
    const size_t id = (size_t)(cx + (k & 1)) +
                      (size_t)nx * ((size_t)(cy + ((k >> 1) & 1)) + (size_t)ny * (cz + (k >> 2)));
    if (!(W[id] > 0.0f)) return -1;
    v[k] = (double)D[id];
    if (v[k] < 0.0) inside |= 1 << k;
  }
  return inside;
}

__global__ __launch_bounds__(kBlock) void k_mc_count(const float* __restrict__ D,
                                                     const float* __restrict__ W, int nx, int ny,
                                                     int nz, int* counts) {
  const int cnx = nx - 1, cny = ny - 1;
  const int ncell = cnx * cny * (nz - 1);
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell) return;
  double v[8];
  const int inside = mc_case(D, W, nx, ny, c % cnx, (c / cnx) % cny, c / (cnx * cny), v);
  counts[c] = inside < 0 ? 0 : (int)c_mc.count[inside];
}

hipError_t launch_mc_count(const float* D, const float* W, int nx, int ny, int nz, int* counts,
                           hipStream_t s) {
  const int ncell = (nx - 1) * (ny - 1) * (nz - 1);
  k_mc_count<<<blocks_for(ncell), kBlock, 0, s>>>(D, W, nx, ny, nz, counts);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mc_emit(MeshParams p, LevelView<T> L,
                                                    const float* __restrict__ D,
                                                    const float* __restrict__ W,
                                                    const int* __restrict__ counts,
                                                    const int* __restrict__ offsets,
                                                    const double* __restrict__ pose, float* canon,
                                                    float* deformed, int* cells, int* edges) {
  const int cnx = L.nx - 1, cny = L.ny - 1;
  const int ncell = cnx * cny * (L.nz - 1);
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell || counts[c] == 0) return;
  const int cx = c % cnx, cy = (c / cnx) % cny, cz = c / (cnx * cny);
  double v[8];
  const int inside = mc_case(D, W, L.nx, L.ny, cx, cy, cz, v);
  if (inside < 0) return;
  double P[12];
  for (int k = 0; k < 12; ++k) P[k] = pose[k];
  const double o[3] = {p.ox, p.oy, p.oz};
  const int n = c_mc.count[inside];
  const size_t base = (size_t)offsets[c];
  const size_t N = L.N;
  for (int t = 0; t < n; ++t) {
    const size_t tri = base + t;
    if (cells) cells[tri] = c;
    for (int m = 0; m < 3; ++m) {
      const int e = c_mc.edge[inside][3 * t + m];
      if (edges) edges[3 * tri + m] = e;
      const int q = e >> 2, j = e & 3;
      const int o1 = q == 0 ? 1 : 0, o2 = q == 2 ? 1 : 2;
      const int a = ((j & 1) << o1) | ((j >> 1) << o2), b = a | (1 << q);
      const int ca[3] = {cx + (a & 1), cy + ((a >> 1) & 1), cz + (a >> 2)};
      const int cb[3] = {cx + (b & 1), cy + ((b >> 1) & 1), cz + (b >> 2)};
      const double s = v[a] / (v[a] - v[b]);
      float xf[3];
      for (int k = 0; k < 3; ++k) {
        const double xa = o[k] + p.h * (double)ca[k];
        const double xb = o[k] + p.h * (double)cb[k];
        xf[k] = (float)(xa + s * (xb - xa));
        canon[9 * tri + 3 * m + k] = xf[k];
      }
      if (!deformed) continue;
      // S(x) = R (x + sum_k alpha_k d_k) + t over the finest cell holding x
      double x[3], f[3], sum[3] = {0.0, 0.0, 0.0}, y[3];
      int cc[3];
      const int nn[3] = {L.nx, L.ny, L.nz};
      for (int k = 0; k < 3; ++k) {
        x[k] = (double)xf[k];
        const double u = (x[k] - o[k]) / p.h;
        double fl = floor(u);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(nn[k] - 2)) fl = (double)(nn[k] - 2);
        cc[k] = (int)fl;
        f[k] = u - fl;
      }
      for (int k = 0; k < 8; ++k) {
        const int ex = k & 1, ey = (k >> 1) & 1, ez = (k >> 2) & 1;
        const double wx = ex ? f[0] : 1.0 - f[0];
        const double wy = ey ? f[1] : 1.0 - f[1];
        const double wz = ez ? f[2] : 1.0 - f[2];
        const double wk = wx * wy * wz;
        const size_t id = (size_t)(cc[0] + ex) +
                          (size_t)L.nx * ((size_t)(cc[1] + ey) + (size_t)L.ny * (cc[2] + ez));
        for (int r = 0; r < 3; ++r) sum[r] += wk * (double)L.d[r * N + id];
      }
      for (int r = 0; r < 3; ++r) x[r] = x[r] + sum[r];
      apply_pose(P, x, y);
      for (int k = 0; k < 3; ++k) deformed[9 * tri + 3 * m + k] = (float)y[k];
    }
  }
}

template <typename T>
hipError_t launch_mc_emit(const MeshParams& p, const LevelView<T>& L, const float* D,
                          const float* W, const int* counts, const int* offsets,
                          const double* pose, float* canon, float* deformed, int* cells,
                          int* edges, hipStream_t s) {
  const int ncell = (L.nx - 1) * (L.ny - 1) * (L.nz - 1);
  k_mc_emit<T><<<blocks_for(ncell), kBlock, 0, s>>>(p, L, D, W, counts, offsets, pose, canon,
                                                    deformed, cells, edges);
  return hipGetLastError();
}

#define VD_FUSION_INSTANTIATE(T)                                                               \
  template hipError_t launch_fuse<T>(const FuseParams&, const LevelView<T>&, const float*,    \
                                     const double*, const int*, float*, float*, int*,         \
                                     hipStream_t);                                            \
  template hipError_t launch_count_frames<T>(const LevelView<T>&, int*, hipStream_t);         \
  template hipError_t launch_mc_emit<T>(const MeshParams&, const LevelView<T>&, const float*, \
                                        const float*, const int*, const int*, const double*,  \
                                        float*, float*, int*, int*, hipStream_t);
VD_FUSION_INSTANTIATE(float)
VD_FUSION_INSTANTIATE(double)

}  // namespace vd
