// Kernel launchers of the lattice solver.  Everything is templated on the
// node-vector type T (float for VD_FP32_FP64RED, double for VD_FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vd.h"

namespace vd {

// Device-resident scalars of one level.  Written only by the last block of a
// reduction kernel (or by a single thread), read by the next kernel.
// Row of a node's 27 symmetric 3x3 data blocks in LevelView::A27r.  Part
// m = dz + 1 holds the 9 blocks of offset dz in (dx, dy) order, 6 entries each
// (xx, xy, xz, yy, yz, zz), padded with zeros to kA27Part entries: entry q of
// part m is entry k = (dx + 1) + 3 (dy + 1), q = 6k + component.  The three
// parts are interleaved by 16-byte chunks (C = 16 / sizeof(T) entries): entry
// q of part m sits at (3 (q / C) + m) C + q % C, so the three lanes that
// evaluate a node's parts read one contiguous span per chunk.
constexpr int kA27Part = 56;
constexpr int kA27Row = 3 * kA27Part;

struct Scalars {
  double rz;      // r^T D^-1 r of the current CG iterate
  double pap;     // p^T A p
  double alpha;   // CG step size
  double beta;    // CG direction update
  double energy[4];
  int beta_valid;  // 0 right after the gradient pass: p = z on the next phase A
  int guard_hits;  // zero-denominator guards taken
  int polar_fp64;  // rotation fits redone in float64
  int polar_keep;  // degenerate rotation fits (previous R kept)
  int n_active;    // cells holding at least one constraint row
  int n_trace;
  int rows;        // constraint rows of the current frame (dense + 3 sparse)
  int n_dense;     // dense rows among them
  unsigned bar;      // arrivals at the grid barrier of the persistent CG loop
  int bar_timeouts;  // grid barrier waits that gave up (bounded spin)
  // energy-target mode: the target, set once E_total <= target (every
  // guarded launch then returns at entry), and iterations completed
  double target;
  int stop;
  int gn_done;
  double trace[VD_MAX_TRACE];
};

// Per-level view of one lattice, passed to kernels by value (or read from a
// device table when a launch covers several lattices).
template <typename T>
struct LevelView {
  int nx, ny, nz;
  int N;            // nx * ny * nz
  int tile;         // tile kind of the stencil / CG kernels
  int ntiles;       // workgroups of that tile kind (= CG block partials)
  int rblocks;      // energy row workgroups (sized by the row capacity)
  T h;              // node spacing of this level
  T wr;             // w_arap
  // node vectors, SoA [3][N] (rot: [9][N], row-major entries)
  T* d;       // displacement t - t_hat (the unknowns)
  T* r;       // CG residual r_0 (= -gradient) and even iterates
  T* r2;      // odd CG iterates
  T* pa;      // CG directions, even / odd iterates
  T* pb;
  T* ap;      // A p, even / odd iterates
  T* ap2;
  T* dinv;    // Jacobi preconditioner 1 / diag(A)
  T* bnode;   // J^T (weighted targets) of the data rows, per node
  T* base;    // finest state injected to this level (for the increment)
  T* rot;     // rotations
  // optimised set M (isosurface points plus their one-ring): 1 per node of
  // M; null when every node is optimised
  const unsigned char* act;
  double* scg0;  // CG block partials [4][ntiles], even / odd iterates
  double* scg1;
  double* pe;    // energy block partials [3][rblocks + node blocks]
  // constraint cache
  const int* cell_map;  // (nx-1)(ny-1)(nz-1) -> active cell index or -1
  const T* K;           // [active][8 corners a][8 corners b][6] sym 3x3 blocks
  const int* node_slot; // node -> row of A27r, -1 if no data term touches it
  const T* A27r;        // [N][kA27Row] 27-point data blocks of each node's row of A
                        // (three parts by dz)
  // constraint rows of the current frame (SoA with stride sc->rows)
  const int* row_cell;
  const T* row_f;
  const T* row_sn;
  const T* row_rho;
  Scalars* sc;
};

// One launch over one or several lattices (all at the same schedule step).
// Workgroup g belongs to lattice b with starts[b] <= g < starts[b + 1].
template <typename T>
struct Dispatch {
  LevelView<T> one;           // the lattice when n == 1
  const LevelView<T>* views;  // device table of n views when n > 1
  const int* starts;          // device [n + 1] first workgroup of each lattice
  int n;
  int blocks;                 // total workgroups
  int masked;                 // some lattice restricts the solve to its set M
  const int* stop;            // non-null: return at entry while *stop is set
};

// Constraint rows of one level (dense rows then 3 rows per sparse pair).
template <typename T>
struct RowView {
  int rows;        // C + 3 S
  int n_dense;     // C
  int* cell;       // linear cell id per row
  T* f;            // [3][rows] fractional coordinates
  T* sn;           // [3][rows] sqrt(w) * normal
  T* rho;          // [rows]    sqrt(w) * normal . (target - canonical)
  int* sorted;     // rows ordered by cell
  int* seg_start;  // [active + 1] start of each active cell's rows in `sorted`
  T* bcell;        // [active][8][3] per-cell right-hand side blocks
  int* active_cell;  // [active] linear cell id
};

struct RawConstraints {
  const float* canon;
  const float* target;
  const float* normal;
  const float* weight;  // may be null (all 1)
  const float* sparse_canon;
  const float* sparse_target;
  int n_dense, n_sparse;
};

// ---- constraint build ----------------------------------------------------
hipError_t launch_validate(const RawConstraints& c, int nx0, int ny0, int nz0, double h0,
                           const double* origin, int* flags, hipStream_t s);

template <typename T>
hipError_t launch_rows(const RawConstraints& c, const LevelView<T>& L, const RowView<T>& R,
                       const double* origin, double w_dense, double w_sparse,
                       unsigned* keys, int* vals, hipStream_t s);

template <typename T>
hipError_t launch_segments(const LevelView<T>& L, const RowView<T>& R, const unsigned* skeys,
                           const int* scan, int* cell_map_w, int ncell, hipStream_t s);

hipError_t launch_heads(const unsigned* skeys, int n, int* heads, hipStream_t s);

template <typename T>
hipError_t launch_build_cells(const LevelView<T>& L, const RowView<T>& R, T* K, int grid,
                              hipStream_t s);

template <typename T>
hipError_t launch_node_flags(const LevelView<T>& L, int* flags, hipStream_t s);

// act[i] = flags[i] or a 6-neighbour's flag (the one-ring of the flagged
// isosurface points).
template <typename T>
hipError_t launch_dilate(const LevelView<T>& L, const int* flags, unsigned char* act,
                         hipStream_t s);

// One layer of grid growth on a level: every node of act that is not
// `known` and has a known 6-neighbour takes the mean of their displacements
// and the rotation of the first of them in the order -x, +x, -y, +y, -z, +z
// (written to tmp_d [3][N], tmp_r [9][N], marked in `fresh`); *count gets
// the number of such nodes.  launch_grow_commit copies them into d / rot
// and marks them known.
template <typename T>
hipError_t launch_grow_layer(const LevelView<T>& L, const unsigned char* act,
                             const unsigned char* known, T* tmp_d, T* tmp_r,
                             unsigned char* fresh, int* count, hipStream_t s);
template <typename T>
hipError_t launch_grow_commit(const LevelView<T>& L, const T* tmp_d, const T* tmp_r,
                              unsigned char* fresh, unsigned char* known, hipStream_t s);

template <typename T>
hipError_t launch_assemble_nodes(const LevelView<T>& L, const RowView<T>& R, const int* flags,
                                 const int* scan, int* node_slot, T* A27r,
                                 hipStream_t s);

// ---- solve (solve.hip) ------------------------------------------------------
enum StencilMode { kModeRhs = 1, kModeApply = 2, kModeGrad = 3 };

// Workgroups of the stencil and CG kernels for a tile kind (0: 8x8x4,
// 1: 8x8x8, 2: 32x8x4), the kind used when none is chosen, and the
// workgroups of the node-parallel and energy kernels.
int tile_blocks(int kind, int nx, int ny, int nz);
int default_tile(int nx, int ny, int nz);
int node_blocks(int N);
int energy_blocks(int rblocks, int N);

// All launchers take a Dispatch whose `blocks`/`starts` were built for the
// kernel's kind of workgroup: tiles (stencil, CG), nodes (CG final step,
// rotations, transfers, rest state), rows+nodes (energy) or one per lattice
// (energy finalize, counters).

// Gradient pass (r = -J^T r into L.r) or the test entry points A p / J^T r
// (n == 1 only; pin / out are SoA [3][N]).
template <typename T>
hipError_t launch_stencil(int mode, const Dispatch<T>& D, const T* pin, T* out, hipStream_t s);

// CG iteration m (first: m == 0) on every lattice of D (tile workgroups).
// stamp (may be NULL): the first workgroup writes the device's constant-rate
// wall clock there when it starts (timing inside a captured graph).
template <typename T>
hipError_t launch_cg(int m, const Dispatch<T>& D, hipStream_t s,
                     unsigned long long* stamp = nullptr);

// d += alpha p of CG iterate `last` (node workgroups); stamp as launch_cg.
template <typename T>
hipError_t launch_cg_final(int last, const Dispatch<T>& D, hipStream_t s,
                           unsigned long long* stamp = nullptr);

// All `iters` CG iterations and the last step of one position solve in one
// launch (one lattice; all its tiles resident at once, with a grid barrier
// between iterations).  Same arithmetic as launch_cg + launch_cg_final.
constexpr int kPersistMaxTiles = 128;
template <typename T>
hipError_t launch_cg_loop(int iters, const Dispatch<T>& D, hipStream_t s);

// Energy of eq. (1) into each lattice's sc->energy (rows+nodes workgroups for
// De, one workgroup per lattice for D1).
template <typename T>
hipError_t launch_energy(const Dispatch<T>& De, const Dispatch<T>& D1, int record_trace,
                         hipStream_t s);

// Per-frame counters back to zero (one workgroup per lattice).
template <typename T>
hipError_t launch_reset_counters(const Dispatch<T>& D1, hipStream_t s);

// Rotation step on every lattice of D (node workgroups), in place.
template <typename T>
hipError_t launch_polar(const Dispatch<T>& D, hipStream_t s);

// Level <- finest injection (node workgroups of the level; F: finest views).
template <typename T>
hipError_t launch_inject(const Dispatch<T>& D, const Dispatch<T>& F, int stride, hipStream_t s);

// fine.d (+)= prolongation of (coarse.d - coarse.base) (node workgroups of the
// fine level; C: coarse views, base may be null).
template <typename T>
hipError_t launch_prolong(const Dispatch<T>& Dfine, const Dispatch<T>& C, int add, hipStream_t s);

// d = 0, R = I (node workgroups).
template <typename T>
hipError_t launch_set_rest(const Dispatch<T>& D, hipStream_t s);

// Single-lattice Dispatch of a view for a given workgroup count.
template <typename T>
inline Dispatch<T> single(const LevelView<T>& L, int blocks) {
  Dispatch<T> D{};
  D.one = L;
  D.views = nullptr;
  D.starts = nullptr;
  D.n = 1;
  D.blocks = blocks;
  D.masked = L.act != nullptr;
  return D;
}

// The same launch, skipped on the device while *stop is set (the launches
// of an energy-target iteration).
template <typename T>
inline Dispatch<T> guarded(Dispatch<T> D, const int* stop) {
  D.stop = stop;
  return D;
}

// Energy-target mode on the device: begin sets sc->target, clears the
// iteration count and sets sc->stop if E_total (sc->energy[0], just
// evaluated) is already <= target; step, after each guarded iteration that
// ran, counts it and sets sc->stop once E_total <= target.
hipError_t launch_target_begin(Scalars* sc, double target, hipStream_t s);
hipError_t launch_target_step(Scalars* sc, hipStream_t s);

// flags |= 1 where any of the n floats is not finite.
hipError_t launch_check_finite(const float* v, int64_t n, int* flags, hipStream_t s);

// sc->rows, sc->n_dense of the current frame.
hipError_t launch_set_counts(Scalars* sc, int rows, int n_dense, hipStream_t s);

template <typename T>
hipError_t launch_state_io(const LevelView<T>& L, const double* origin, float* pos, float* rot,
                           const float* pos_in, const float* rot_in, int dir, int* flags,
                           hipStream_t s);

// d[i] += h * delta[i] for the 3N displacement entries (warm start).
template <typename T>
hipError_t launch_add_delta(T* d, const float* delta, double h, int64_t n, hipStream_t s);

template <typename T>
hipError_t launch_convert(const float* in, T* out, int n, hipStream_t s);
template <typename T>
hipError_t launch_convert_back(const T* in, float* out, int n, hipStream_t s);

// Batched rotation fit of raw matrices (test entry point).
template <typename T>
hipError_t launch_fit_batch(const float* M, const float* R_prev, float* R, int* keep, int64_t n,
                            hipStream_t s);

// Stable radix sort of (key, value) pairs by the low end_bit bits of the
// keys and exclusive integer prefix sums (sort.hip); temp holds at least
// sort_temp_bytes / scan_temp_bytes bytes.
size_t sort_temp_bytes(int n);
hipError_t sort_pairs(void* temp, size_t bytes, const unsigned* kin, unsigned* kout,
                      const int* vin, int* vout, int n, int end_bit, hipStream_t s);
size_t scan_temp_bytes(int n);
hipError_t exclusive_scan(void* temp, size_t bytes, const int* in, int* out, int n,
                          hipStream_t s);

}  // namespace vd
