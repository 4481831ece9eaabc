/*
 * vd.h -- C-ABI of the MI355X (gfx950) lattice deformation solver.
 *
 * The library solves, per frame, the non-rigid tracking problem of
 * VolumeDeform (Innmann et al., "VolumeDeform: Real-time Volumetric Non-rigid
 * Reconstruction", 2016):
 *
 *   Given  a regular deformation lattice with per-node positions t_i and
 *          rotations R_i (Sec. 4), dense point-to-plane correspondences and
 *          sparse point-to-point correspondences (Sec. 6, eqs. (2)-(3)) and
 *          the energy weights (eq. (1)),
 *   find   the t_i, R_i minimising E_total = w_s E_sparse + w_d E_dense +
 *          w_r E_reg (eqs. (1)-(4)), by the flip-flop of Sec. 7.1
 *          (positions by preconditioned CG on the normal equations, rotations
 *          by Procrustes) over the nested coarse-to-fine hierarchy of
 *          Sec. 7.2.
 *
 * Conventions shared by every call:
 *   - Return value: VD_OK (0) or a negative VD_E* code; vd_strerror() names it.
 *     No exception crosses the ABI.  On a validation error the handle is left
 *     unchanged.
 *   - Lengths are world units.  Node (a,b,c) of the finest level rests at
 *     origin + spacing * (a,b,c) and is numbered a + nx*(b + ny*c).
 *   - Point arrays are float32, array-of-structs xyz triples (3*n floats).
 *     Rotations are row-major 3x3 (9 floats per node).
 *   - `mem` says where caller pointers live: VD_MEM_HOST or VD_MEM_DEVICE
 *     (device memory of the handle's GPU, e.g. a torch tensor's data_ptr()).
 *   - The library owns all device memory it allocates; the caller owns every
 *     buffer it passes.  No caller pointer is kept after a call returns.
 *   - Work is issued on the stream given at creation (a hipStream_t passed as
 *     void*; NULL = the null stream).  One handle must not be used by two host
 *     threads at once.
 *   - vd_set_constraints takes targets and normals in the lattice frame,
 *     where the global rigid pose (R, t of Sec. 4) is the identity; the pose
 *     and the projective association that produce such constraints from a
 *     depth map are in vd_track.h.
 */
#ifndef VD_H
#define VD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define VD_OK 0
#define VD_EINVAL (-1)   /* bad argument, non-finite value or negative weight */
#define VD_ERANGE (-2)   /* a canonical sample lies outside the coarsest level */
#define VD_ENOMEM (-3)   /* device allocation failed */
#define VD_EHIP (-4)     /* a HIP runtime call failed */
#define VD_ESTATE (-5)   /* call not valid in the handle's current state */

/* ---- precision modes (arithmetic type of the node vectors) -------------- */
#define VD_FP32_FP64RED 0 /* float32 vectors, stencil and rotations; float64
                             CG reductions and step sizes (applied to the
                             float32 vectors as two float32 parts) and
                             energy sums; float64 rotation refit when the
                             float32 fit is ill-conditioned */
#define VD_FP64 1         /* float64 everywhere */

/* ---- pointer location --------------------------------------------------- */
#define VD_MEM_HOST 0
#define VD_MEM_DEVICE 1

/* ---- creation flags ----------------------------------------------------- */
#define VD_FLAG_GRAPH 1u /* capture each frame's schedule in a hipGraph and
                            replay it (default launch path when set) */
#define VD_FLAG_TRACE 2u /* record E_total after every half-step */
#define VD_FLAG_PROFILE 4u /* time every finest-level launch with HIP events;
                              with VD_FLAG_GRAPH, device clock stamps captured
                              in the frame time the finest level's CG
                              iterations (class VD_PROF_CG_A) of every
                              replay, unless that level runs its CG solves
                              as persistent launches (then nothing is
                              stamped) */
#define VD_FLAG_PERSIST 8u /* on levels of at most 128 tiles, run each CG
                              solve as one persistent launch with a grid
                              barrier between iterations (default: on levels
                              of at most 16 tiles; one launch per CG
                              iteration on larger ones) */
#define VD_FLAG_ACTIVE_SET 16u /* optimise only the set M of Sec. 6-7: on each
                                  level the corners of the cells holding
                                  samples (the isosurface's points) plus their
                                  6-neighbours.  E_reg then sums the edges
                                  inside M (points outside M are not used);
                                  points outside M keep their state
                                  through the frame; tiles without points of M
                                  are skipped.  Each constraint build grows M
                                  from the previous build's: points that join
                                  it are initialised by extrapolating the
                                  field (Sec. 8; see vd_get_active) */
#define VD_FLAG_ITERATIVE 32u /* one launch per CG iteration on every level
                                 (overrides VD_FLAG_PERSIST and the default
                                 persistent launch of levels of at most 16
                                 tiles; the iterates are the same).  A
                                 persistent launch needs all its workgroups
                                 resident at once; if concurrent work on the
                                 GPU prevents that, its barrier's bounded
                                 wait gives up and the report carries
                                 VD_REPORT_BARRIER_TIMEOUT: use this flag
                                 there */

/* ---- kernel classes timed under VD_FLAG_PROFILE ------------------------ */
#define VD_PROF_GRADIENT 0  /* gradient / CG initialisation pass */
#define VD_PROF_CG_A 1      /* one CG iteration: step, direction, A p stencil */
#define VD_PROF_CG_B 2      /* the last CG step (d += alpha p) */
#define VD_PROF_ROTATION 3  /* rotation fits */
#define VD_PROF_ENERGY 4    /* energy evaluation */
#define VD_PROF_TRANSFER 5  /* injection / prolongation */
#define VD_PROF_CG_LOOP 6   /* a whole CG solve in one persistent launch */
#define VD_PROF_KINDS 8

/* ---- report bits -------------------------------------------------------- */
#define VD_REPORT_PCG_GUARD 1u    /* a CG step size hit its zero guard */
#define VD_REPORT_POLAR_FP64 2u   /* some rotation fits were redone in float64 */
#define VD_REPORT_POLAR_KEEP 4u   /* some rotation fits were degenerate and kept
                                     the previous rotation */
#define VD_REPORT_WARM_REJECTED 8u /* the predicted initialisation had the
                                      higher energy and was dropped */
#define VD_REPORT_BARRIER_TIMEOUT 16u /* a persistent CG loop's grid barrier
                                         gave up waiting: the frame's result
                                         is unreliable (rerun it without
                                         VD_FLAG_PERSIST) */

#define VD_MAX_LEVELS 4
#define VD_TILE_KINDS 8
#define VD_MAX_TRACE 512

typedef struct vd_lattice vd_lattice;
typedef struct vd_batch vd_batch;

/* Lattice description.  dims[] are the finest level's node counts (>= 2);
 * level l-1 has ceil(n_l / 2) nodes per axis and twice the spacing, all levels
 * sharing `origin` (vertex-nested: coarse node j sits on fine node 2j).
 * gn_iters[] and pcg_iters[] list the schedule coarse -> fine (entries beyond
 * num_levels are ignored; zero is allowed).  Weights are >= 0. */
typedef struct {
  int32_t dims[3];
  double spacing;
  double origin[3];
  int32_t num_levels;               /* 1 .. VD_MAX_LEVELS */
  int32_t gn_iters[VD_MAX_LEVELS];  /* flip-flop iterations per level */
  int32_t pcg_iters[VD_MAX_LEVELS]; /* CG iterations per position step */
  double w_dense;                   /* w_d of eq. (1) */
  double w_sparse;                  /* w_s */
  double w_arap;                    /* w_r */
  int32_t precision;                /* VD_FP32_FP64RED or VD_FP64 */
  uint32_t flags;                   /* VD_FLAG_* */
  int32_t tile[VD_MAX_LEVELS];      /* stencil tile per level: 0 = library
                                       default, 1 = 8x8x4, 2 = 8x8x8,
                                       3 = 32x8x4 (256 threads), 4 = 32x8x4
                                       (1024 threads), 5 = 8x8x16 (1024
                                       threads), 6 = 16x4x16 (1024 threads),
                                       7 = 16x4x8 (512 threads), 8 = 8x8x4
                                       (512 threads, two per node) (see
                                       vd_tune) */
} vd_lattice_desc;

/* Correspondences of one frame (Sec. 5, used by eqs. (2)-(3)).
 *   canon[3n]   canonical sample positions p_hat_c (must lie inside the
 *               coarsest level's node box)
 *   target[3n]  observed points p_c^a
 *   normal[3n]  observed normals n_c^a (renormalised; a zero normal gives the
 *               row weight 0)
 *   weight[n]   confidences w_c >= 0 (NULL: all 1)
 *   sparse_canon[3m], sparse_target[3m]  feature pairs (f_hat_s, f_s)
 * n or m may be 0 (the matching pointers may then be NULL). */
typedef struct {
  int64_t n_dense;
  const float* canon;
  const float* target;
  const float* normal;
  const float* weight;
  int64_t n_sparse;
  const float* sparse_canon;
  const float* sparse_target;
  int32_t mem; /* VD_MEM_HOST or VD_MEM_DEVICE for all pointers above */
} vd_constraints;

/* Per-frame options; a NULL opts means all zero.
 *
 * Warm start (not in the paper; see vd_net.h for the network that produces
 * init_delta).  When init_delta is given the call first evaluates eq. (1) at
 * the plain initialisation (the previous frame's state) and at the predicted
 * one (finest displacement + spacing * init_delta, or with warm_mode 1 the
 * minimum along init_delta, followed by one rotation fit; with
 * VD_FLAG_ACTIVE_SET only the points of the optimised set move), and keeps
 * the lower of the two.  The solve then runs from the kept
 * state.  When energy_target > 0 the call runs finest-level flip-flop
 * iterations only, and stops after the first one whose energy is <=
 * energy_target, or after max_gn of them; with energy_target == 0 the full
 * schedule runs.  Target mode decides on the device: every launch of an
 * iteration returns at entry once an earlier iteration has reached the
 * target.  The call queues as many iterations as its previous target-mode
 * call needed, waits for the stream, and then adds one iteration per wait
 * until the target is reached or max_gn iterations are queued. */
typedef struct {
  int32_t reset_to_rest;    /* start from t = t_hat, R = I instead of the
                               previous frame's state */
  int32_t init_mem;         /* VD_MEM_HOST or VD_MEM_DEVICE for init_delta */
  const float* init_delta;  /* NULL or [3][N] (x block, y block, z block)
                               predicted displacement change, in units of the
                               finest spacing */
  double energy_target;     /* > 0: finest-level iterations until E <= it */
  int32_t max_gn;           /* iteration cap in target mode (0: the finest
                               level's gn_iters) */
  int32_t warm_mode;        /* with init_delta: 0 the predicted state is the
                               finest displacement + spacing * init_delta;
                               1 it is the minimum of eq. (1) along
                               init_delta at the current rotations (E is
                               quadratic in the positions: displacement +
                               b * init_delta, b = -g.v / v.Av, g = J^T r,
                               A = J^T J, v = init_delta), which can only
                               lower E.  Other values: VD_EINVAL */
} vd_solve_opts;

/* Filled by vd_solve_frame when a report pointer is given (the call then
 * waits for the frame to finish). */
typedef struct {
  double energy[4];   /* E_total, w_d E_dense, w_s E_sparse, w_r E_reg at the
                         final finest state, eq. (1), no factor 1/2 */
  uint32_t bits;      /* VD_REPORT_* */
  int32_t polar_fp64; /* rotation fits redone in float64 (last frame) */
  int32_t polar_keep; /* degenerate fits that kept the previous rotation */
  int32_t n_trace;    /* entries used in trace[] (VD_FLAG_TRACE) */
  double trace[VD_MAX_TRACE]; /* E_total on the current level after each
                                 position step and each rotation step */
  double prof_us[VD_PROF_KINDS]; /* VD_FLAG_PROFILE: mean duration (us) of
                                    the finest level's launches per class */
  int32_t prof_n[VD_PROF_KINDS];  /* launches timed per class */
  double init_energy[2]; /* init_delta given: E_total at the plain and at the
                            predicted initialisation */
  int32_t warm_used;     /* 1 if the predicted initialisation was kept */
  int32_t gn_done;       /* target mode: finest-level iterations run */
  int32_t target_reached; /* target mode: 1 if E <= energy_target */
  int32_t reserved;
} vd_solve_report;

/* Create a handle: allocates every per-level device array and puts the state
 * at rest (t = t_hat, R = I).  `stream` is a hipStream_t or NULL.  Sec. 4
 * (lattice, regular-grid initialisation), Sec. 7.2 (hierarchy). */
int vd_lattice_create(const vd_lattice_desc* desc, void* stream, vd_lattice** out);

/* Free the handle and all its device memory.  NULL is a no-op. */
int vd_lattice_destroy(vd_lattice* l);

/* Replace the correspondences.  Copies and validates the inputs (VD_EINVAL:
 * non-finite value or negative weight; VD_ERANGE: a canonical sample outside
 * the coarsest level), then rebuilds, for every level, the trilinear rows of
 * eqs. (2)-(3), the per-cell cache of B^T B and B^T b (Sec. 7.1: computed
 * once, before CG starts) and the Jacobi preconditioner.  Waits for the
 * validation result; the rebuild itself is queued on the stream. */
int vd_set_constraints(vd_lattice* l, const vd_constraints* c);

/* Solve one frame (Sec. 7): for each level coarse -> fine, start from the
 * finest state injected to the level plus the prolongated increment of the
 * previous level (then one rotation fit), and run gn_iters flip-flop
 * iterations: a position step (pcg_iters of Jacobi-preconditioned CG on
 * A delta = -J^T r) followed by a rotation step (per-node Procrustes).  The
 * finest result becomes the state.  Asynchronous unless `report` is non-NULL.
 * VD_ESTATE if no constraints were set. */
int vd_solve_frame(vd_lattice* l, const vd_solve_opts* opts, vd_solve_report* report);

/* Batched solve of several independent lattices (same number of levels,
 * schedule, stream and VD_FLAG_GRAPH setting; any sizes and either
 * precision).  Every step of the frame schedule is one launch covering the
 * workgroups of all lattices of one precision, with per-lattice reductions;
 * the float64 lattices, if any, form a second part that runs on a
 * library-owned stream forked from the lattices' stream and joined back into
 * it, so both parts overlap on the GPU.  The batch does not own the handles:
 * they must outlive it.  Creating it sets every handle's stencil tile, per
 * level, to the tile of the largest lattice of its part at that level.
 * VD_EINVAL on mismatched handles. */
int vd_batch_create(vd_lattice* const* lattices, int32_t n, vd_batch** out);

/* Solve one frame of every lattice of the batch (Sec. 7, as vd_solve_frame);
 * VD_ESTATE if a handle has no constraints.  energies (may be NULL) receives
 * n x 4 values, eq. (1) per lattice, after waiting for the stream; without it
 * the call is asynchronous.  The schedule is replayed from a hipGraph when
 * the first handle was created with VD_FLAG_GRAPH.  Only reset_to_rest of
 * opts applies; a warm start or energy target gives VD_EINVAL. */
int vd_batch_solve(vd_batch* b, const vd_solve_opts* opts, double* energies);

/* Tile autotuner of the batch (as vd_tune, over the batched launches): per
 * part (float32 lattices, then float64 ones) and level, times one batched
 * position step (gradient pass and `iters` CG iterations) from the current
 * state with every tile kind, keeps the fastest for every handle of the part
 * and restores the displacements.  tile_out[2 * VD_MAX_LEVELS] (may be NULL)
 * receives the chosen kinds (1-based; 0 for a missing part), us_out[2 *
 * VD_MAX_LEVELS * VD_TILE_KINDS] (may be NULL) the microseconds per CG
 * iteration, gradient pass included, of every (part, level, kind).
 * VD_ESTATE if a handle has no constraints.  Waits for the stream. */
int vd_batch_tune(vd_batch* b, int32_t iters, int32_t* tile_out, double* us_out);

/* Mean duration (us) and count of the finest level's launches per kernel
 * class (VD_PROF_*) of the last batch frame, when the first handle was
 * created with VD_FLAG_PROFILE and without VD_FLAG_GRAPH (zeros otherwise).
 * Call after the frame finished (e.g. after vd_batch_solve with energies). */
int vd_batch_profile(vd_batch* b, double prof_us[VD_PROF_KINDS], int32_t prof_n[VD_PROF_KINDS]);

/* Free the batch (not the handles).  NULL is a no-op. */
int vd_batch_destroy(vd_batch* b);

/* Mean duration (us) and count of the launches per kernel class (VD_PROF_*)
 * timed during the last frame (VD_FLAG_PROFILE; zeros otherwise).  Waits for
 * the stream. */
int vd_get_profile(vd_lattice* l, double prof_us[VD_PROF_KINDS], int32_t prof_n[VD_PROF_KINDS]);

/* Energy terms at the current finest state, eq. (1): out = {E_total,
 * w_d E_dense, w_s E_sparse, w_r E_reg}.  Waits for the stream. */
int vd_get_energy(vd_lattice* l, double out[4]);

/* Copy the finest state out: pos[3N] positions t_i, rot[9N] rotations R_i
 * (either pointer may be NULL).  Waits for the stream. */
int vd_get_state(vd_lattice* l, float* pos, float* rot, int32_t mem);

/* The finest state in float64 (Sec. 4: t_i = t_hat_i + d_i, R_i): the
 * VD_FP64 state without rounding to float32 (a VD_FP32_FP64RED state
 * widened), for checkpoints and comparisons at float64 precision.  pos[3N],
 * rot[9N], either may be NULL.  Waits for the stream. */
int vd_get_state64(vd_lattice* l, double* pos, double* rot, int32_t mem);

/* Overwrite the finest state (checkpoint / resume).  rot may be NULL (then
 * R = I).  VD_EINVAL on non-finite input. */
int vd_set_state(vd_lattice* l, const float* pos, const float* rot, int32_t mem);

/* The optimised set M of a level (VD_FLAG_ACTIVE_SET; without it every
 * point): mask[N] (may be NULL) receives 1 for the points of M, *count (may be
 * NULL) their number, *growth_layers (may be NULL) the number of layers the
 * last constraint build extrapolated on the finest level (a point that joins
 * M takes the mean displacement of its already initialised 6-neighbours and
 * the rotation of the first of them in the order -x, +x, -y, +y, -z, +z).
 * Waits for the stream. */
int vd_get_active(vd_lattice* l, int32_t level, uint8_t* mask, int64_t* count,
                  int32_t* growth_layers);

/* Node count and dims of a level (0 = coarsest). */
int vd_level_info(const vd_lattice* l, int32_t level, int32_t dims[3], double* spacing);

/* Text for a status code. */
const char* vd_strerror(int code);

/* Autotuner of the stencil tile shape (the brick each workgroup stages in
 * LDS).  For every level it times a position step -- the gradient pass and
 * `iters` CG iterations -- with each tile kind on the current constraints
 * (the state is saved and restored; one warm-up pass, then the fastest of
 * three timed passes), keeps the fastest for later frames and reports it in
 * tile_out[level] (1..7, as in vd_lattice_desc.tile) with the step's time
 * divided by `iters` (microseconds per CG iteration, the gradient pass
 * included) of each kind in us_out[VD_TILE_KINDS * level + kind - 1]
 * (either pointer may be NULL).
 * VD_ESTATE if no constraints were set.  Synchronous. */
int vd_tune(vd_lattice* l, int32_t iters, int32_t* tile_out, double* us_out);

/* ---- test entry points (unstable; for parity tests) -------------------- */

/* Ap = A p on `level` for the current constraints, A = J^T J of Sec. 7.1
 * (the paper's L + B^T B with the energy weights): p, Ap are [3N] xyz
 * triples.  Synchronous. */
int vd_debug_apply(vd_lattice* l, int32_t level, const float* p, float* Ap, int32_t mem);

/* g = J^T r at the given level state (pos [3N], rot [9N]) and the current
 * constraints, so that E(t + d) = E + 2 g^T d + d^T A d.  Synchronous. */
int vd_debug_gradient(vd_lattice* l, int32_t level, const float* pos, const float* rot,
                      float* g, int32_t mem);

/* Energy terms (as vd_get_energy) at a given level state.  Synchronous. */
int vd_debug_energy(vd_lattice* l, int32_t level, const float* pos, const float* rot,
                    double out[4], int32_t mem);

/* Jacobi preconditioner diagonal diag(A) of a level, [3N].  Synchronous. */
int vd_debug_diag(vd_lattice* l, int32_t level, float* diag, int32_t mem);

/* Rotation step on a level state: R_out[9N] = Procrustes fit of the
 * cross-covariances of pos [3N] (Sec. 7.1), degenerate fits keeping rot_prev
 * [9N].  Synchronous. */
int vd_debug_rotations(vd_lattice* l, int32_t level, const float* pos, const float* rot_prev,
                       float* rot_out, int32_t mem);

/* Batched rotation fit of n cross-covariances M[9n] (row-major): R[9n] is the
 * rotation maximising trace(R^T M) (Sec. 7.1, Procrustes).  keep[n] (may be
 * NULL) receives 0 for a direct fit, 1 for a fit redone in float64, 2 for a
 * degenerate M (rank <= 1), where R copies R_prev[9n] (or I if R_prev is
 * NULL).  precision: VD_FP32_FP64RED or VD_FP64.  Synchronous, on `stream`. */
int vd_debug_fit_rotations(const float* M, const float* R_prev, float* R, int32_t* keep,
                           int64_t n, int32_t precision, int32_t mem, void* stream);

/* The library's stable radix sort of n (key, value) pairs by the low end_bit
 * bits of the keys (0 <= end_bit <= 32; the higher bits must be zero), equal
 * keys keeping their input order: keys_out, vals_out [n].  The binning of
 * constraint rows by cell (Sec. 7.1).  Synchronous, on `stream`. */
int vd_debug_sort_pairs(const uint32_t* keys, const int32_t* vals, uint32_t* keys_out,
                        int32_t* vals_out, int64_t n, int32_t end_bit, int32_t mem,
                        void* stream);

/* The library's exclusive prefix sum of n int32 values: out[i] = sum of
 * in[0 .. i).  Synchronous, on `stream`. */
int vd_debug_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t mem,
                            void* stream);

/* Prolongation of a coarse per-node field (level-1) to `level`: out[3N_fine]
 * = trilinear evaluation of coarse[3N_coarse] at the fine rest positions.
 * Synchronous. */
int vd_debug_prolong(vd_lattice* l, int32_t level, const float* coarse, float* out, int32_t mem);

#ifdef __cplusplus
}
#endif

#endif /* VD_H */
