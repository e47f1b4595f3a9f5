/*
 * homelbm.h -- C ABI of the MI355X HOME-LBM library (libhomelbm.so).
 *
 * One D3Q27 HOME-LBM time step per lbm_step iteration, after "High-Performance
 * Moment-Encoded Lattice Boltzmann Method with Stability-Guided Quantization"
 * (arXiv 2602.05295):
 *   - state: per cell the ten moments of Eq. (rho_u_stress), Sec. 3.1:
 *     rho, j = rho u (3) and P = rho S (6, S the Hermite second moment
 *     sum (c c - cs^2 delta) f / rho), stored after streaming (Alg. 2);
 *   - step: moment-space collision (App. A, with an optional uniform body
 *     force) -> third-order Hermite
 *     reconstruction of f+ (Eq. three_order_f, Sec. 3.2) -> pull streaming
 *     f_i(x) = f+_i(x - c_i) -> projection back to moments (Sec. 4.2, Alg. 2);
 *   - boundaries in a separate pass over a compacted list of boundary cells
 *     (the split of Sec. 4.2): halfway bounce-back against a voxel solid mask,
 *     an inflow face at x = 0 using the moment boundary of Sec. 3.2
 *     (rho^p = rho^x, S^p = u^p u^p + (S^x - u^x u^x)) with u^p = u_in, and a
 *     zero-gradient outflow face at x = nx-1;
 *   - storage either FP32 (ten float planes, 40 B/cell) or the 16-bit form of
 *     Sec. 5.3 (rho in [0.8, 1.5], u in [-0.4, 0.4] and the non-equilibrium
 *     stress rho S - rho u u in [-0.1, 0.1], b = 16 with dithering, two codes
 *     per 32-bit word, five word planes, 20 B/cell).
 *
 * Conventions shared by every call
 *   - Cell (x, y, z) has linear index x + nx * (y + ny * z) (x fastest).
 *   - A moment field is ten planes of nx*ny*nz floats, plane order
 *     rho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz.
 *   - Pointers passed with on_device = 1 are HIP device pointers (e.g. a torch
 *     tensor's data_ptr); with on_device = 0 they are host pointers.  The
 *     caller owns every pointer it passes; the library keeps none of them after
 *     the call returns.  The context owns all device memory it allocates.
 *   - Work is enqueued on the context's stream (lbm_set_stream, default the
 *     null stream).  Calls that read into or write from host memory
 *     synchronise that stream before returning.
 *   - Every call returns an lbm_status.  No call aborts or throws across the
 *     ABI; lbm_last_error(ctx) (or lbm_last_error(NULL) for a failed
 *     lbm_create) gives a message for the last failure.
 *   - Calls on one context are not thread-safe; distinct contexts are
 *     independent.
 */
#ifndef HOMELBM_H
#define HOMELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

/* Moment storage formats. */
enum lbm_moment_format {
  LBM_MOMENTS_FP32 = 0,   /* ten float planes */
  LBM_MOMENTS_Q16 = 1,    /* five uint32 planes of paired 16-bit codes (Sec. 5.3) */
  /* The b_rho_u / b_S bit allocations of the double-layer vortex study:
   * the codes of rho and u take b_rho_u bits, those of the non-equilibrium
   * stress b_S bits (Sec. 5.3's ranges, rounding and dither with b bits),
   * concatenated low bit first in the order rho, ux, uy, uz, Nxx, Nyy, Nzz,
   * Nxy, Nxz, Nyz into ceil((4 b_rho_u + 6 b_S)/32) uint32 planes (16/16 is
   * the layout of LBM_MOMENTS_Q16).  Single-domain contexts only. */
  LBM_MOMENTS_P16_15 = 2, /* 5 planes */
  LBM_MOMENTS_P15_14 = 3, /* 5 planes */
  LBM_MOMENTS_P14_13 = 4, /* 5 planes */
  LBM_MOMENTS_P13_12 = 5, /* 4 planes, 16 B/cell */
  LBM_MOMENTS_P12_11 = 6  /* 4 planes, 16 B/cell */
};

enum lbm_status {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = 1,   /* bad dimensions, tau, mask, pointer or size */
  LBM_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed */
  LBM_ERR_DEVICE = 3,        /* a HIP call failed (message names it) */
  LBM_ERR_UNSUPPORTED = 4,   /* valid request the library does not implement */
  LBM_ERR_UNSTABLE = 5       /* the state holds non-finite values or saturated codes */
};

/* Dither modes for the 16-bit encode (Sec. 5.3, "Dithering"). */
enum lbm_dither_mode {
  LBM_DITHER_OFF = 0,      /* round to nearest, half up */
  LBM_DITHER_PER_STEP = 1, /* zero-mean uniform noise per (cell, step, component) */
  LBM_DITHER_STATIC = 2    /* one spatial noise pattern reused every step */
};

typedef struct lbm_options {
  int dither_mode;    /* lbm_dither_mode; default LBM_DITHER_PER_STEP */
  uint32_t seed;      /* dither seed; default 0 */
  int inflow;         /* 1: x = 0 is an inflow face and x = nx-1 an outflow face;
                         0 (default): x is periodic.  y and z are always periodic. */
  float u_in[3];      /* inflow velocity (used when inflow = 1) */
  int check_health;   /* 1 (default): lbm_step scans the state once at its end and
                         returns LBM_ERR_UNSTABLE if any stored value is non-finite
                         (FP32) or any code sits at 0 or its maximum (integer formats) */
  int tile_rows;      /* fluid-pass tile height: 8, 10, 12 or 13 force it.  0 (default):
                         the first lbm_step, lbm_step_into, lbm_prepare or lbm_profile_*
                         call (after the boundary list is built) times the fluid pass
                         once per height, three rounds, from the current state into the
                         other buffer (the state is unchanged; synchronous), and keeps
                         the fastest; changing inflow, force or tile_rows times again.
                         Results do not depend on the height. */
  float force[3];     /* uniform body force F per cell and step, lattice units (App. A
                         with its force terms; the stored momentum holds F/2 as in
                         Eq. rho_u_stress).  Default 0; each |F_a| <= 0.01.  Not
                         supported by lbm_adjoint_step (LBM_ERR_UNSUPPORTED) nor by
                         batches (force must be 0 there). */
  int wall_rule;      /* solid links: 0 (default) halfway bounce-back, f_i(x) = f+_opp(i)(x);
                         1 the solid coupling of Sec. 3.2: f_i(x) reconstructed from
                         rho^p = rho^x, u^p = V + W x (p - C) of the link's object (see
                         lbm_set_object) at the link midpoint p = x - c_i/2, and
                         S^p = u^p u^p + (S^x - u^x u^x) of x's post-collision moments.
                         The reconstruction does not depend on where p lies on the link,
                         so the no-slip point of a voxel wall is the solid node.  Not
                         supported by lbm_adjoint_step nor by batches.
                         2 (mixed pipeline only, else LBM_ERR_UNSUPPORTED): the same
                         coupling with p where the link first meets the obstacle meshes
                         of lbm_set_triangles and u^p from that triangle's object,
                         applied by the per-triangle solid correction of Sec. 4.2
                         (Alg. 3) instead of per-link corrections. */
  int track_forces;   /* 1: every step adds the force and torque the fluid exerts on each
                         object (momentum exchange over its links, -(f_i(x) + f+_opp(i)(x)) c_i
                         per link, torque about the object's center) to sums read by
                         lbm_get_object_forces; 0 (default): not computed.  Not supported
                         by batches. */
  int pipeline;       /* 0 (default): the fluid pass keeps the unrounded moments of the
                         listed cells and the boundary pass overwrites them (40 B of state
                         traffic per cell and step).  1: the paper's mixed-precision pipeline
                         (Sec. 5.3, atomic accumulation), for comparison: the 16-bit buffer
                         holds post-collision moments; a step streams them into an FP32
                         post-stream buffer, adds the changed links' corrections with
                         atomicAdd and re-encodes (120 B per cell and step; 60 B of state
                         per cell).  16-bit contexts without force or force tracking only
                         (LBM_ERR_UNSUPPORTED).  lbm_get_raw returns the codes of the
                         post-collision moments; lbm_set_raw, lbm_step_into and the adjoint
                         are not supported.  lbm_get_moments returns the post-stream
                         moments, as in pipeline 0.  Switching moves the current moments to
                         the other storage. */
  int graph_steps;    /* 256 (default), 1..4096: lbm_step (pipeline 0) replays captured HIP
                         graphs of up to this many steps, each step's dither key read from a
                         device-side step counter set before the replay, so the result is
                         the same as launching every kernel (graphs are captured on first
                         use and dropped when options or the boundary list change); 0:
                         every kernel is launched one by one. */
} lbm_options;

/* Fills *opt with the defaults listed above. */
int lbm_default_options(lbm_options* opt);

/*
 * Creates a context for an nx*ny*nz grid (dims[0..2] = nx, ny, nz, each in
 * 1..65535, nx*ny*nz <= 2^30).  tau > 1/2 is the relaxation time of App. A (kinematic
 * viscosity nu = (tau - 1/2)/3).  solid_mask is a host array of nx*ny*nz bytes,
 * 0 = fluid, 1..255 = solid, the value naming the object the cell belongs to
 * (lbm_set_object), or NULL for no solids; it is copied.  moment_format is
 * an lbm_moment_format.  The state starts at rest (rho = 1, j = 0, P = 0).
 * On success *out receives the context; on failure *out is set to NULL.
 * Errors: LBM_ERR_INVALID_ARG (dims, tau, format),
 * LBM_ERR_OUT_OF_MEMORY, LBM_ERR_DEVICE.
 */
int lbm_create(const int dims[3], double tau, const uint8_t* solid_mask, int moment_format, lbm_ctx** out);

/* Releases the context and its device memory (after synchronising its stream). NULL is a no-op. */
int lbm_destroy(lbm_ctx* ctx);

/* Message for the last failed call on ctx, or of the calling thread's last failed lbm_create when ctx is NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Sets the hipStream_t (passed as void*) all later work is enqueued on; NULL selects the null stream. */
int lbm_set_stream(lbm_ctx* ctx, void* hip_stream);

/*
 * Sets options.  Turning inflow on requires nx >= 6 and no solid cell within
 * two cells of the x faces (LBM_ERR_INVALID_ARG otherwise); the boundary-cell
 * list is rebuilt when the face setting changes.
 */
int lbm_set_options(lbm_ctx* ctx, const lbm_options* opt);
int lbm_get_options(const lbm_ctx* ctx, lbm_options* opt);

/*
 * Sets the state from a full moment field (ten planes, see conventions).  Integer
 * contexts encode it without dither.  Solid cells are set to rest whatever m
 * holds there.
 */
int lbm_set_moments(lbm_ctx* ctx, const float* m, int on_device);

/*
 * Sets the equilibrium state of given rho (one plane) and u (three planes
 * ux, uy, uz): j = rho u, P = rho u u.  Solid cells are set to rest.
 */
int lbm_set_equilibrium(lbm_ctx* ctx, const float* rho, const float* u, int on_device);

/*
 * Advances n >= 0 time steps; each is one fluid pass over every cell followed
 * by one boundary pass over the compacted boundary list.  Asynchronous on the
 * context stream unless check_health is set (then it synchronises once at the
 * end).  The dither of step t (t counts all steps since create or the last
 * lbm_set_step_count) is drawn from (cell, t, seed).
 */
int lbm_step(lbm_ctx* ctx, int n);

/*
 * Does ahead of time, without advancing the state, what the first
 * lbm_step(ctx, n) would do before its first kernel: builds the boundary list
 * if needed, times the tile heights (tile_rows = 0), and, with graph_steps > 0
 * and pipeline 0, captures and
 * instantiates the step sequences that lbm_step(ctx, n) replays, from either
 * buffer, so that a later lbm_step(ctx, n) only launches them.  Synchronous;
 * the captures are dropped like any others (options or boundary list
 * changed, or more than eight sequences held).  Errors: LBM_ERR_INVALID_ARG
 * for a NULL ctx or n < 0, LBM_ERR_HIP from the capture.
 */
int lbm_prepare(lbm_ctx* ctx, int n);

/* Writes the current state as a full moment field (ten planes); solid cells read as rest. */
int lbm_get_moments(lbm_ctx* ctx, float* m, int on_device);

/*
 * Raw state copy.  FP32: ten float planes (40 B/cell) in the moment order
 * above except that plane 0 holds rho - 1 (for precision); Q16: five uint32 planes
 * (20 B/cell), word p of a cell packs code 2p in its low and code 2p+1 in its
 * high half, code order rho, ux, uy, uz, Nxx, Nyy, Nzz, Nxy, Nxz, Nyz; the
 * LBM_MOMENTS_P formats: their planes of packed codes (see the enum).
 * bytes must equal lbm_raw_bytes().
 */
size_t lbm_raw_bytes(const lbm_ctx* ctx);
int lbm_get_raw(lbm_ctx* ctx, void* out, size_t bytes, int on_device);
int lbm_set_raw(lbm_ctx* ctx, const void* in, size_t bytes, int on_device);

/*
 * One time step from a caller-owned raw state to another (Alg. 2 followed by
 * the boundary pass, as one lbm_step iteration): in and out are device
 * pointers to lbm_raw_bytes() bytes each in the lbm_get_raw layout, and must
 * not overlap (LBM_ERR_INVALID_ARG otherwise).  in must hold the rest state at
 * the solid cells next to fluid, as every state that lbm_get_raw returns does.
 * Uses the context's geometry, mask, tau and options, draws the dither of the
 * context's step count and advances that count by one.  The context's own
 * state is neither read nor written, and no health scan is made.
 * Asynchronous on the context stream; the caller keeps both buffers alive
 * until the step has run.  Meant for rollouts that keep every state, such as
 * the recomputation of a checkpointed segment before its adjoint steps.
 */
int lbm_step_into(lbm_ctx* ctx, const void* in, void* out);

/*
 * Motion of solid object id (1..255, the mask value of its cells) for wall
 * rule 1, and the point torques are taken about: center C, velocity V and
 * angular velocity W in lattice units (wall velocity V + W x (p - C), with p
 * taken from the fluid cell's coordinates without periodic wrapping).  The
 * cells do not move: this sets the velocity of the wall, as for a rotating
 * cylinder or a sliding lid.  Every object starts at C = V = W = 0.  Ordered
 * after the steps already enqueued; synchronises the context stream.
 */
int lbm_set_object(lbm_ctx* ctx, int id, const float center[3], const float velocity[3], const float omega[3]);

/*
 * Sums of the force and torque on every object over the steps since create
 * or the last reset, computed while track_forces is set: out is a host array
 * of 256 x 6 doubles, row id = (Fx, Fy, Fz, Tx, Ty, Tz), row 0 unused.
 * reset = 1 zeroes the sums after reading them.  Synchronises the stream.
 * The per-workgroup partial sums are added with atomics, so the last bits of
 * the sums may differ from run to run.
 */
int lbm_get_object_forces(lbm_ctx* ctx, double* out, int reset);

/* Step counter used by the dither. */
int lbm_get_step_count(const lbm_ctx* ctx, uint64_t* t);
int lbm_set_step_count(lbm_ctx* ctx, uint64_t t);

/*
 * Bytes of the two ping-pong state buffers (2 x 40 B or 2 x 20 B per cell:
 * the 50% saving of Sec. 6.2.1) and of all device memory the context holds.
 */
int lbm_memory_bytes(const lbm_ctx* ctx, size_t* state_bytes, size_t* total_bytes);

/*
 * Sizes of the boundary list: fluid cells recomputed by the boundary pass, and
 * solid cells next to fluid, which hold the rest state at the start of every
 * step (reset by the boundary pass; with the inflow on, the fluid pass stores
 * every solid cell as the rest state and the boundary pass visits none).
 */
int lbm_boundary_counts(const lbm_ctx* ctx, int64_t* fluid_cells, int64_t* solid_cells);

/*
 * The fluid pass's tile height in use (see tile_rows in lbm_options): the
 * option when set, else the height the context timed as fastest, else 0
 * (not timed yet: the planner chooses).  Errors: LBM_ERR_INVALID_ARG.
 */
int lbm_tile_rows(const lbm_ctx* ctx, int* rows);

/* Scans the state now; *bad receives the number of offending values (see check_health). */
int lbm_check(lbm_ctx* ctx, uint64_t* bad);

/*
 * Adjoint of one step, for gradients through lbm_step (FP32 contexts without
 * a body force only, else LBM_ERR_UNSUPPORTED).  All pointers are device pointers to ten planes
 * of nx*ny*nz floats:
 *   m_t      the raw FP32 state the step was taken from (the lbm_get_raw
 *            layout: plane 0 holds rho - 1);
 *   lam_next the adjoint of the moments after the step (moment order; the
 *            adjoint of rho equals that of rho - 1);
 *   lam_prev receives J(m_t)^T lam_next, the adjoint of the moments before the
 *            step (zero at solid cells).  It must not alias the inputs.
 * It follows the same step as lbm_step: App. A collision, the third-order
 * reconstruction of Eq. (three_order_f), pull streaming, projection, and the
 * boundary rules (bounce-back, inflow, outflow).  Asynchronous on the context
 * stream.  Every output cell is written by one thread (boundary contributions
 * are gathered, not scattered), so the result is the same on every run.
 */
int lbm_adjoint_step(lbm_ctx* ctx, const float* m_t, const float* lam_next, float* lam_prev);

/*
 * lbm_adjoint_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same kernels and result, with the per-cell flags the
 * adjoint passes read kept in a fixed 32 MiB device array of the library
 * (one per GPU, held until the process ends) instead of a buffer the context
 * allocates on first use.  It calls no hipMalloc, hipFree or other
 * allocating routine.  Arguments, layout and errors as lbm_adjoint_step,
 * plus LBM_ERR_INVALID_ARG when nx*ny*nz exceeds 33,554,432 (the array's
 * size) or when the boundary list still has to be rebuilt after an inflow
 * change (any lbm_step, lbm_step_into or lbm_adjoint_step rebuilds it).
 * Every call on a GPU rewrites the whole flag array for its context, so calls
 * on one GPU that overlap in time (on different streams or host threads)
 * race and must be ordered by the caller.
 */
int lbm_adjoint_step_noalloc(lbm_ctx* ctx, const float* m_t, const float* lam_next, float* lam_prev);

/*
 * Vector-Jacobian product of lbm_set_equilibrium's map (rho, u) -> (rho, rho u,
 * rho u u): given lam (ten planes), writes grad_rho (one plane; may be NULL)
 * and grad_u (three planes); zero at solid cells.  Device pointers, async.
 */
int lbm_equilibrium_vjp(lbm_ctx* ctx, const float* rho, const float* u, const float* lam, float* grad_rho,
                        float* grad_u);

/*
 * Obstacle meshes for wall rule 2 (Sec. 4.2, Alg. 3): ntris triangles, tris
 * a host array of 9 floats per triangle (x0 y0 z0 x1 y1 z1 x2 y2 z2, lattice
 * units, cell (x, y, z) at integer coordinates, not wrapped), obj a host
 * array of ntris object ids (1..255, the lbm_set_object ids that give each
 * triangle's wall motion).  Both are copied; ntris = 0 removes the meshes.
 * The solid mask still decides which links are replaced: every link from a
 * fluid cell to a solid one should meet a triangle (the mask should mark the
 * lattice points inside the closed meshes); a link that meets none keeps the
 * distribution the stream pass pulled from the solid cell.  One thread per
 * triangle visits the listed fluid cells of its bounding box (widened by one
 * cell) and tests their links to solid sources; the nearest hit on a link
 * (ties to the lowest triangle index) is found once per mesh and boundary
 * list, and each step the winning triangle adds (f_i(p) - f_i pulled) times
 * the link's moments to the cell's FP32 post-stream moments with atomicAdd.
 * Synchronises.  Errors: LBM_ERR_INVALID_ARG (NULL arrays, non-finite
 * vertices), LBM_ERR_OUT_OF_MEMORY, LBM_ERR_DEVICE.
 */
int lbm_set_triangles(lbm_ctx* ctx, int64_t ntris, const float* tris, const uint8_t* obj);

/* Waits for all work on the context stream. */
int lbm_synchronize(lbm_ctx* ctx);

/*
 * Runs n steps like lbm_step, timing each stage with HIP events on the
 * context stream: ms[0] the fluid (or stream) pass, ms[1] the boundary pass
 * (or the link corrections), ms[2] the requantize pass of pipeline 1 (0
 * otherwise); sums over the n steps.  Synchronises.
 */
int lbm_profile_stages(lbm_ctx* ctx, int n, double ms[3]);

/*
 * Runs n steps like lbm_step while timing every kernel launch with HIP events
 * on the context stream; returns the summed device time (ms) of the fluid
 * passes and of the boundary passes, and the number of launches of each.
 * Synchronises.
 */
int lbm_profile_steps(lbm_ctx* ctx, int n, double* fluid_ms, double* boundary_ms, int* fluid_launches,
                      int* boundary_launches);

/*
 * Host-only: the fluid pass's work split for a grid, without touching the
 * device.  tile_rows 8, 10, 12 or 13, or 0 for the planner's own choice (a
 * context with tile_rows = 0 times the heights instead); cus = compute units
 * of the device.
 * out = {tile rows, tiles along x (64 cells each), tiles along y, z segments
 * per tile, workgroups launched, tail planes, tail workgroups}.  The z range
 * below the tail, [0, nz - tail), is cut into the segments: work item q
 * (0 <= q < tiles * segments) is tile q % tiles in z segment q / tiles, and
 * the first workgroups - tail workgroups workgroups take items w, w + that
 * count, ...  When the tail is not empty, tail workgroup j takes z in
 * [nz - tail, nz) of tiles [tiles j / n, tiles (j + 1) / n), n the tail
 * workgroups.  Errors: LBM_ERR_INVALID_ARG.
 */
int lbm_fluid_plan(const int dims[3], int tile_rows, int cus, int out[7]);

/*
 * Device-side dither generator, for known-answer tests: for each of the n
 * host cell indices idx[k] writes the two 32-bit hash words of step t to
 * h_out[2k], h_out[2k+1] (host).  Synchronous.
 */
int lbm_debug_dither(int n, const uint32_t* idx, uint32_t t, uint32_t seed, int mode, uint32_t* h_out);

/* ======================================================================
 * Batched step: many independent small domains advanced together.
 *
 * The same step as above (fluid pass, then the boundary pass over listed
 * cells) applied to `count` periodic domains of their own sizes, relaxation
 * times and solid masks.  One fluid launch covers every domain (a persistent
 * grid walking a host-built list of strips and z runs) and one boundary
 * launch covers every listed cell; lbm_batch_step captures a sequence of
 * steps in a HIP graph once and replays it.  A domain's result is the one the
 * single-domain API gives it with the same options and step count, up to the
 * order of float rounding.
 * ====================================================================== */
typedef struct lbm_batch lbm_batch;

/* Work split of the batched fluid pass (see lbm_batch_tune). */
typedef struct lbm_batch_tuning {
  int block;         /* threads per fluid workgroup: 256, 512 or 1024 */
  int wg_per_cu;     /* persistent workgroups per compute unit */
  int workgroups;    /* workgroups launched */
  int segments;      /* (strip, z run) work units in the split */
  double balance;    /* mean / largest workgroup load of the split (1 = even) */
  double fluid_ms;   /* measured fluid-pass time of this split (0 if not timed) */
  int from_cache;    /* 1: read from the autotune cache instead of measured */
} lbm_batch_tuning;

/*
 * Creates a batch of `count` (1..65535) domains.  dims: 3*count ints (nx, ny,
 * nz of each domain, each 1..65535; nx <= 341 unless nx*ny <= 1024); taus:
 * count relaxation times > 1/2; masks: NULL, or count host pointers, each NULL
 * (no solids) or nx*ny*nz bytes of 0/1 (copied).  Total cells <= 2^30.
 * moment_format as in lbm_create.  Every domain starts at rest; every axis is
 * periodic.  Errors: LBM_ERR_INVALID_ARG, LBM_ERR_OUT_OF_MEMORY, LBM_ERR_DEVICE.
 */
int lbm_batch_create(int count, const int* dims, const double* taus, const uint8_t* const* masks,
                     int moment_format, lbm_batch** out);
int lbm_batch_destroy(lbm_batch* b);
const char* lbm_batch_last_error(const lbm_batch* b);
int lbm_batch_set_stream(lbm_batch* b, void* hip_stream);
/* dither_mode, seed and check_health as in lbm_options; inflow and force
 * must be 0 (LBM_ERR_UNSUPPORTED otherwise) and tile_rows 0
 * (LBM_ERR_INVALID_ARG otherwise). */
int lbm_batch_set_options(lbm_batch* b, const lbm_options* opt);
int lbm_batch_get_options(const lbm_batch* b, lbm_options* opt);
/* dims of domain d, its first cell in the batch's planes and its cell count. */
int lbm_batch_info(const lbm_batch* b, int d, int dims[3], int64_t* offset, int64_t* cells);
int lbm_batch_total_cells(const lbm_batch* b, int64_t* cells);
/* Per-domain state access, with the layouts and conventions of the
 * single-domain calls of the same names (d = domain index). */
int lbm_batch_set_moments(lbm_batch* b, int d, const float* m, int on_device);
int lbm_batch_set_equilibrium(lbm_batch* b, int d, const float* rho, const float* u, int on_device);
int lbm_batch_get_moments(lbm_batch* b, int d, float* m, int on_device);
size_t lbm_batch_raw_bytes(const lbm_batch* b, int d);
int lbm_batch_get_raw(lbm_batch* b, int d, void* out, size_t bytes, int on_device);
int lbm_batch_set_raw(lbm_batch* b, int d, const void* in, size_t bytes, int on_device);
/*
 * Advances every domain n steps, asynchronously on the batch stream: up to
 * 256 steps are captured once per (length, buffer parity) in a HIP graph and
 * replayed (the dither key of each step is read from a device-side step
 * counter, so a graph is valid at any step).  With check_health set, the
 * state is scanned once at the end (synchronising).
 */
int lbm_batch_step(lbm_batch* b, int n);
/* The same n steps launched one kernel at a time (no graph). */
int lbm_batch_step_eager(lbm_batch* b, int n);
/* n eager steps with HIP events around each launch; sums of the fluid and
 * boundary launch times in ms.  Synchronous. */
int lbm_batch_profile_steps(lbm_batch* b, int n, double* fluid_ms, double* boundary_ms);
int lbm_batch_get_step_count(const lbm_batch* b, uint64_t* t);
int lbm_batch_set_step_count(lbm_batch* b, uint64_t t);
/* Sizes of the batch's boundary list: fluid cells the boundary pass recomputes,
 * and solid cells next to fluid (the fluid pass stores every solid cell as the
 * rest state, so the boundary pass visits none of them). */
int lbm_batch_boundary_counts(const lbm_batch* b, int64_t* fluid_cells, int64_t* solid_cells);
int lbm_batch_memory_bytes(const lbm_batch* b, size_t* state_bytes, size_t* total_bytes);
int lbm_batch_check(lbm_batch* b, uint64_t* bad);
int lbm_batch_synchronize(lbm_batch* b);
/*
 * Autotuner: times the fluid pass under every workgroup shape that fits
 * every domain (256, 512 or 1024 threads; 1, 2 or 4 per CU as occupancy
 * allows) on the current state (writing only the idle buffer) and keeps the
 * fastest.  cache_path (or, when NULL, the LBM_AUTOTUNE_CACHE environment
 * variable; neither: no cache) names a JSON file keyed by device, format and
 * domain shapes: a hit applies the stored shape without timing, a miss adds
 * the result.  *result (may be NULL) receives the chosen split.
 */
int lbm_batch_tune(lbm_batch* b, const char* cache_path, lbm_batch_tuning* result);
int lbm_batch_get_tuning(const lbm_batch* b, lbm_batch_tuning* t);
int lbm_batch_set_tuning(lbm_batch* b, int block, int wg_per_cu);
/*
 * Host-only: the work split for domains `dims` (3*count ints) with `block`
 * threads per workgroup and nwg workgroups, without touching the device.
 * On entry *n_segments is the capacity of `segments` (4 uint16 per segment:
 * domain, strip, first plane, end plane; may be NULL to query the count);
 * wg_first (nwg + 1, may be NULL) receives each workgroup's first segment;
 * strips (3*count, may be NULL) receives rows loaded, output rows and the
 * whole-plane flag of each domain's strips; balance as in lbm_batch_tuning.
 */
int lbm_batch_plan(int count, const int* dims, int block, int nwg, int* n_segments, uint16_t* segments,
                   uint32_t* wg_first, int* strips, double* balance);

#ifdef __cplusplus
}
#endif

#endif /* HOMELBM_H */
