/*
 * flood.h -- C interface of libflood, the MI355X (gfx950) library for the
 * explicit local-inertial shallow-water flood step of Pierce et al.,
 * "Accelerating Physics Simulations with TPUs: An Inundation Modeling
 * Example" (arXiv 2204.10323).
 *
 * What one step computes (Methods, "Shallow Water Equations"):
 *   1. dt: a fixed step (the paper's results use 0.1 s at 1 m) or the
 *      CFL-limited step min(dt_max, alpha*dx/sqrt(g*h_max)), shortened so the
 *      run ends exactly at t_end (Appendix, DynamicStepUpdater).
 *   2. boundary faces (eq. 5, 6): the inflow section receives Q_in(t) split
 *      over its cells by solving for the water level W of eq. (6); each outflow
 *      cell passes the Manning discharge of its own depth; every other border
 *      face is a closed wall.
 *   3. interior faces, eq. (3): semi-implicit update of the discharge per unit
 *      width from the water-surface gradient with Manning friction, using the
 *      flow depth h_f = max(eta_L, eta_R) - max(z_L, z_R) of the face.
 *   4. donor-cell scaling of outgoing discharges so that no cell sends out more
 *      water than it holds (keeps depths non-negative, conserves volume).
 *   5. depth update, eq. (4), from the discharge divergence.
 *   6. the deepest cell of the new state (for the next CFL step) and the FP64
 *      volume budget of the applied boundary discharges.
 *
 * Conventions
 *   Grids are nx columns (x, contiguous in memory) by ny rows (y), square
 *   cells of side dx metres.  Cell (i, j) is row j, column i.  Discharges are
 *   per unit width (m^2/s), positive toward +x / +y.  Discharge arrays
 *   exchanged through this interface include the border faces:
 *     qx: ny rows of nx+1 faces, qx[j][i] between cells i-1 and i
 *         (i = 0 is the west border, i = nx the east border);
 *     qy: ny+1 rows of nx faces, qy[j][i] between rows j-1 and j
 *         (j = 0 is the south border, j = ny the north border).
 *   Element type of every field is float for FL_F32 contexts and double for
 *   FL_F64 contexts.  Row strides are in elements.
 *   A pointer passed with on_device = 1 (and the memory of fl_bind_workspace)
 *   must be device or managed memory of the context's device: anything else
 *   is refused with EINVAL before it is read or written.  Host pointers may be
 *   any host memory.  The interface takes no sizes for arrays: each must hold
 *   the rows and columns its call describes.
 *
 * Ownership: every fl_set_* call copies its input; the caller keeps its
 * buffers.  Device memory of a context belongs to the context and is freed by
 * fl_destroy.  A batch borrows its member contexts, which must outlive it.
 *
 * Asynchrony: fl_step, fl_advance's launches and fl_batch_run enqueue work on
 * the context's stream and return.  fl_get_* and fl_get_report synchronise
 * that stream.
 *
 * Errors: every call returns a status; nothing aborts, exits or throws across
 * the interface.  fl_last_error gives a message for the last failure on a
 * context (or, for a NULL context, the last failure of fl_create on the
 * calling thread).  A context is not thread-safe; distinct contexts are
 * independent.
 */
#ifndef FLOOD_H
#define FLOOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_ctx fl_ctx;
typedef struct fl_batch fl_batch;

typedef enum {
    FL_OK = 0,
    FL_EINVAL = 1,      /* an argument is out of range (see each call) */
    FL_ENOMEM = 2,      /* device or host allocation failed */
    FL_EHIP = 3,        /* a HIP runtime call failed; message has hipGetErrorString */
    FL_ESTATE = 4,      /* call out of order (e.g. stepping before fl_commit) */
    FL_ENONFINITE = 5   /* a depth became NaN or infinite; the clock has stopped */
} fl_status;

typedef enum { FL_F32 = 0, FL_F64 = 1 } fl_precision;

/* Boundary side of the grid ("BoundarySide" input of the paper's Appendix). */
typedef enum { FL_WEST = 0, FL_EAST = 1, FL_SOUTH = 2, FL_NORTH = 3 } fl_side;

/*
 * Run parameters (Appendix "Inputs": dt, start time, num_secs).
 *   g          gravitational acceleration, m/s^2 (> 0; 9.81 by default)
 *   alpha      CFL number of the variable step, in (0, 1]
 *   dt_max     largest step, s (> 0); used when the grid is dry
 *   h_eps      a face with flow depth h_f <= h_eps is dry (>= 0, metres)
 *   dt_fixed   > 0: use this constant step (the paper's mode); 0: CFL step
 *   t_end      absolute end time, s; +inf for none.  Steps after t_end have
 *              dt = 0 and leave the state unchanged.
 *   steps_per_graph  steps captured per HIP graph replay (rounded up to a
 *              multiple of 6; 0 selects 60)
 *   positivity 1: donor-cell scaling on (default); 0: off
 */
typedef struct {
    double g, alpha, dt_max, h_eps, dt_fixed, t_end;
    int32_t steps_per_graph;
    int32_t positivity;
} fl_params;

/* State of the clock and the FP64 volume budget (m^3). */
typedef struct {
    double t;            /* simulated time, s */
    double last_dt;      /* dt of the last step taken, s */
    int64_t steps;       /* steps taken with dt > 0 */
    double v0;           /* volume at commit */
    double v_in;         /* inflow volume applied since commit */
    double v_out;        /* outflow volume applied since commit */
    double v_now;        /* current volume, dx^2 * sum(h), summed in FP64 */
    int32_t done;        /* 1 once t reached t_end */
    int32_t nonfinite;   /* 1 if a depth became NaN/inf (steps stop) */
} fl_report;

/* Fill *p with the defaults: g 9.81, alpha 0.7, dt_max 0.1, h_eps 1e-4,
 * dt_fixed 0, t_end +inf, steps_per_graph 60, positivity 1. */
void fl_default_params(fl_params *p);

/*
 * Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (for example PyTorch's current stream) or NULL to have the
 * context create its own.  EINVAL: bad device or precision.  EHIP: HIP error.
 */
fl_status fl_create(fl_ctx **ctx, int device, void *hip_stream, fl_precision prec);

/* Grid of nx x ny cells of side dx metres: the raster of square cells on
 * which eqs. (3)-(4) are discretised (Methods, "Shallow Water Equations"),
 * with dx the DEM's "resolution" input (Appendix, "Inputs").  EINVAL: nx or
 * ny < 1, dx <= 0 or not finite, nx + 264 > 2^28 or ny + 8 > 2^30.  Resets
 * everything set before (DEM, roughness, boundaries, state). */
fl_status fl_init_grid(fl_ctx *ctx, int32_t nx, int32_t ny, double dx);

/* Bed elevation z (metres, "unpadded_dem"), ny rows of row_stride elements,
 * host or device memory (on_device = 1).  EINVAL: NULL, row_stride < nx, or a
 * non-finite value. */
fl_status fl_set_dem(fl_ctx *ctx, const void *z, int64_t row_stride, int on_device);

/* Per-cell Manning coefficient n (s m^-1/3), same layout.  EINVAL: n <= 0 or
 * not finite. */
fl_status fl_set_manning(fl_ctx *ctx, const void *n, int64_t row_stride, int on_device);

/*
 * Inflow section (eq. 6): cells first .. first+count-1 along `side`
 * (rows for west/east, columns for south/north), channel slope `slope` and
 * the hydrograph Q_in(t) as nsamples pairs (t_s seconds, q_m3s m^3/s), host
 * memory.  Q_in is piecewise linear between samples and constant outside.
 * count = 0 removes the inflow.  EINVAL: section outside the side, slope <= 0,
 * Q < 0 or not finite, times not strictly increasing, nsamples < 1 or > 4096.
 */
fl_status fl_set_inflow(fl_ctx *ctx, fl_side side, int32_t first, int32_t count, double slope,
                        const double *t_s, const double *q_m3s, int32_t nsamples);

/* Outflow section: each cell passes the Manning discharge of its own depth
 * with slope `slope`, outward only.  count = 0 removes it.  EINVAL: section
 * outside the side, slope <= 0, or overlap with the inflow section. */
fl_status fl_set_outflow(fl_ctx *ctx, fl_side side, int32_t first, int32_t count, double slope);

/* EINVAL: g <= 0, alpha outside (0, 1], dt_max <= 0, h_eps < 0, dt_fixed < 0,
 * t_end NaN. */
fl_status fl_set_params(fl_ctx *ctx, const fl_params *p);

/*
 * Initial state: depth h (ny x nx, row stride nx), discharges qx (ny x (nx+1))
 * and qy ((ny+1) x nx) in the layout described above (NULL = zero), and the
 * time t.  Border-face discharges are accepted but recomputed by the boundary
 * conditions each step.  EINVAL: h < 0 or any value not finite.
 * Without this call the grid starts dry and still at t = 0.
 */
fl_status fl_set_state(fl_ctx *ctx, const void *h, const void *qx, const void *qy, double t,
                       int on_device);

/* Device memory for the buffers fl_commit allocates, for a caller that owns
 * its memory (for example a PyTorch tensor):
 * fl_workspace_bytes gives the bytes a grid needs (0 for invalid arguments);
 * flags: FL_WS_TWO_STEP adds the buffers of fl_set_fusion(ctx, 2 or 3, ...),
 * FL_WS_ACTIVE_TILES those of fl_set_active_tiles(ctx, 1).
 * fl_bind_workspace makes the following commits carve their buffers from
 * dev_ptr (256-byte aligned, on the context's device) instead of allocating;
 * the caller keeps ownership and must keep the memory alive until fl_destroy,
 * another bind or fl_init_grid (which unbinds).  NULL unbinds.  Binding
 * frees the current device buffers, so a commit must follow.  Reverse mode
 * (fl_adj_setup) still allocates its checkpoints itself.  ESTATE before
 * fl_init_grid; EINVAL: misaligned or smaller than fl_workspace_bytes (flags
 * 0); fl_commit returns EINVAL if the workspace is smaller than its flags
 * need. */
#define FL_WS_TWO_STEP 1u
#define FL_WS_ACTIVE_TILES 2u
size_t fl_workspace_bytes(int32_t nx, int32_t ny, fl_precision prec, uint32_t flags);
fl_status fl_bind_workspace(fl_ctx *ctx, void *dev_ptr, size_t bytes);

/* Validate, allocate device memory, upload, reset clock and budget, capture
 * the multi-step graph: the set-up the paper's run_simulation performs before
 * stepping (Appendix, "Code structure": DEM, Manning matrix, boundary
 * conditions of eqs. 5-6, initial state).  Must follow fl_init_grid,
 * fl_set_dem and fl_set_manning (ESTATE otherwise).  Any fl_set_* after
 * commit needs a new commit before stepping.  The context's device memory
 * (or the bound workspace) holds the state; nothing is allocated by later
 * steps. */
fl_status fl_commit(fl_ctx *ctx);

/* Enqueue nsteps steps (graph replays plus single launches).  Each step is
 * the explicit update of Methods, "Shallow Water Equations": boundary faces
 * (eqs. 5, 6), interior faces (eq. 3), donor scaling, depths (eq. 4), with dt
 * from the device clock (the paper's time step, Methods and Appendix,
 * "Inputs").  Asynchronous on the context's stream, except with several steps
 * per launch (fl_set_fusion), which synchronises before it returns.  ESTATE
 * before commit.  EINVAL: nsteps < 0. */
fl_status fl_step(fl_ctx *ctx, int64_t nsteps);

/* Advance the simulated time by `seconds` (the last step shortened to land on
 * it), like the paper's DynamicStepUpdater.  Synchronises periodically to
 * watch the clock; returns when the target time is reached (or a non-finite
 * depth stopped the clock: ENONFINITE). */
fl_status fl_advance(fl_ctx *ctx, double seconds);

/* Copy the current depth h (the water height of eq. 4; the "height of the
 * water" output, Appendix, "Outputs") into dst (ny rows of row_stride
 * elements, host or device memory owned by the caller).  Synchronises.
 * EINVAL: NULL dst or row_stride < nx; ESTATE before commit. */
fl_status fl_get_depth(fl_ctx *ctx, void *dst, int64_t row_stride, int on_device);

/* Copy the current face discharges q_x, q_y of eq. (3) (the "flux in the x
 * and y directions" output, Appendix, "Outputs"), border faces included, in
 * the layout above; caller-owned host or device memory.  Synchronises.
 * EINVAL: a NULL output; ESTATE before commit. */
fl_status fl_get_discharge(fl_ctx *ctx, void *qx, void *qy, int on_device);

/* The whole state of eqs. (3)-(4) (Appendix, "Outputs": h, q_x, q_y) in the
 * layout fl_set_state takes: depth h (ny x nx), qx
 * (ny x (nx+1)) and qy ((ny+1) x nx) with the border faces, and the time t;
 * any of them may be NULL (qx and qy together).  Host or device memory.
 * Synchronises.  ENONFINITE if a depth became non-finite (the outputs are
 * still filled).  Feeding the result to fl_set_state on a context with the
 * same inputs continues the run bit for bit. */
fl_status fl_get_state(fl_ctx *ctx, void *h, void *qx, void *qy, double *t, int on_device);

/* Clock and volume budget.  Synchronises.  ENONFINITE if a depth became
 * non-finite (the report is still filled). */
fl_status fl_get_report(fl_ctx *ctx, fl_report *r);

/* Message of the last failure on ctx (ctx NULL: last fl_create failure on
 * this thread).  Never NULL. */
const char *fl_last_error(const fl_ctx *ctx);

/* Free the context and its device memory (synchronises first).  NULL is a no-op. */
void fl_destroy(fl_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* Timing helper used by the benchmark: enqueue nsteps steps exactly as
 * fl_step does, bracketed by HIP events recorded on the context's stream, and
 * return the elapsed milliseconds (synchronises).  */
fl_status fl_time_steps(fl_ctx *ctx, int64_t nsteps, double *elapsed_ms);

/* Launch configuration of the step kernel: cells per lane along x (1, 2, 4)
 * and rows per work item (>= 1).  Takes effect at the next fl_commit. 0 keeps
 * the default.  EINVAL: unsupported value. */
fl_status fl_set_tiling(fl_ctx *ctx, int32_t cells_per_lane, int32_t rows_per_item);

/* Steps per launch of fl_step and fl_time_steps: 1 (default), 2 or 3, and
 * the tiling of the multi-step kernel (0 = default: 2 cells per lane in FP32,
 * 1 in FP64; rows as fl_set_tiling).  With k > 1, one launch reads the state
 * once and makes up to k steps (Methods, eqs. 3-6, applied k times), dividing
 * the HBM traffic per step by k.  The dt of every step after a launch's first
 * is taken as if the deepest cell of the state before it were shallow (the
 * paper's fixed dt is never shortened by depth); the next launch checks each
 * against that state's actual maximum and, at the first that differs, redoes
 * the launch up to that step from the kept input.  Under the CFL clock a
 * launch makes fewer steps when the bound is close to active.  Results are
 * bitwise those of one step per launch.  fl_step then synchronises the
 * context's stream before it returns; a count of 1 still makes a
 * single-step launch.  fl_advance, fl_autotune and reverse mode use
 * single-step launches, batches one, two or three steps per queue entry
 * (fl_batch_set_fusion).  4 cells per lane allow at most 2 (fl_commit:
 * EINVAL otherwise).  Takes effect at the next fl_commit.
 * EINVAL: steps_per_launch not 1, 2 or 3, an unsupported tiling. */
fl_status fl_set_fusion(fl_ctx *ctx, int32_t steps_per_launch, int32_t cells_per_lane,
                        int32_t rows_per_item);

/* Method variants, to check how much results depend on two readings of the
 * paper (Methods, "Shallow Water Equations").  Defaults: FL_FRICTION_FACE, the
 * face's own |q| in the friction term of eq. (3) (the per-axis 1-D form the
 * paper describes); FL_BOUNDARY_SECTION, A in eq. (5)/(6) is the face's
 * cross-section dx*h, so a boundary cell passes h^{5/3} sqrt(S)/n per unit
 * width (the steady state of eq. 3 itself).
 *   FL_FRICTION_VECTOR: |q| is the magnitude of the discharge vector at the
 *     face (the vector norm of eq. 2), sqrt(q^2 + q_perp^2), where q_perp is
 *     the mean of the start-of-step discharges on the perpendicular faces of
 *     the two cells beside the face; faces on the border of the grid are left
 *     out of the mean (4 faces inside, 2 along the border).
 *   FL_BOUNDARY_CELL_AREA: eq. (5)/(6) as printed, A = dx^2 and the hydraulic
 *     radius = the depth: a boundary cell passes dx^2 h^{2/3} sqrt(S)/n, i.e.
 *     dx h^{2/3} sqrt(S)/n per unit width of its face; W of eq. (6) is then
 *     bisected 64 times in FP64.
 * Variants run one step per launch (fl_step, fl_advance, fl_time_steps,
 * fl_autotune); fl_commit fails with EINVAL with several steps per launch or
 * active tiles, fl_batch_create with a member that has a variant, and
 * fl_adj_setup on such a context.  Takes effect at the next fl_commit.
 * EINVAL: an unknown value. */
typedef enum { FL_FRICTION_FACE = 0, FL_FRICTION_VECTOR = 1 } fl_friction;
typedef enum { FL_BOUNDARY_SECTION = 0, FL_BOUNDARY_CELL_AREA = 1 } fl_boundary;
fl_status fl_set_variant(fl_ctx *ctx, int32_t friction, int32_t boundary);

/* Active-tile skipping (wet-region skipping) for fl_step, fl_time_steps,
 * fl_advance and the forward of reverse mode, with one, two or three steps
 * per launch.  A launch does not recompute a work item when no water can reach
 * it: every face between two cells without water is dry in eq. (3) (its
 * water-surface height above the higher bed is <= 0), so no water moves, and
 * the outflow of eq. (5) is zero for an empty edge cell.  One step per launch
 * skips an item when the item and the four items that share an edge with it
 * held no water (h <= 0), kept their depths and carried no discharge in the
 * step before, and the item itself also in the step before that.  Two or
 * three steps per launch reach two or three cells further, so they look at
 * the 3 x 3 items around it, by launch (a launch that redoes a guessed later
 * step skips exactly what the launch it replaces skipped).  Items behind an inflow face (eq. 6)
 * are always computed.  Each item records one flag byte per step or launch
 * (three kept).  Results are the values of computing every item (a zero may
 * differ in sign; after a non-finite depth, which stops the clock, the states
 * may differ).  Work scales with the wet area (a flood on a mostly dry DEM)
 * instead of the grid.  Another path that moves the state (batches, frozen
 * tiling trials, the reverse sweep, switching between one and several steps
 * per launch) marks the flags stale; the next skipping launch then computes
 * every item for two launches.  fl_autotune and fl_autotune_fusion time
 * skipping trial steps.
 * on: 0 off; 1 on, each work item of a single-step launch makes the skip
 * test itself (one wave per item); 2 on, single-step launches first select
 * the items to compute (one thread per item, an ordered list) and a
 * persistent grid computes the list, which is faster when few items hold
 * water.  fl_autotune times both and keeps the faster with the tiling.
 * Several steps per launch and batches always use the per-item test.  Takes
 * effect at the next fl_commit, which fails with EINVAL for k steps per
 * launch with work items of fewer than k rows.  EINVAL: on not 0, 1 or 2. */
fl_status fl_set_active_tiles(fl_ctx *ctx, int32_t on);

/* Work items the next launch computes under active-tile skipping
 * (*next_items) and work items of a launch (*total_items): those of the
 * multi-step kernel after a multi-step run, else of the single-step kernel.
 * Synchronises.  ESTATE: not committed with active tiles on (mode 1 or 2).
 * EINVAL: a NULL output. */
fl_status fl_active_items(fl_ctx *ctx, int64_t *next_items, int64_t *total_items);

/* Time each (cells_per_lane, rows_per_item) pair of candidates[2*ncand] over
 * trial_steps frozen steps (dt = 0: the state is streamed like a real step but
 * left unchanged) and keep the fastest for the following steps (the captured
 * graph is rebuilt).  With active tiles on, the trial steps skip work items as
 * real steps would, so the choice fits the current wet extent (small items
 * when few items hold water, large ones when many do); call it again as the
 * flood grows.  best[2] receives it, *best_ms its time per step.  The state,
 * clock and budget are unchanged.  ESTATE before commit; EINVAL: a candidate
 * fl_set_tiling would reject. */
fl_status fl_autotune(fl_ctx *ctx, const int32_t *candidates, int32_t ncand, int32_t trial_steps,
                      int32_t *best, double *best_ms);

/* Time one step per launch (the current tiling) against the committed k
 * steps per launch (fl_set_fusion; its tiling) over trial_steps frozen steps
 * each (dt = 0:
 * the state is streamed but left as it is), and keep the faster for the
 * following fl_step calls; both give the same bits.  With active tiles the
 * trial steps skip as real steps would (after untimed steps that set the
 * flags).  Two steps per launch pay off on large grids that HBM bandwidth
 * bounds, and under active tiles when many items hold water; small,
 * cache-resident or nearly dry grids can be faster with one.  *steps_per_launch receives the choice (1 or k),
 * *ms_per_step its time per step.  ESTATE: not committed, or committed
 * without fl_set_fusion(ctx, 2 or 3, ...) (the multi-step buffers).  EINVAL:
 * trial_steps < 2. */
fl_status fl_autotune_fusion(fl_ctx *ctx, int32_t trial_steps, int32_t *steps_per_launch,
                             double *ms_per_step);

/* Bytes of device memory the context holds after commit. */
size_t fl_device_bytes(const fl_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* Reverse mode: gradients of a gauge misfit with respect to the per-cell
 * Manning n and the inflow hydrograph samples, for runs with a fixed time
 * step (the paper's constant-dt mode, Methods).  Motivated by calibration
 * (Introduction) and data assimilation (Future Work).  The forward run keeps
 * checkpoints of the state every ckpt_stride steps (default ceil(sqrt(N)));
 * the backward sweep recomputes one segment at a time and reverses its steps
 * with hand-written adjoint kernels.  Gradients are accumulated in FP64. */

/* Gauges (flat cell indices j*nx + i, host memory) observed after every
 * obs_every steps; obs [nobs][ngauges] (element type of the context, host or
 * device) are the observations of the squared misfit, or NULL when the caller
 * supplies dL/dseries to fl_adj_backward.  EINVAL: dt_fixed == 0, no gauges,
 * a gauge outside the grid, obs_every < 1, ckpt_stride < 0.  ESTATE: not
 * committed. */
fl_status fl_adj_setup(fl_ctx *ctx, const int32_t *gauge_cells, int32_t ngauges, int32_t obs_every,
                       const void *obs, int64_t nobs, int obs_on_device, int32_t ckpt_stride);

/* Run nsteps steps from the current state, keeping checkpoints; series
 * [nsteps/obs_every][ngauges] receives the gauge depths (host or device, may
 * be NULL); *loss = sum (series - obs)^2 if observations were set, else 0.
 * Synchronises.  EINVAL: t_end inside the run, too few observations. */
fl_status fl_adj_forward(fl_ctx *ctx, int64_t nsteps, void *series, int on_device, double *loss);

/* Gradients of the last fl_adj_forward run: dl_dseries [nobs][ngauges]
 * (element type of the context, host or device) are the adjoint seeds, or
 * NULL for the squared misfit against the observations.  grad_n receives
 * dL/dn [ny][nx] in FP64 (host or device), grad_q (host, may be NULL) dL/dQ_k
 * for each hydrograph sample.  The context is left at the end of the forward
 * run.  ESTATE: no forward run, or the context was stepped since. */
fl_status fl_adj_backward(fl_ctx *ctx, const void *dl_dseries, double *grad_n, int grad_on_device,
                          double *grad_q);

/* ---------------------------------------------------------------------- */
/* Batched ensemble: many independent committed contexts (same device and
 * precision, any sizes) stepped together by ONE persistent launch.  Members
 * run the same kernels as fl_step, so each member's result is bitwise the
 * result of stepping it alone; a member's step k waits only for its own step
 * k-1, never for the other members.  Members with active tiles skip the work
 * items no water can reach, in the batch as in their own steps; members
 * without are computed in full.  The batch borrows its members: they must
 * outlive it and stay committed.  Motivated by the what-if and
 * parameter-space ensembles the paper points to (Broader Impacts, Future
 * Work). */

/* Create a batch of nmembers committed contexts.  EINVAL: no members,
 * mixed devices or precisions, a context listed twice, a member with a method
 * variant (fl_set_variant).  ESTATE: a member not committed. */
fl_status fl_batch_create(fl_batch **batch, int32_t nmembers, fl_ctx *const *members);

/* Work decomposition of the batch launch: cells per lane along x (1, 2, 4;
 * FP64: 1, 2) and rows per work item (>= 1).  Default 4 (FP64 2) and 16. */
fl_status fl_batch_set_tiling(fl_batch *batch, int32_t cells_per_lane, int32_t rows_per_item);

/* Steps per queue entry of the batch launch: 1 (default), 2 or 3.  With k > 1
 * every member makes the k-step launches of fl_set_fusion(ctx, k, ...) (one
 * read and one write of its state per k steps of Methods, eqs. 3-6; under the
 * CFL clock the later steps' dts are speculated, checked by the member's next
 * launch and redone if wrong) inside the one persistent launch, so members
 * wait for their own previous launch k times less often; results stay bitwise
 * those of stepping each member alone.  Every member must have been committed
 * after fl_set_fusion(ctx, 2 or 3, ...) (ESTATE otherwise) and run without
 * active tiles (EINVAL).  cells_per_lane (1 or 2; 0: 2 in FP32, 1 in FP64)
 * and rows_per_item (>= 1; 0: 64) are the multi-step tiling, which
 * fl_batch_autotune then tunes.  fl_batch_run_noalloc always runs one step
 * per entry.  EINVAL: other values. */
fl_status fl_batch_set_fusion(fl_batch *batch, int32_t steps_per_entry, int32_t cells_per_lane,
                              int32_t rows_per_item);

/* Time each (cells_per_lane, rows_per_item) pair of candidates[2*ncand] over
 * trial_steps frozen steps (dt = 0: the state is streamed like a real step
 * but left unchanged) and keep the fastest (the two-step tiling when the batch
 * runs two steps per entry, fl_batch_set_fusion).  Members with active tiles first
 * take two untimed frozen steps per candidate, so that the timed ones skip
 * as real steps would.  best[2] receives it, *best_ms its time per step.  The
 * members' states and clocks are unchanged. */
fl_status fl_batch_autotune(fl_batch *batch, const int32_t *candidates, int32_t ncand,
                            int32_t trial_steps, int32_t *best, double *best_ms);

/* Advance every member by nsteps steps in one launch.  Synchronises the
 * members' streams first and the batch's stream at the end.  EHIP if the
 * launch fails or a wait ran into its limit. */
fl_status fl_batch_run(fl_batch *batch, int64_t nsteps);

/* fl_batch_run for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and the same results, bit for bit, but the launch's scratch (member
 * descriptors, queue heads, per-member completion counters, the error flag)
 * lives in a library-owned static device array of 1 MiB per GPU, cleared by
 * a kernel at each call, and the descriptors are staged through pinned host
 * memory that fl_batch_create allocated; the call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  The array is held until
 * the process ends and is shared by every call on that GPU: calls that
 * overlap on one GPU (from several threads or streams) race and must not be
 * issued.  Synchronises like fl_batch_run.  EINVAL: nsteps < 0, or more than
 * FL_NOALLOC_MAX_MEMBERS members; ESTATE: a member not committed; EHIP as
 * fl_batch_run.  Always one step per queue entry (fl_batch_set_fusion does not
 * apply; the results are the same bits). */
#define FL_NOALLOC_MAX_MEMBERS 256
fl_status fl_batch_run_noalloc(fl_batch *batch, int64_t nsteps);

/* fl_batch_run bracketed by HIP events; returns the launch's milliseconds. */
fl_status fl_batch_time(fl_batch *batch, int64_t nsteps, double *elapsed_ms);

/* Message of the last failure on the batch (NULL: last fl_batch_create failure). */
const char *fl_batch_last_error(const fl_batch *batch);

/* Free the batch (not its members).  NULL is a no-op. */
void fl_batch_destroy(fl_batch *batch);

#ifdef __cplusplus
}
#endif
#endif /* FLOOD_H */
