/*
 * biotlbm.h -- C ABI of the MI355X (gfx950) solver for the semi-implicit lattice
 * Boltzmann scheme for Biot's consolidation model of Lunowa & Wohlmuth,
 * "A lattice Boltzmann method for Biot's consolidation model of linear
 * poroelasticity" (arXiv:2409.11382).
 *
 * Problem (Sec. 2.1, eqs. 1-4): find displacement eta and pressure p with
 *   -div sigma + alpha grad p = f,  sigma = lambda div(eta) I + mu (grad eta + grad eta^T),
 *   d/dt (c0 p + alpha div eta) + div u = s,  u = -kappa grad p,
 * on a rectangle of nx x ny cells of width dx, time step dt, with periodic,
 * Dirichlet or Neumann (no-flow / traction) boundary conditions (Sec. 3.6) and a
 * symmetry (roller, impermeable mirror) condition.
 *
 * Method per time step (Algorithm 5): explicit force, N_E multigrid cycles
 * (Algorithm 4) of the pseudo-time MRT elasticity LBM (Algorithm 2, Tables 2-3),
 * then one SRT flow step (Algorithm 3) with the centred coupling source
 * (eq. source:implicit, ratio r).
 *
 * Conventions
 *   - Every function returns a bp_status; nothing throws across the ABI.  On an
 *     error bp_last_error() returns a message for the calling thread.
 *   - Host arrays are row-major [y][x] (x fastest), vector fields component
 *     first; they are read during the call and not retained.
 *   - Device memory: the caller allocates one workspace of bp_workspace_bytes()
 *     bytes (256-byte aligned) and passes it to bp_create; the library never
 *     allocates device memory.  The workspace must outlive the solver.
 *   - All device work is enqueued on the HIP stream given to bp_create
 *     (NULL = legacy default stream).  Calls on one solver are not thread-safe.
 *   - Inputs are dimensional; the library converts to lattice units.
 */
#ifndef BIOTLBM_H
#define BIOTLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BP_OK = 0,
  BP_ERR_ARG = -1,        /* invalid argument or parameter */
  BP_ERR_SHAPE = -2,      /* grid not compatible with the level hierarchy */
  BP_ERR_DEVICE = -3,     /* a HIP call failed */
  BP_ERR_DIVERGED = -4,   /* non-finite populations or residual norms, or (fixed N_E) the
                             norm of the finest populations at the end of a step grown
                             above 1e8 times the largest of its first 16 non-zero
                             step-end values (the coupled scheme's instability, Sec. 4.1) */
  BP_ERR_WORKSPACE = -5,  /* workspace missing, misaligned or too small */
  BP_ERR_STATE = -6       /* solver unusable after an earlier error */
} bp_status;

/* population storage and collision precision; "shifted" stores populations as
 * offsets from a per-cell displacement / pressure reference (re-based at the
 * start of every step, the displacement again before every later V-cycle of
 * the step).  Divergence fields, the coupling source, residual norms and the
 * coarsest multigrid level are FP64 in every mode. */
typedef enum { BP_FP64 = 0, BP_FP32 = 1, BP_FP32_SHIFTED = 2, BP_FP64_SHIFTED = 3 } bp_precision;

/* shape of the multigrid cycle.  The paper gives the V-cycle (Algorithm 4:
 * one visit of the coarser level per cycle) and names W- and F-cycles and
 * full multigrid as future work (Sec. 5) without defining them; they take
 * the textbook form.  W visits the coarser level twice, F makes an F-visit
 * and then a V-visit, the second visit continuing from the first's coarse
 * iterate with the same restricted right-hand side.  Large levels run on the
 * tile kernels; the one-workgroup coarse tail runs the levels of at most 1024
 * cells in any shape (W- and F-visits included), and a problem of at most
 * 1024 cells runs whole cycles of any shape there.  A cycle on L levels
 * solves the coarsest 2^(L-1) (W) or L (F) times, so they pay off only on
 * shallow hierarchies.
 * BP_CYCLE_FMG makes the first cycle of every time step a full-multigrid
 * cycle on the correction of the warm start: the residual is restricted
 * level by level (on coarse levels the residual of a zero iterate), the
 * coarsest level is smoothed from zero, and every finer level takes the
 * prolongated correction as its starting iterate for one V-cycle; later
 * cycles of the step are V-cycles.  Its coarse levels run on the tile
 * kernels.  A batch takes one shape; the server runs V-cycles. */
typedef enum { BP_CYCLE_V = 0, BP_CYCLE_W = 1, BP_CYCLE_F = 2, BP_CYCLE_FMG = 3 } bp_cycle;

/* flow boundary types (Sec. 3.6): periodic, pressure Dirichlet (halfway
 * anti-bounce-back, eq. BC:pressure), no flow (halfway bounce-back,
 * eq. BC:noFlow), symmetry (mirror reflection; impermeable) */
enum { BP_FLOW_PERIODIC = 0, BP_FLOW_DIRICHLET = 1, BP_FLOW_NOFLOW = 2, BP_FLOW_SYMMETRY = 3 };
/* elastic boundary types (Sec. 3.6): periodic, displacement Dirichlet
 * (eq. BC:elasticity), traction (eq. BC:traction), symmetry (roller: zero normal
 * displacement and zero shear traction, mirror reflection) */
enum { BP_EL_PERIODIC = 0, BP_EL_DIRICHLET = 1, BP_EL_TRACTION = 2, BP_EL_SYMMETRY = 3 };
enum { BP_LEFT = 0, BP_RIGHT = 1, BP_BOTTOM = 2, BP_TOP = 3 };

/* One side of the domain.  Left/right arrays have ny entries (indexed by row),
 * bottom/top arrays nx entries (indexed by column); data are given at the face
 * centre of each boundary cell.  Periodic must hold on both opposite sides for
 * both fields. */
typedef struct {
  int32_t el;               /* BP_EL_*, uniform along the side */
  int32_t flow_uniform;     /* BP_FLOW_* used when flow_type is NULL */
  const int8_t *flow_type;  /* per boundary cell BP_FLOW_*, or NULL */
  const double *el_value;   /* 2 per boundary cell: eta_D (Dirichlet) or traction
                               t = sigma n (traction); NULL means zero */
  const double *p_value;    /* 1 per boundary cell: p_D; NULL means zero */
} bp_side;

typedef struct {
  int32_t nx, ny;           /* cells */
  double dx, dt;            /* cell width, time step (> 0) */
  double lambda, mu;        /* Lame coefficients: mu > 0, lambda + mu > 0 */
  double c0;                /* specific storage (> 0; Sec. 2.2 excludes c0 = 0) */
  double alpha;             /* Biot-Willis coefficient in [0, 1] */
  const double *kappa;      /* per-cell permeability (N values) or NULL */
  double kappa_uniform;     /* permeability when kappa is NULL (> 0) */
  const double *body_f;     /* body force f, 2 x N, or NULL (zero) */
  const double *source_s;   /* fluid source s, N, or NULL (zero) */
  double r;                 /* explicit/implicit coupling ratio in [0, 1]; 0.5 = centred */
  int32_t levels;           /* multigrid levels L (0 = as many halvings as keep >= 2 cells) */
  int32_t K;                /* pre- and post-smoothing steps (>= 1) */
  double gamma;             /* smoother under-relaxation in (0, 1] (eq. MG:smoother); 1 with
                               levels = 1 is the plain pseudo-time stepping of Algorithm 1,
                               2K applications per cycle */
  int32_t ne_fixed;         /* > 0: that many V-cycles per time step */
  double ne_tol;            /* ne_fixed == 0: stop when ||g - S(g)|| <= ne_tol ||g|| */
  int32_t ne_max;           /* ne_fixed == 0: at most this many V-cycles */
  bp_side side[4];
  int32_t prec;             /* bp_precision */
  int32_t pressure_gradient; /* gradient of p in the explicit force: 0 = first moments of the
                               flow populations (eq. pressure:gradient), 1 = central
                               difference of p (eq. pressure:gradient:alternative); both
                               add half the central gradient of the source */
  int32_t cycle;            /* bp_cycle: shape of the multigrid cycle (0 = the V-cycle of
                               Algorithm 4) */
  int32_t fstar_literal;    /* self-dependence force f_* of eq. MG:selfdependence with the
                               printed constant alpha^2/2 for every r (1), or with the
                               implicit share r alpha^2/2 of the centred source of
                               eq. source:implicit (0, default; equal for r = 1) */
  int32_t coarse_sweeps;    /* smoothing steps on the coarsest level of a hierarchy
                               (levels >= 2): 0 = the 2K of Algorithm 4, else an even
                               number >= 2 (a batch needs one value and, if > 0, one
                               hierarchy depth) */
  int32_t lag;              /* Algorithm 1 with the lag of eq. source:implicit: the
                               implicit source of pseudo-time step tau uses the
                               divergence of step tau - dtau (a step starts with
                               g(-1) = g(0)); needs levels = 1 and a fixed N_E
                               (single solvers).  0: the current iterate, as the
                               multigrid of Algorithm 4 evaluates f_* */
} bp_problem;

typedef struct bp_solver bp_solver;

typedef struct {
  int32_t step;             /* completed time steps */
  int32_t last_ne;          /* V-cycles of the last step */
  int64_t total_cycles;     /* V-cycles since creation */
  double last_ratio;        /* last ||g - S(g)|| / ||g|| measured (adaptive mode; else -1) */
  int32_t levels;           /* multigrid levels in use */
  int32_t diverged;         /* non-finite norm or growth above 1e8 seen */
  int32_t adaptive_steps;   /* adaptive mode: steps since creation */
  int32_t steps_at_cap;     /* adaptive mode: steps that stopped at ne_max with the
                               ratio still above ne_tol */
  double max_ratio;         /* adaptive mode: largest ratio at the end of a step */
  double mean_ratio;        /* adaptive mode: mean ratio at the end of a step */
} bp_run_stats;

/* Device bytes needed for problem p (host-only, pure). */
bp_status bp_workspace_bytes(const bp_problem *p, size_t *device_bytes);

/* Validate p, convert to lattice units (Sec. 2.2), build the level hierarchy
 * (Sec. 3.5: each coarse cell covers 2x2 fine cells; homogeneous boundary data
 * on coarse levels), upload parameters and boundary data into device_ws and set
 * the initial conditions (eqs. ICs, ICs:moments).  hip_stream is a hipStream_t
 * or NULL.  *out owns host metadata only. */
bp_status bp_create(const bp_problem *p, void *device_ws, size_t ws_bytes, void *hip_stream,
                    bp_solver **out);

/* Advance nsteps coupled time steps (Algorithm 5).  Asynchronous on the
 * solver's stream in fixed-N_E mode (captured HIP graphs of four steps, and
 * of one for the rest).  The adaptive mode (Sec. 3.4 leaves the pseudo-time
 * stopping test open) runs the test on the device and enqueues the cycles in
 * batches: it reads the stop flag once per batch (as many cycles as the
 * fewer of the last two steps needed, then four at a time), or once per step where all of a step's cycles run in one
 * whole-problem launch.  Within one call the flow step and the next step's
 * first cycle are enqueued before each read, gated on a normal stop, so the
 * device does not wait for the host; the call returns with its last step's
 * work enqueued. */
bp_status bp_step(bp_solver *s, int32_t nsteps);

/* Replace body force f and fluid source s of eqs. 1-4 (host arrays, NULL =
 * zero) for the next steps; reinit != 0 also resets the state to the initial
 * conditions of eqs. ICs, ICs:moments, which depend on the loads at t = 0. */
bp_status bp_set_loads(bp_solver *s, const double *body_f, const double *source_s, int32_t reinit);

/* Synchronise and copy the fields of the last completed step n (time n dt):
 * eta (2 x N, eq. displacement with the bared moments of eq. moments:bared),
 * p (N, eq. pressure, before the flow update as Algorithm 5 computes it) and
 * sigma (3 x N: 11, 12, 22, from the bared stress moments of eq.
 * moments:stress) in dimensional units; any pointer may be NULL.  Returns
 * BP_ERR_DIVERGED if the state is not finite or has grown above 1e8 times
 * its first norm. */
bp_status bp_get_fields(bp_solver *s, double *eta, double *p, double *sigma, int32_t *step);

/* Checkpoint access in FP64 component planes: f (9 x N, D2Q9 order of Table 1),
 * g (8 x N, D2Q8 order 10,01,-10,0-1,11,-11,-1-1,1-1, full populations),
 * D1 = D^{n-1}, D2 = D^{n-2} (lattice divergences, N each).  bp_set_state also
 * sets the step counter; a NULL array leaves that part of the state as it is.
 * In shifted storage bp_set_state splits f and g in FP64 into the references
 * the step-start re-base would take (the displacement moments of g, the sum
 * of f) and the offsets from them, so a restored state carries the same
 * rounding as one the solver reached itself. */
bp_status bp_get_state(bp_solver *s, double *f, double *g, double *D1, double *D2, int32_t *step);
bp_status bp_set_state(bp_solver *s, const double *f, const double *g, const double *D1,
                       const double *D2, int32_t step);

/* Single operations on host FP64 planes (lattice units), for inspection:
 * out = S(g) = ELASTIC_STEP(g - r, Ft + F_*(g)) on level l (l = levels is the
 * finest, Algorithm 4 line with g**), one ELASTIC_MULTIGRID cycle on level l
 * (g in/out), and the explicit force of the current state (2 x N).
 * bp_apply_elastic and bp_mg_cycle work in the solver's own buffers: they
 * replace its elastic populations, force and (shifted storage) displacement
 * reference, so a solver that is to step on afterwards needs bp_set_state
 * (or bp_set_loads with reinit) first.  bp_explicit_force leaves the state
 * alone. */
bp_status bp_apply_elastic(bp_solver *s, int32_t level, const double *g, const double *r,
                           const double *Ft, double *out);
bp_status bp_mg_cycle(bp_solver *s, int32_t level, double *g, const double *r, const double *Ft);
bp_status bp_explicit_force(bp_solver *s, double *Ft);
bp_status bp_level_shape(const bp_solver *s, int32_t level, int32_t *nx, int32_t *ny);

/* Run statistics: time steps, the multigrid cycles N_E of Algorithm 5 per
 * step, and the stopping test's ratios of the adaptive mode. */
bp_status bp_stats(const bp_solver *s, bp_run_stats *st);

/* ---- launch shapes and their autotuner.  The time-step schedule picks, per
 * multigrid depth and by the cells the depth covers over all problems, how
 * many smoothing applications one launch does and the region of a block
 * (see the kernels' notes in lbm_engine.h).  These choices change the order
 * of operations only: results agree to rounding (bitwise for the same
 * choices).  Bounds are cell counts; a depth takes:
 *   four applications per launch     if cells <= quad_max_cells
 *   pairs on tall regions            if cells <= tall_max_cells
 *   the restriction fused into the last pre-smoothing launch
 *                                    if cells <= fuse_res_max_cells
 *   four applications with the restriction on 32 x 32 regions
 *                                    if cells <= quad_res_narrow_max_cells
 *                                    (else on 64 x 32 regions)
 * bp_autotune searches the bounds by coordinate descent: each bound in turn
 * takes the value among five candidates whose time steps run fastest on this
 * engine (HIP events, `steps` steps per candidate after one warm-up step; a
 * candidate must beat the best so far by 2%), the others held.  It steps the
 * problems while timing and re-initialises them at the end, so it must be
 * called before the first step (else BP_ERR_STATE) and needs a fixed number
 * of V-cycles (ne_fixed > 0, else BP_ERR_ARG).  *out (may be null) receives
 * the chosen bounds and the measured milliseconds per step.  bp_set_tuning
 * applies bounds (>= 0) at any time, for instance ones found earlier for the
 * same sizes; bp_get_tuning reports the current ones (ms_per_step 0).  The
 * server uses the default bounds. */
typedef struct {
  int64_t quad_max_cells;
  int64_t tall_max_cells;
  int64_t fuse_res_max_cells;
  int64_t quad_res_narrow_max_cells;
  double ms_per_step;
} bp_tuning;
bp_status bp_get_tuning(bp_solver *s, bp_tuning *out);
bp_status bp_set_tuning(bp_solver *s, const bp_tuning *t);
bp_status bp_autotune(bp_solver *s, int32_t steps, bp_tuning *out);

/* Average device time (microseconds, HIP events on the solver's stream) of
 * `iters` back-to-back launches of one kernel on the current state, replayed
 * as one captured graph: which = 0 finest-level smoothing sweep, 1 finest-level
 * residual/restriction, 2 flow step, 3 explicit force, 4 the finest level's
 * multi-application smoothing launch of the time-step schedule (two or four
 * applications).  *bytes receives the algorithmic HBM bytes of one launch:
 * each value the kernel must read or write, once per application (the
 * multi-application launch counts each of its applications).  The state is
 * left unchanged (the smoothing launches' input buffer is not written). */
bp_status bp_time_kernel(bp_solver *s, int32_t which, int32_t iters, double *avg_us, double *bytes);

/* Where a time step's device time goes (measurement of Algorithm 5 as this
 * library schedules it).  Runs `steps` fixed-cycle time steps (they advance
 * the solver like bp_step) with the step's kernels launched directly and a
 * HIP event before every launch; the table has one row per kernel variant
 * and multigrid depth, in order of first launch: launches per step, device
 * time per step (from the launch's event to the next one, so launch gaps
 * are included), and algorithmic bytes per step (each value an application
 * must read or write, once per application: a pair launch counts two
 * applications).  *n_out receives the number of rows; at most cap are
 * written. */
typedef struct {
  char name[48];            /* e.g. "pair shift f32", "quad+restrict f32", "tail", "flow" */
  int32_t depth;            /* multigrid depth of a sweep or the tail's top (0 = finest), else -1 */
  int32_t launches;         /* launches per step */
  double us_per_step;       /* device microseconds per step */
  double bytes_per_step;    /* algorithmic bytes per step */
} bp_kernel_stat;
bp_status bp_profile_step(bp_solver *s, int32_t steps, bp_kernel_stat *out, int32_t cap, int32_t *n_out);
/* the same for a batch (declared below): its time steps' kernels */
typedef struct bp_batch bp_batch;
bp_status bp_batch_profile_step(bp_batch *b, int32_t steps, bp_kernel_stat *out, int32_t cap, int32_t *n_out);

/* Plain device copy of `bytes` (multiple of 16) on a stream; used to calibrate
 * hardware byte counters. */
bp_status bp_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

bp_status bp_destroy(bp_solver *s);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bp_create on a workspace
 * the library owns, a file-scope static device array of 64 MiB per device
 * (held from the library's first use on that device until the process ends;
 * a problem whose bp_workspace_bytes exceed it is refused with
 * BP_ERR_WORKSPACE).  The solver then allocates nothing: no device or pinned
 * host memory, and no captured graphs (its time steps launch their kernels
 * directly, with the same kernels and results as bp_create's solver).  The
 * caller still passes the problem's host arrays and reads the fields with
 * bp_get_fields.  One such solver per device at a time: the array is shared
 * by every call on that device and keeps the last solver's contents, so a
 * second bp_create_static on the same device returns BP_ERR_STATE until
 * bp_destroy releases the first; calls from several threads that would
 * overlap on one device race and must be serialised by the caller.  The
 * workspace is cleared where the solver needs zeros at creation. */
bp_status bp_create_static(const bp_problem *p, void *hip_stream, bp_solver **out);

/* ---- batches: many independent problems advanced together.  Every launch of
 * a time step covers the same multigrid depth of all problems (levels aligned
 * from the finest), so n problems cost about the launches of one.  Problems
 * must share the precision, K and the fixed number of V-cycles; grids,
 * parameters and boundary data may differ.  Each problem's arithmetic is that
 * of solving it alone; results are bitwise identical when the batch leaves the
 * launch variants unchanged (a depth takes four-application launches, fuses
 * the restriction and picks the region width of four applications with the
 * restriction according to the cells it covers in all), and otherwise
 * agree to rounding (operations are fused differently in the variants). */
/* A problem whose state diverges (BP_ERR_DIVERGED above) leaves the batch at
 * the next check (every 8 steps of bp_batch_step, and at its end): its later
 * steps are not run, its fields stay those of the check, bp_batch_get_fields
 * returns BP_ERR_DIVERGED for it, and the others step on unchanged. */
bp_status bp_batch_workspace_bytes(const bp_problem *probs, int32_t n, size_t *device_bytes);
bp_status bp_batch_create(const bp_problem *probs, int32_t n, void *device_ws, size_t ws_bytes,
                          void *hip_stream, bp_batch **out);
bp_status bp_batch_step(bp_batch *b, int32_t nsteps);
bp_status bp_batch_get_fields(bp_batch *b, int32_t i, double *eta, double *p, double *sigma,
                              int32_t *step);
/* the launch-shape tuning of a batch, as for a solver (bp_autotune) */
bp_status bp_batch_get_tuning(bp_batch *b, bp_tuning *out);
bp_status bp_batch_set_tuning(bp_batch *b, const bp_tuning *t);
bp_status bp_batch_autotune(bp_batch *b, int32_t steps, bp_tuning *out);
bp_status bp_batch_destroy(bp_batch *b);

/* ---- serving: continuous batching of solve requests on one GPU.  The caller
 * gives one workspace; the server keeps its own area (descriptors and work
 * lists for up to max_slots problems) at the start and manages the rest as a
 * pool.  bp_server_submit deep-copies the request's host arrays and queues it.
 * Each time step of bp_server_advance first admits queued requests in arrival
 * order while a slot, pool memory (bp_server_request_bytes of the request) and
 * work-list room are free, writes their initial conditions, then advances
 * every admitted request by one coupled step in the same launches (levels
 * aligned from the finest, as in a batch; one captured graph per membership),
 * and finally retires requests that reached their step count: their fields
 * are copied to host memory held by the server and their pool memory is
 * released.  Results equal solving each request alone as in a batch (bitwise
 * when the mix leaves the launch variants unchanged, else to rounding).
 * Requests must use the server's precision, K and fixed V-cycle count.
 * Calls on one server are not thread-safe; all device work runs on hip_stream.
 *
 * A request whose state diverges (BP_ERR_DIVERGED) is failed and retired at
 * the next check, every 8 steps, instead of running to its step count.
 *
 * Request states (bp_server_poll): 0 queued, 1 running, 2 done, 3 failed. */
typedef struct bp_server bp_server;
bp_status bp_server_request_bytes(const bp_problem *p, size_t *device_bytes);
bp_status bp_server_create(void *device_ws, size_t ws_bytes, void *hip_stream, int32_t prec, int32_t K,
                           int32_t ne_fixed, int32_t max_slots, bp_server **out);
bp_status bp_server_submit(bp_server *s, const bp_problem *p, int32_t nsteps, int64_t *ticket);
/* Run up to nsteps time steps (fewer if nothing is left to run); reports the
 * requests running and queued afterwards. */
bp_status bp_server_advance(bp_server *s, int32_t nsteps, int32_t *n_active, int32_t *n_queued);
/* state of a request and the time steps it has run (all of them once done;
 * a failed request reports those it ran before it failed) */
bp_status bp_server_poll(const bp_server *s, int64_t ticket, int32_t *state, int32_t *steps_done);
/* Copy the fields of a finished request (eta 2 x N, p N, sigma 3 x N, any may
 * be NULL; fields at time nsteps dt, as bp_get_fields) and forget the ticket.
 * A failed request returns its error and is forgotten too. */
bp_status bp_server_result(bp_server *s, int64_t ticket, double *eta, double *p, double *sigma);
bp_status bp_server_stats(const bp_server *s, size_t *pool_bytes, size_t *free_bytes, int32_t *n_active,
                          int32_t *n_queued);
bp_status bp_server_destroy(bp_server *s);

/* Message of the last error on the calling thread ("" if none). */
const char *bp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BIOTLBM_H */
