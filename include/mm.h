/*
 * mm.h -- C ABI of the MI355X moving-mesh finite-volume step.
 *
 * The library computes one explicit step of the arbitrary Lagrangian-Eulerian
 * finite-volume scheme of Chang, Wadsley & Quinn (2017), "A moving mesh
 * hydrodynamic solver for ChaNGa", on one AMD Instinct MI355X (gfx950):
 *   periodic Voronoi tessellation of the mesh-generating points (Sec. 3),
 *   cell volumes, centroids, face areas and face centres,
 *   least-squares gradients with the S10 slope limiter (Sec. 4.1),
 *   the half-step predictor (Sec. 4.1),
 *   limited linear reconstruction to the face centres (Sec. 4.1),
 *   HLLC fluxes in the frame of each moving face (Sec. 4, items 1-5),
 *   the conserved-charge update (Sec. 4, update of the charges),
 *   mesh velocities and the CFL timestep (Sec. 4.2), and the drift.
 *
 * Conventions shared by every call:
 *   - Pointers named "dev" are device pointers on the context's device; the
 *     caller owns them and the library never frees them.  Pointers named
 *     "host" are host memory.
 *   - Per-point arrays are row-major, in the caller's point order:
 *     positions [n][3] (x, y, z), primitives [n][5] (rho, vx, vy, vz, P),
 *     charges Q [n][5] (mass, momentum x/y/z, total energy, i.e. the
 *     integral of (rho, rho v, rho e) over the cell, Sec. 4), conserved
 *     densities U [n][5] = Q / V, gradients [n][5][3] (d U_q / d x_a),
 *     mesh velocities [n][3].
 *   - U and gradients are double for MM_FP64 and float for MM_MIXED;
 *     positions, charges, mesh velocities and charge changes are always
 *     double.
 *   - All work is enqueued on the HIP stream given to mm_create, in order.
 *     Calls that report a status computed on the device (mm_tessellate,
 *     mm_cell_state, mm_step) wait for that stream once, at their end, to
 *     read a small status block; the others return without waiting.
 *   - The context owns every internal buffer, all reserved by mm_create for
 *     n_capacity points; no call after mm_create allocates device memory.
 *   - Errors are returned as mm_status codes; mm_last_error() gives a
 *     message.  No C++ exception crosses this interface.  A context is not
 *     thread-safe; use one context per host thread.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_ctx mm_ctx;

typedef enum {
  MM_OK = 0,
  MM_EINVAL = -1,       /* bad argument: null pointer, n > capacity, point outside [0, L) or not finite */
  MM_ENOMEM = -2,       /* device allocation failed in mm_create */
  MM_ECAPACITY = -3,    /* a fixed per-cell or per-mesh capacity was exceeded (see mm_last_error) */
  MM_EDEGENERATE = -4,  /* tessellation failed: incomplete cell, asymmetric faces or box too small */
  MM_ENONFINITE = -5,   /* a state became NaN or infinite */
  MM_EHIP = -6,         /* a HIP runtime call failed */
  MM_ESTATE = -7,       /* call out of order, e.g. mm_gradients before any mm_tessellate */
  MM_EFULL = -8         /* batch admission: not enough room now (retry after an eviction) */
} mm_status;

enum { MM_FP64 = 0, MM_MIXED = 1 };
/* Riemann solver of the face fluxes (Sec. 4 item 4): HLLC, the paper's
 * default, or the more diffusive HLL; both with Davis wave-speed bounds. */
enum { MM_HLLC = 0, MM_HLL = 1 };

/* Scheme parameters.  Defaults (mm_default_params): gamma = 5/3, cfl = 0.3,
 * eta = 1 (Lagrangian mesh, Sec. 4.2), chi = 1 and zeta = 0.25 (roundness
 * correction, Sec. 4.2), theta = 0.49 (Duffell-MacFadyen factor, Sec. 4.1
 * and Sec. 5.1; theta <= 0 switches it off), rho_floor = 1e-12,
 * p_floor = 1e-14 (floors, Sec. 4.1), limit_mask = 3. */
typedef struct {
  double box[3];             /* periodic box lengths L (Sec. 4.4: periodic boundaries) */
  double gamma;              /* ideal-gas adiabatic index */
  double cfl;                /* CFL coefficient of the per-cell timestep (Sec. 4.2) */
  double eta;                /* mesh velocity w = eta v + dw (Sec. 4.2) */
  double chi;                /* roundness correction speed in units of c_s (Sec. 4.2) */
  double zeta;               /* roundness correction distance in units of R (Sec. 4.2) */
  double theta;              /* Duffell-MacFadyen limiter parameter (Sec. 4.1) */
  double rho_floor;          /* density floor (Sec. 4.1) */
  double p_floor;            /* pressure floor (Sec. 4.1) */
  int32_t precision;         /* MM_FP64, or MM_MIXED: gradients, predictor, reconstruction and
                                Riemann solves in float; geometry and charge sums in double */
  int32_t riemann;           /* MM_HLLC or MM_HLL */
  int32_t limit_mask;        /* S10 limiter: bit 0 on the time-n gradient, bit 1 on the half-step one */
  int32_t predictor_frame;   /* 0: rate following the generator, -div F + w . grad U; 1: Eulerian -div F */
  int32_t half_step_mesh;    /* 1: the second gradient, the face states and the fluxes use a mesh rebuilt
                                at the half-step positions r + w dt/2 (the paper's first future
                                improvement, Sec. 6), at the cost of a second tessellation per step;
                                0 (default): the mesh of the start of the step, as in the paper's runs.
                                Single simulations only (mm_batch_admit rejects 1). */
  int32_t reserved;          /* must be 0 */
  double mach_threshold;     /* entropy switch (Sec. 4.3): a cell whose largest face shock Mach number
                                stays below it takes its pressure from the advected entropy (the paper
                                uses 1.1); 0 (default): the energy equation alone.  Above 0, steps go
                                through mm_step_entropy; single simulations only. */
} mm_params;

/* Per-step report, filled by mm_step (and partly by mm_tessellate). */
typedef struct {
  double dt;                 /* timestep used: min(dt_max, dt_cfl) */
  double dt_cfl;             /* CFL timestep min_i dt_i (Sec. 4.2) */
  int64_t n_faces;           /* unique faces of the tessellation */
  int32_t max_faces_cell;    /* largest number of faces of one cell */
  int32_t deferred_cells;    /* cells re-run with a wider neighbour stencil */
  int64_t floor_hits[4];     /* floors fired: [0] cell states at the start, [1] half-step states,
                                [2] face states, [3] charges after the update (Sec. 4.1) */
  int32_t flags;             /* internal failure bits (0 when the step succeeded) */
  int32_t rebuilt_cells;     /* cells the two-cells-per-wavefront first passes handed to the one-cell
                                first passes (too many candidates, faces or vertices for their slots,
                                a thin region, or more distance shells than they take) */
} mm_step_info;

/* Device views of the current tessellation, in the library's internal
 * (bucket-sorted) cell order.  Valid until the next mm_tessellate or
 * mm_step on the context; read-only for the caller. */
typedef struct {
  int64_t n;                 /* cells */
  int64_t n_faces;           /* unique faces */
  const int32_t *perm;       /* dev [n]: internal cell s holds caller point perm[s] */
  const double *pos;         /* dev [n][3]: generator positions, internal order */
  const double *geo;         /* dev [n][4]: volume V, then centroid minus generator (3) */
  const void *faces;         /* dev [n_faces] records of 48 bytes: int32 i, j (internal cells, i the
                                owner), int32 image code of j as (kx+1) + 3(ky+1) + 9(kz+1), int32 0,
                                double area A, double[3] face centroid minus r_i */
} mm_mesh_view;

/* Fills *p with the defaults listed above and box = (1, 1, 1). */
void mm_default_params(mm_params *p);

/* Creates a context on the current HIP device.  n_capacity bounds n in every
 * later call; face_capacity bounds the number of unique faces (0 selects
 * 12 n_capacity, enough for jittered lattices (about 8 per cell) and Poisson
 * points (about 7.8 per cell)).  hip_stream is a hipStream_t (NULL: the null
 * stream).  *out receives the context.  Errors: MM_EINVAL, MM_ENOMEM, MM_EHIP. */
mm_status mm_create(mm_ctx **out, const mm_params *p, int64_t n_capacity, int64_t face_capacity,
                    void *hip_stream);

/* Releases the context and all its device memory (after waiting for its stream). */
mm_status mm_destroy(mm_ctx *ctx);

/* Replaces the scheme parameters (box, gamma, ...).  precision may not change. */
mm_status mm_set_params(mm_ctx *ctx, const mm_params *p);

/* Periodic Voronoi tessellation of n generators (Sec. 3: each cell is cut
 * from the box around its generator by the bisector planes of the
 * neighbours, nearest first, until no farther neighbour can cut it).
 * pos: dev [n][3], each coordinate in [0, L).  Keeps the mesh in the
 * context for mm_mesh_view/mm_mesh_export/mm_init_charges/mm_cell_state/
 * mm_gradients/mm_predict/mm_fluxes.  info (host, may be NULL) receives
 * n_faces, max_faces_cell, deferred_cells and rebuilt_cells.  Waits for the stream.
 * Errors: MM_EINVAL (bad n or positions), MM_ECAPACITY, MM_EDEGENERATE. */
mm_status mm_tessellate(mm_ctx *ctx, int64_t n, const double *pos, mm_step_info *info);

/* Device views of the last tessellation (see mm_mesh_view). */
mm_status mm_get_mesh_view(const mm_ctx *ctx, mm_mesh_view *out);

/* Copies the last tessellation out in caller order (all dev, caller-owned):
 * V [n], centroid [n][3] (absolute), and the unique faces, each once:
 * face_i, face_j [face_cap] caller indices (face_i is the owner side),
 * face_code [face_cap] periodic image of j, face_A [face_cap],
 * face_f [face_cap][3] absolute face centroid r_i + (f - r_i), which may lie
 * outside the box.  *n_faces (host) receives the count; MM_ECAPACITY if it
 * exceeds face_cap (nothing is written then).  Any output may be NULL. */
mm_status mm_mesh_export(mm_ctx *ctx, double *V, double *centroid, int64_t face_cap, int32_t *face_i,
                         int32_t *face_j, int32_t *face_code, double *face_A, double *face_f,
                         int64_t *n_faces);

/* Charges from primitives after a tessellation (Sec. 4.3: the cell holds the
 * primitive state of its generator): Q_i = U(prim_i) V_i.
 * prim: dev [n][5] double, Q: dev [n][5] double. */
mm_status mm_init_charges(mm_ctx *ctx, const double *prim, double *Q);

/* Cell state at the start of a step (Sec. 4; Sec. 4.1 floors; Sec. 4.2):
 * U = Q/V with floors, mesh velocities w and dt_cfl = min_i dt_i.
 * Q: dev [n][5] double; U: dev [n][5] (precision type); w: dev [n][3]
 * double; dt_cfl, floor_hits: host (may be NULL).  Waits for the stream. */
mm_status mm_cell_state(mm_ctx *ctx, const double *Q, void *U, double *w, double *dt_cfl,
                        int64_t *floor_hits);

/* Least-squares gradients about the cell centroids, optionally S10-limited
 * (Sec. 4.1).  U: dev [n][5], grad: dev [n][5][3], both of the precision
 * type.  limit: 0 or 1. */
mm_status mm_gradients(mm_ctx *ctx, const void *U, void *grad, int32_t limit);

/* Half-step predictor (Sec. 4.1): U_half = U + dt/2 (-div F(U, grad U)
 * + w . grad U), then floors.  U, grad, U_half of the precision type,
 * w: dev [n][3] double. */
mm_status mm_predict(mm_ctx *ctx, const void *U, const void *grad, const double *w, double dt,
                     void *U_half);

/* Face fluxes and their sum per cell (Sec. 4, items 1-5 and the update of
 * the charges; Sec. 4.1 reconstruction): for each face, the face velocity,
 * limited reconstruction of U_half from both sides to the face centre,
 * face floors, HLLC in the face frame, boost back; then
 * dQ_i = - sum_faces dt A F (F from i toward its neighbour).
 * U_half [n][5], grad_half [n][5][3] of the precision type; w [n][3] and
 * dQ [n][5] double; all dev. */
mm_status mm_fluxes(mm_ctx *ctx, const void *U_half, const void *grad_half, const double *w, double dt,
                    double *dQ);

/* One whole step (Sec. 2 outline): tessellate pos, cell states, timestep
 * dt = min(dt_max, dt_cfl), gradient, predictor, half-step gradient, face
 * fluxes, update of Q with floors, drift pos += w dt with periodic wrap.
 * pos: dev [n][3] in/out; w: dev [n][3] out (the mesh velocities used);
 * Q: dev [n][5] in/out; info: host out (may be NULL).  Waits for the
 * stream once, at the end.  MM_EINVAL when p.mach_threshold > 0 (use
 * mm_step_entropy).
 * On any error pos and Q keep the values they had before the call (the
 * results are copied out only once the step is known to have succeeded),
 * so the caller can retry from them: after MM_ECAPACITY for the face
 * capacity (mm_last_error names it), with a context created with a larger
 * face_capacity; after MM_ENONFINITE (a start-of-step state that is not
 * finite, or a step that produced one), with a smaller dt_max or repaired
 * charges.  w may hold partial results after an error. */
mm_status mm_step(mm_ctx *ctx, int64_t n, double *pos, double *w, double *Q, double dt_max,
                  mm_step_info *info);

/* Entropy charges S_i = m_i P_i rho_i^-gamma (Sec. 4.3: the column rho s
 * with the entropic function A = P rho^-gamma as s) of primitive states on
 * the last tessellation.  prim: dev [n][5] as for mm_init_charges; S: dev
 * [n] out, caller order, caller-owned.  Errors: MM_EINVAL, MM_ESTATE. */
mm_status mm_init_entropy(mm_ctx *ctx, const double *prim, double *S);

/* One whole step with the entropy column (Sec. 4.3), otherwise as mm_step.
 * The state gains X = rho A, advected by the mass flux (reconstructed,
 * limited and predicted like the other columns); every face reports a
 * shock Mach number from its Riemann problem, and a cell whose largest one
 * is below p.mach_threshold takes its pressure from S / m, while the others
 * keep the energy and reset S from the new state.  S: dev [n] in/out
 * entropy charges (caller order); mach: dev [n] float out, each cell's
 * largest face Mach number (1 without compression), or NULL.  With
 * mach_threshold = 0 the charges Q are exactly those of mm_step.
 * Errors as mm_step (S, like pos and Q, keeps its values on an error), and
 * MM_EINVAL with half_step_mesh = 1. */
mm_status mm_step_entropy(mm_ctx *ctx, int64_t n, double *pos, double *w, double *Q, double *S, float *mach,
                          double dt_max, mm_step_info *info);

/* Largest n of mm_step_static. */
#define MM_STATIC_MAX_POINTS 8192

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): mm_step
 * without a context.  It runs the same kernels as mm_step with the context
 * of parameters p (a one-simulation context of MM_STATIC_MAX_POINTS points
 * and 12 faces per point) carved from a fixed device array of 64 MiB that
 * the library holds on each GPU it runs on until the process ends; the call
 * allocates no device or pinned memory and creates no events.  pos, w, Q,
 * dt_max and info as for mm_step (caller-owned device arrays, caller order;
 * on an error pos and Q keep their values); hip_stream is a hipStream_t
 * (NULL: the null stream) on the current device.  Every call on a device
 * shares that device's array and overwrites what the last call left there,
 * so calls that overlap on one device (from several host threads, or on
 * several streams without ordering between them) race and must be
 * serialised by the caller.  Waits for the stream once, at its end.
 * Errors: MM_EINVAL (n outside [1, MM_STATIC_MAX_POINTS], bad parameters,
 * half_step_mesh = 1 or mach_threshold > 0), then those of mm_step; the
 * message is mm_last_error(NULL) on the calling thread. */
mm_status mm_step_static(const mm_params *p, int64_t n, double *pos, double *w, double *Q, double dt_max,
                         mm_step_info *info, void *hip_stream);

/* Message for the last error on this context (static storage of the context);
 * with ctx NULL, of the last failed mm_create or mm_step_static on the
 * calling thread. */
const char *mm_last_error(const mm_ctx *ctx);

/* Library version string. */
const char *mm_version(void);

/* Stage timing of mm_step, for profiling.  When enabled, mm_step records HIP
 * events on the context stream around its stages: [0] sort, [1] cell
 * construction, [2] mesh assembly, [3] cell states, [4] gradient + predictor,
 * [5] half-step gradient, [6] face fluxes, [7] update + drift, [8] the
 * rebuild of the mesh at the half step (half_step_mesh = 1; else 0).
 * mm_get_stage_ms writes up to n_stages (at most 9) milliseconds of the last
 * step. */
mm_status mm_set_stage_timing(mm_ctx *ctx, int32_t enable);
mm_status mm_get_stage_ms(const mm_ctx *ctx, double *ms, int32_t n_stages);

/* ---------------------------------------------------------------------------
 * Batched serving.
 *
 * A batch keeps many independent simulations resident on the device, each
 * with its own periodic box, point count, parameters (precision excepted:
 * one per batch) and timestep, and advances all of them together: one
 * mm_batch_step runs every kernel of the step once, over the cells of all
 * resident simulations (the paper's step, Sec. 2 outline, per simulation).
 * Simulations are admitted while their device footprint fits the batch's
 * memory budget and leave when evicted, so new ones join between the steps
 * of those already in flight (continuous batching).  A simulation's results
 * are bitwise the same alone and in any mix: its cells keep their relative
 * order in every launch and no kernel combines data of two simulations.
 * Positions and charges of a resident simulation live in the batch;
 * mm_batch_read copies them out.  A batch is not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct mm_batch mm_batch;

/* Per-simulation report of one mm_batch_step. */
typedef struct {
  int32_t sim;               /* simulation id from mm_batch_admit */
  int32_t status;            /* MM_OK, or the error of this simulation's step (it is then parked:
                                no longer stepped, still resident until evicted) */
  int64_t steps;             /* steps completed so far */
  int64_t n;                 /* points */
  double dt;                 /* timestep of this step */
  double t;                  /* simulated time after the step */
  int64_t floor_hits[4];     /* as in mm_step_info */
  int32_t flags;             /* internal failure bits of this simulation */
  int32_t reserved;
} mm_sim_info;

/* Device bytes one simulation of n points takes in a batch of the given
 * precision (the unit of admission). */
int64_t mm_batch_footprint(int32_t precision, int64_t n);

/* Creates a batch on the current HIP device that reserves, once, the device
 * memory for hbm_budget bytes of simulations (mm_batch_footprint each) and at
 * most max_sims of them.  precision: MM_FP64 or MM_MIXED for every
 * simulation of the batch.  hip_stream: hipStream_t (NULL: null stream).
 * Errors: MM_EINVAL, MM_ENOMEM, MM_EHIP (message: mm_batch_last_error(NULL)). */
mm_status mm_batch_create(mm_batch **out, int32_t precision, int64_t hbm_budget, int32_t max_sims,
                          void *hip_stream);
mm_status mm_batch_destroy(mm_batch *b);

/* Admits a simulation of n points: p its parameters (p->precision must be
 * the batch's), pos [n][3] its generator positions in [0, L), prim [n][5]
 * its primitive state (rho, vx, vy, vz, P) at the generators, both in caller
 * order, in device or host memory (copied; the caller keeps ownership),
 * dt_max the cap of each of its timesteps.  Its charges are formed from the
 * first tessellation of its first step (Sec. 4.3).  *sim receives its id.
 * Errors: MM_EINVAL; MM_EFULL when its footprint, a slot range or a
 * simulation slot is not free now; MM_ECAPACITY when it could never fit. */
mm_status mm_batch_admit(mm_batch *b, const mm_params *p, int64_t n, const double *pos, const double *prim,
                         double dt_max, int32_t *sim);

/* One step of every resident simulation that has not failed, in one set of
 * launches.  info (host, may be NULL) receives up to info_cap reports, one
 * per simulation stepped, *n_info (may be NULL) their number.  Waits for
 * the stream once.  Returns MM_OK when the launches ran; errors of single
 * simulations are in their reports.  A simulation whose step fails keeps
 * its positions and charges as they were before the step (a newly admitted
 * one holds its first charges) and is parked; the others advance exactly
 * as they would without it.  MM_ECAPACITY if a batch-wide capacity was
 * exceeded (then no simulation advances and every stepped one reports it). */
mm_status mm_batch_step(mm_batch *b, mm_sim_info *info, int32_t info_cap, int32_t *n_info);

/* Copies a simulation's state out, in its caller order: pos [n][3],
 * Q [n][5] charges, w [n][3] mesh velocities of its last step; device or
 * host memory, any may be NULL.  Waits for the copies.  MM_ESTATE before
 * its first step. */
mm_status mm_batch_read(mm_batch *b, int32_t sim, double *pos, double *Q, double *w);

/* Removes a simulation and frees its room. */
mm_status mm_batch_evict(mm_batch *b, int32_t sim);

/* Occupancy: resident points and simulations, and the point capacity. */
mm_status mm_batch_usage(const mm_batch *b, int64_t *cells, int64_t *cell_capacity, int32_t *sims);

const char *mm_batch_last_error(const mm_batch *b);

/* A request of the serving loop. */
typedef struct {
  double arrival;            /* seconds after the start of mm_serve (non-decreasing over requests) */
  int64_t n;                 /* points */
  const double *pos;         /* [n][3] device or host, caller order */
  const double *prim;        /* [n][5] device or host */
  mm_params params;
  double dt_max;             /* cap of each timestep */
  int32_t steps;             /* steps to run */
  int32_t reserved;
  double *pos_out;           /* [n][3] device or host: positions after the last step (may be NULL) */
  double *Q_out;             /* [n][5] device or host: charges after the last step (may be NULL) */
} mm_request;

typedef struct {
  double admitted;           /* seconds after the start */
  double finished;
  int32_t status;            /* MM_OK, or the error that ended the request */
  int32_t steps;             /* steps completed */
  double t;                  /* simulated time reached */
} mm_request_result;

typedef struct {
  double wall;               /* seconds from the start to the last completion */
  int64_t batch_steps;       /* mm_batch_step calls */
  int64_t sim_steps;         /* simulation steps completed */
  int64_t cell_updates;      /* sum over simulation steps of their points */
  double cell_updates_per_s;
  double step_p50, step_p99, step_mean;   /* ms, over simulation steps: the duration of the batch
                                             step each took part in, readback included */
  double turnaround_p50, turnaround_p99;  /* s, over requests: finished - arrival */
  int32_t max_resident;      /* most simulations resident at once */
  int32_t reserved;
} mm_serve_stats;

/* Serving loop over a request trace on an empty batch: requests are
 * admitted first come, first served, as soon as they have arrived (wall
 * clock from the call) and fit; every resident simulation advances one step
 * per batch step; a simulation that completes its steps (or fails) is read
 * out to pos_out/Q_out and evicted, and its room goes to the next arrivals.
 * res [n_req] and stats (host) receive the outcome.  Returns MM_OK unless
 * the loop itself could not run. */
mm_status mm_serve(mm_batch *b, const mm_request *req, int32_t n_req, mm_request_result *res,
                   mm_serve_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
