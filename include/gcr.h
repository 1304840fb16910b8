/*
 * gcr.h -- C-ABI of the MI355X ghost-cell reconstruction library (libgcr.so).
 *
 * The library implements the direct, non-iterative ghost-cell method of
 * Rapaka, Jagad, Addad & Riahi ("Stable, Compact, and Direct Ghost-Cell
 * Reconstruction"): it tags ghost cells on a Cartesian grid cut by an
 * embedded body (classical CGC, extended-stencil CGC_ES and hybrid HGC;
 * Sec. 3.1 and Sec. 7), orders them by the levels of their dependency graph
 * (Sec. 3.2), fills them level by level with the analytical Dirichlet and
 * Neumann relations (Sec. 4 and Sec. 5), and evaluates boundary values,
 * gradients and forces from the same polynomials (Sec. 6).
 *
 * Conventions shared by every call
 *  - Cells are cell-centred: cell (i,j,k) has centre lo + (idx + 1/2) h per
 *    axis (midway between its faces on a stretched axis) and linear index
 *    i + n[0]*(j + n[1]*k) (x fastest).  A grid holds fewer than 2^31
 *    cells.
 *  - Fields are dense FP64 arrays in that layout, one device pointer per field.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are host memory owned by the caller.  The library keeps no
 *    reference to caller memory after a call returns.
 *  - `stream` is a hipStream_t (NULL: the null stream).  Every call that
 *    launches work is asynchronous on that stream, except gcr_plan_create
 *    and gcr_batch_create, which synchronise it twice (to size the band
 *    arrays, then to read the level offsets), and the first gcr_fill with
 *    the automatic schedule or gcr_batch_forward for a kind of plan, which
 *    times candidate schedules once and remembers the winner.
 *  - Every call returns GCR_OK or an error code; gcr_status_str() names it.
 *    Geometry and graph errors are detected when a plan is built; apply
 *    calls fail only on bad arguments or HIP errors.  On error nothing the
 *    caller owns has been modified, except by already-enqueued work of the
 *    same call for GCR_E_HIP.
 *  - Ghost-indexed arrays use the canonical order: level ascending, linear
 *    index ascending inside a level (Sec. 3.2: cells of one level are
 *    independent, so the order inside a level is free; this one is fixed).
 */
#ifndef GCR_H
#define GCR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GCR_OK = 0,
  GCR_E_ARG = 1,         /* invalid argument (null, size, range, dimension) */
  GCR_E_HIP = 2,         /* a HIP runtime call failed */
  GCR_E_NOMEM = 3,       /* device or host allocation failed */
  GCR_E_CYCLE = 4,       /* the ghost graph could not be layered (internal) */
  GCR_E_STENCIL = 5,     /* a stencil point leaves the grid or is a solid cell;
                            or a query point has no ghost within 2 cells */
  GCR_E_DEGENERATE = 6,  /* zero denominator in a relation */
  GCR_E_GEOMETRY = 7,    /* closest-point projection did not converge */
  GCR_E_UNSUPPORTED = 8, /* size or combination not supported */
  GCR_E_TIMEOUT = 9      /* a bounded wait between workgroups gave up: the
                            outputs of the call it belongs to are not valid */
} gcr_status;

/* Ghost placement (Sec. 3.1, Sec. 7.2). */
typedef enum { GCR_CGC = 0, GCR_CGC_ES = 1, GCR_HGC = 2 } gcr_scheme;
/* Flag or-ed into a scheme: a second ghost layer (Sec. 7.1).  Solid cells
 * with psi <= 1.5 delta n (Eq. delta_n) that the scheme does not already
 * make ghosts join the ghost set; they are reconstructed on the extended
 * stencil of Eq. stencil_anisotropic, the scheme's own ghosts as before. */
#define GCR_LAYER2 4

/* Boundary-condition kind per field (Sec. 4.1, 5.1).  GCR_MIXED: a per-ghost
 * uint8 array (0 Dirichlet, 1 Neumann) is supplied. */
typedef enum { GCR_DIRICHLET = 0, GCR_NEUMANN = 1, GCR_MIXED = 2 } gcr_bc;

/* Body kinds. */
typedef enum {
  GCR_SPHERE = 0,   /* circle (2D) or sphere (3D), radius r0 about center */
  GCR_STAR2D = 1,   /* r(t) = r0 (1 + sum_k A_k cos kt + B_k sin kt);
                       coef = {A_0,B_0,A_1,B_1,...}, ncoef = number of k     */
  GCR_SHSTAR = 2,   /* r(w) = r0 (1 + sum_lm a_lm Y_lm(w)), real Schmidt
                       semi-normalised harmonics, no Condon-Shortley phase;
                       coef[l*l + l + m], ncoef = (L+1)^2, L <= 8            */
  GCR_AIRFOIL = 3   /* symmetric four-digit section: thickness ratio
                       `thickness`, chord `chord`, leading edge at center,
                       nose-up incidence `incidence` (radians), closed
                       trailing edge                                         */
} gcr_shape_kind;

typedef struct {
  int32_t dim;     /* 2 or 3 */
  int32_t pad;
  int64_t n[3];    /* cells per axis (n[2] ignored in 2D) */
  double lo[3];    /* lower corner */
  double h[3];     /* uniform spacing per axis, > 0 */
  /* Stretched axes (the flows of Secs. 8.1-8.2 run on grids stretched toward
   * the outer boundaries; Sec. 7.1 takes the local spacing per direction):
   * faces[a], if not NULL, holds host double [n[a] + 1] cell faces of axis
   * a, strictly increasing (copied by the library; lo[a], h[a] then
   * unused).  Cell centres lie midway between faces; Eq. delta_n and Eq.
   * stencil_anisotropic take the local cell widths; a stencil's x_2 - x_1
   * is the difference of the two cell centres.  With GCR_LAYER2,
   * (1.5 + sqrt(dim)/2) times the largest cell width over the smallest
   * width along any axis must stay below 63 (else GCR_E_UNSUPPORTED). */
  const double* faces[3];
} gcr_grid;

typedef struct {
  int32_t kind;            /* gcr_shape_kind */
  int32_t ncoef;
  double center[3];
  double r0;
  const double* coef;      /* host; copied by the library */
  double chord, thickness, incidence;
} gcr_shape;

typedef struct gcr_plan gcr_plan;
typedef struct gcr_batch gcr_batch;

typedef struct {
  int32_t dim;
  int32_t n_levels;            /* depth of the (condensed) dependency graph */
  int64_t n_cells;
  int64_t n_interface;         /* cells with a face neighbour of the other class */
  int64_t n_ghost;
  int64_t n_ghost_fluid_side;  /* HGC ghosts with fluid centres (tag -2) */
  int32_t n_units_coupled;     /* strongly connected groups of >1 ghost */
  int32_t max_unit;            /* their largest size (0 if none) */
  int32_t max_level_width;     /* largest level */
  int32_t schedule;            /* fill schedule in use, see gcr_set_schedule */
  double max_alpha[3];         /* max (x_s - x_1)/(x_2 - x_1) per axis (Sec. 8) */
  int64_t n_band_segments;     /* 16-cell row segments whose classification needed
                                  the exact test of every cell (near the body), in
                                  the build that made the plan (a batch: all of its
                                  instances) */
} gcr_stats;

/* Builds the plan of one grid + body + scheme: classification (Sec. 3.1,
 * cell centres, psi >= 0 solid), ghost tags, foot points S = x_c + psi n with
 * the analytic outward normal at the closest boundary point, stencil
 * multipliers (Eq. stencil_anisotropic for CGC_ES), the ghost dependency
 * graph and its Kahn levels (Sec. 3.2).  Where the graph is not acyclic
 * (concave bodies), each strongly connected group of ghosts forms one unit
 * whose relations are solved together.  The library solves units of up to
 * 8 ghosts (at most 1024 units and 1024 ghosts in cycles per instance) and
 * reports larger ones as GCR_E_UNSUPPORTED, a capacity limit.  grid,
 * shape: host.  Synchronises `stream` twice.  The plan owns all its device
 * memory; *out is NULL on error. */
gcr_status gcr_plan_create(const gcr_grid* grid, const gcr_shape* shape,
                           int32_t scheme, void* stream, gcr_plan** out);
/* (scheme: a gcr_scheme, optionally | GCR_LAYER2; gcr_stats.n_interface
 * then still counts interface cells only.) */
void gcr_plan_destroy(gcr_plan* plan);

/* Re-plan after the body moved (Sec. 7.1: a moving boundary; the plan of
 * Secs. 3.1-3.2 at the new position).  plan: made by gcr_plan_create (a
 * plan of a batch: GCR_E_UNSUPPORTED); shape: the body at its new position
 * or of a new form, any kind valid on the plan's grid; grid, scheme and
 * second layer stay.  The result equals gcr_plan_create with the same grid,
 * shape and scheme, array for array.  The plan's tag array is updated in
 * place: a chunk of 4096 cells is classified again only when one of its
 * 1024-cell spans was not settled on one side of the old boundary, is not
 * settled on one side of the new one, or changed side, or when it holds a
 * ghost of the old plan; every other chunk keeps its tags (its cells and
 * their face neighbours lie on the same side of both boundaries).  Ghosts,
 * dependencies, levels, units and the lookup tables are rebuilt from the
 * new tags; caches of the old plan (ghost weights, adjoint stencils, tuned
 * schedule) are dropped.  Synchronises `stream` twice, as gcr_plan_create;
 * work on other streams that reads the plan must be complete.  For the
 * fresh cells of a move keep the plan of the previous position alive: two
 * plans updated in turn, each from two positions back, give
 * gcr_plan_fresh_cells(previous, updated).  On error the plan is as it was
 * before the call (rebuilt at the old position if the update had begun),
 * except if that rebuild fails too (GCR_E_NOMEM): then every call on it
 * but gcr_plan_destroy returns GCR_E_ARG. */
gcr_status gcr_plan_update(gcr_plan* plan, const gcr_shape* shape, void* stream);

/* Host copy of the plan's sizes and statistics. */
gcr_status gcr_plan_stats(const gcr_plan* plan, gcr_stats* out);

/* Level offsets into the canonical ghost order, host array [n_levels + 1]. */
gcr_status gcr_plan_level_offsets(const gcr_plan* plan, int32_t* out);

/* Device copies of the plan (any pointer may be NULL):
 *   tags     int8  [n_cells]  0 fluid, 1 solid, +2 / -2 ghost (Sec. 3.1)
 *   cell     int32 [n_ghost]  linear index of each ghost
 *   level    int32 [n_ghost]  1-based level
 *   delta    f64 [dim][n_ghost] x_s - x_c
 *   normal   f64 [dim][n_ghost] unit normal into the fluid at S
 *   psi      f64 [n_ghost]    signed distance (Eq. signed_distance)
 *   r        int32 [dim][n_ghost] stencil multipliers
 *   unit     int32 [n_ghost]  canonical position of the unit's first ghost,
 *                             or -1 for a ghost that is its own unit */
gcr_status gcr_plan_export(const gcr_plan* plan, int8_t* tags, int32_t* cell,
                           int32_t* level, double* delta, double* normal,
                           double* psi, int32_t* r, int32_t* unit, void* stream);

/* Where the caller evaluates boundary data (Sec. 3: the Dirichlet value or
 * normal derivative is prescribed at the foot point S of each ghost):
 *   S        device f64 [dim][n_ghost]  S = x_c + delta, canonical order
 *   normal   device f64 [dim][n_ghost]  unit normal into the fluid at S
 * Either may be NULL.  One kernel on `stream`. */
gcr_status gcr_plan_foot_points(const gcr_plan* plan, double* S, double* normal,
                                void* stream);

/* Fresh cells of a moved body (Sec. 7.1: a moving boundary exposes fresh
 * fluid cells, one reason for a second ghost layer).  before, after: plans
 * of the body before and after a move, on the same grid (same sizes, origin
 * and spacing; a stretched grid's faces must be the same too, which is not
 * checked).  A cell is fresh when its centre was solid before (tag 1 or 2)
 * and is fluid after (tag 0 or -2); it is uncovered when it was not a
 * ghost before (tag 1), so no value was reconstructed there.
 *   counts  device int64 [2]: fresh cells, uncovered fresh cells
 *   list    device int32 [cap] or NULL: the fresh cells' linear indices,
 *           ascending, the first cap of them
 * Stream-ordered, no host synchronisation; uses scratch held by `after`.
 * GCR_E_ARG if the grids differ. */
gcr_status gcr_plan_fresh_cells(const gcr_plan* before, const gcr_plan* after,
                                int64_t* counts, int32_t* list, int64_t cap,
                                void* stream);

/* Fill schedule.  0 = automatic (tuned), 1 = one launch per level,
 * 2 = one workgroup sweeping all levels, 3 = per-level launches captured in a
 * HIP graph and replayed.  `param` is reserved (0). */
gcr_status gcr_set_schedule(gcr_plan* plan, int32_t schedule, int32_t param);

/* Level-by-level ghost fill (Sec. 3.2 with Eqs. phi_G_Dir_2d, phi_G_Neu_2d,
 * phi_G_Dir_3d, phi_G_Neu_3d).  nf fields, 1 <= nf <= 8:
 *   fields   host array [nf] of device f64 [n_cells], in/out: ghost slots are
 *            overwritten; every other cell is read only.
 *   bc_kind  host int32 [nf]: gcr_bc per field.
 *   bc_type  host array [nf] of device uint8 [n_ghost] (0/1), read only for
 *            fields with GCR_MIXED; may be NULL if no field is mixed.
 *   bc_val   host array [nf] of device f64 [n_ghost]: phi at S (Dirichlet) or
 *            dphi/dn at S (Neumann), canonical ghost order.
 * A plan with no ghosts reads no boundary data: its bc_val and bc_type
 * entries may be NULL.  Otherwise a NULL field, bc_val, or bc_type of a
 * GCR_MIXED field, is GCR_E_ARG. */
gcr_status gcr_fill(const gcr_plan* plan, int32_t nf, double* const* fields,
                    const int32_t* bc_kind, const uint8_t* const* bc_type,
                    const double* const* bc_val, void* stream);

/* Value and Cartesian gradient of each ghost's reconstruction polynomial at
 * its foot point S (Sec. 6; Eqs. derivative_bilinear, derivative_trilinear_*).
 *   fields   host array [nf] of device f64 [n_cells] (filled)
 *   val      device f64 [nf][n_ghost]         (may be NULL)
 *   grad     device f64 [nf][dim][n_ghost]    (may be NULL) */
gcr_status gcr_surface_ghost(const gcr_plan* plan, int32_t nf,
                             const double* const* fields, double* val,
                             double* grad, void* stream);

/* The same at caller points xq (device f64 [dim][nq]): each point is served
 * by its anchor ghost, the ghost within 2 cells per axis of the point's cell
 * whose S is nearest (ties: smaller linear index).
 *   val [nf][nq], grad [nf][dim][nq], anchor int32 [nq] (canonical position);
 *   any output may be NULL.  GCR_E_STENCIL is not reported for points
 *   without an anchor: their outputs are NaN and anchor -1. */
gcr_status gcr_surface(const gcr_plan* plan, int64_t nq, const double* xq,
                       int32_t nf, const double* const* fields, double* val,
                       double* grad, int32_t* anchor, void* stream);

/* Force on the body, F = sum_q w_q (-p n_q + mu (grad u + grad u^T) n_q)
 * (Sec. 6: pressure and wall stress from the boundary values and gradients).
 *   xq, nrm  device f64 [dim][nq]: points and outward unit normals
 *   wq       device f64 [nq]: quadrature weights
 *   p        device f64 [n_cells] (filled); u: host array [dim] of device
 *            f64 [n_cells] (filled velocity components)
 *   F        device f64 [dim].  Deterministic (fixed reduction order). */
gcr_status gcr_forces(const gcr_plan* plan, int64_t nq, const double* xq,
                      const double* nrm, const double* wq, const double* p,
                      const double* const* u, double mu, double* F,
                      void* stream);

/* gcr_forces for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The
 * same computation and result, bit for bit, as gcr_forces; the per-block
 * partial sums live in a static device array of the library (1.5 MiB per
 * device, 65,536 blocks: up to 262,144 points in 3D and 524,288 in 2D; more
 * gives GCR_E_UNSUPPORTED) instead of scratch the plan allocates on first
 * use, and the call allocates nothing.  Every call on one device shares that
 * device's array, so calls that overlap on one device (concurrent streams or
 * host threads) race: the caller must order them. */
gcr_status gcr_forces_noalloc(const gcr_plan* plan, int64_t nq, const double* xq,
                              const double* nrm, const double* wq, const double* p,
                              const double* const* u, double mu, double* F,
                              void* stream);

/* Adjoint of gcr_surface: lam[f] (device f64 [n_cells]) += (d outputs /
 * d filled field)^T (gval [nf][nq], ggrad [nf][dim][nq]; either may be NULL).
 * Deterministic. */
gcr_status gcr_surface_adjoint(const gcr_plan* plan, int64_t nq,
                               const double* xq, int32_t nf,
                               const double* gval, const double* ggrad,
                               double* const* lam, void* stream);

/* Adjoint of gcr_forces for the functional J = gF . F (gF device f64 [dim]):
 * lam_p += dJ/dp, lam_u[i] += dJ/du_i (device f64 [n_cells] each). */
gcr_status gcr_forces_adjoint(const gcr_plan* plan, int64_t nq,
                              const double* xq, const double* nrm,
                              const double* wq, double mu, const double* gF,
                              double* lam_p, double* const* lam_u,
                              void* stream);

/* Adjoint of gcr_fill: the levels in reverse.  lam[f] (device f64 [n_cells])
 * holds dJ/d(filled field) on entry and dJ/d(input field) on return (zero in
 * ghost slots, whose inputs the fill overwrites); lam_bc[f] (device f64
 * [n_ghost]) receives dJ/d(bc_val).  bc_kind / bc_type as in gcr_fill.
 * Deterministic: every cell is written by one thread, sums in fixed order. */
gcr_status gcr_fill_adjoint(const gcr_plan* plan, int32_t nf,
                            double* const* lam, const int32_t* bc_kind,
                            const uint8_t* const* bc_type,
                            double* const* lam_bc, void* stream);

/* Batched plans: ninst instances of uneven size built by shared launches.
 * grids, shapes, schemes: host arrays [ninst].  Synchronises twice. */
gcr_status gcr_batch_create(int32_t ninst, const gcr_grid* grids,
                            const gcr_shape* shapes, const int32_t* schemes,
                            void* stream, gcr_batch** out);
/* Waits for the batch's gcr_batch_forward launches (on whatever stream) and
 * releases its memory; other work on its plans must have finished.
 * Forward calls on one batch may use different streams: each waits for the
 * previous one's launches (they share the batch's scratch state), so one
 * batch's forwards never overlap; calls from several host threads on one
 * batch must be serialised by the caller. */
void gcr_batch_destroy(gcr_batch* batch);
/* Plan of instance i, owned by the batch (valid until gcr_batch_destroy). */
gcr_status gcr_batch_plan(const gcr_batch* batch, int32_t i,
                          const gcr_plan** out);
/* Sizes of every instance's plan at once (host copies, no synchronisation):
 * n_ghost host int64 [ninst] ghosts, n_levels host int32 [ninst] levels of
 * the dependency graph (Sec. 3.2); either may be NULL. */
gcr_status gcr_batch_counts(const gcr_batch* batch, int64_t* n_ghost,
                            int32_t* n_levels);

/* Foot points and normals of every ghost of a batch in one launch, as
 * gcr_plan_foot_points gives them per plan (S = x_c + delta, Sec. 3.1),
 * with the instances' ghosts one after another: columns g_0 .. g_0 + n_0 - 1
 * are instance 0's in its plan's order, then instance 1's, and so on.
 *   S, normal  device f64 [dim][n_total], n_total the sum of the plans'
 *              n_ghost; either may be NULL.
 * Every instance must have the same dimension (else GCR_E_UNSUPPORTED).
 * One kernel on `stream`. */
gcr_status gcr_batch_foot_points(const gcr_batch* batch, double* S, double* normal,
                                 void* stream);

/* Batched forward in one persistent launch: for every instance, fill its nf
 * fields, then (if nq != NULL) the force on its body from field p_field
 * (pressure) and the dim fields u_first.. (velocity).  Host arrays of device
 * pointers are instance-major, [ninst * nf]:
 *   fields, bc_val, bc_type (bc_type may be NULL);  bc_kind host [nf].
 *   An instance whose plan has no ghosts reads no boundary data: its
 *   bc_val (and bc_type) entries may be NULL; every other NULL entry of
 *   fields, bc_val, or bc_type where its field's kind is GCR_MIXED, is
 *   GCR_E_ARG.
 *   nq host int64 [ninst]; xq, nrm, wq host [ninst] device pointers;
 *   F device f64 [ninst][3] (unused components zero).
 * Surface values (Sec. 6) of the filled fields at the same points, as
 * gcr_surface gives them (NaN at a point with no ghost within two cells):
 *   sval, sgrad  host [ninst * nf] of device pointers, or NULL (none), an
 *                entry NULL for a field not wanted: value f64 [nq_i] and
 *                gradient f64 [dim][nq_i] of field f of instance i.
 *   Either needs nq (else GCR_E_ARG). */
gcr_status gcr_batch_forward(gcr_batch* batch, int32_t nf,
                             double* const* fields, const int32_t* bc_kind,
                             const uint8_t* const* bc_type,
                             const double* const* bc_val, const int64_t* nq,
                             const double* const* xq, const double* const* nrm,
                             const double* const* wq, int32_t p_field,
                             int32_t u_first, double mu, double* F,
                             double* const* sval, double* const* sgrad,
                             void* stream);

/* Timing, process-wide.  mask: bit 0 (GCR_PROFILE_BUILD) stage timing of
 * plan building, bit 1 (GCR_PROFILE_FORWARD) timing of the batched forward;
 * 0 turns both off (the default: no events recorded); other bits:
 * GCR_E_ARG.  With bit 0 set, gcr_plan_create
 * and gcr_batch_create record HIP events on their stream around each stage;
 * gcr_last_build_times copies the device times in milliseconds of the last
 * build on the calling thread into ms[13]: [0] classification, [1] interface
 * scan, [2] interface compaction, [3] geometry and ghost tags, [4] ghost
 * compaction, [5] stencils and dependencies, [6] levels and canonical order,
 * [7] finalize; [8], [9], [10] split [0] into the span pass, the store pass
 * and the interface marks; [11] the stream's wait for the host between the
 * two halves of the build (the first synchronisation and the sizing of the
 * ghost arrays); [12] the host time of the whole call (both
 * synchronisations included). */
#define GCR_PROFILE_BUILD 1
#define GCR_PROFILE_FORWARD 2
gcr_status gcr_set_profiling(int32_t mask);
gcr_status gcr_last_build_times(float* ms);
/* With bit 1 set, each gcr_batch_forward records HIP events around
 * its two kernels (the surface-point anchor search and the persistent fill
 * + force launch).  This call waits for the recorded work, writes the mean
 * ms of each over the calls since the last query to out[0] and out[1] and
 * their number to out[2] (-1, -1, 0 if none), and clears the record. */
gcr_status gcr_forward_times(float* out);

/* Tiled batched fill (process-wide).  Tiled, gcr_batch_forward fills the
 * levels (Sec. 3.2) tile by tile: each instance's ghosts are grouped by the
 * tile of cells holding them, each tile's workgroup fills the tile's ghosts
 * and every ghost they depend on, transitively, in LDS, and writes its own;
 * the values are those of the level-by-level sweep, bit for bit.  Finding
 * the tiles' closures costs about as much as one sweep, so:
 *   mode 0  always the level-by-level sweep;
 *   mode 1  tiles from a batch's second forward call on (the default: a
 *           batch forwarded once never pays for them);
 *   mode 2  tiles from the first call.
 * Batches with coupled units, graphs deeper than 128 levels or an instance
 * of more than about 980,000 ghosts, and any batch whose tile closures would
 * not fit, take the sweep.  Applies to batches not yet set up. */
gcr_status gcr_set_batch_tiling(int32_t mode);
/* Which fill a batch's forward calls use: *state = -1 the level-by-level
 * sweep, 0 not decided yet (no forward call so far), 1 the tiled fill,
 * 2 the sweep after the tile closures did not fit.  Synchronises the
 * device (a diagnostic, not for the hot path). */
gcr_status gcr_batch_tiled(const gcr_batch* batch, int32_t* state);

/* The launch shape a batch's forward calls use (see gcr_set_batch_shape):
 * *threads per workgroup and *grid, > 0 one workgroup per (instance, field)
 * item times grid (k_batch_forward), < 0 the split sweep with -grid
 * workgroups per instance (k_batch_split); both 0 before the first forward
 * call.  Host only, no synchronisation. */
gcr_status gcr_batch_shape(const gcr_batch* batch, int32_t* threads, int32_t* grid);

/* Launch shape of the batched forward's level sweep (Sec. 3.2 fill, one
 * level after another).  By default it is picked by timing candidates on the
 * first call for a kind of batch and kept for the process: per-item
 * workgroups (one (instance, field) pair each, sweeping all its levels), or
 * a split sweep in which `-grid` workgroups per instance share each level
 * and meet at a device-scope counter between levels.  Both give the same
 * field values bit for bit; the force is the same bit for bit at the same
 * `threads`.  threads = 0 and grid = 0 restore the tuned choice; otherwise
 * threads is a power of two from 64 to 1024 and grid is 1..4 (per-item
 * kernel on min(items, 256 grid) workgroups) or -1..-128 (split sweep; a
 * batch with instances x -grid above 256 then fails with GCR_E_ARG, and one
 * whose workgroups cannot all be resident at once with GCR_E_UNSUPPORTED:
 * the split sweep is a cooperative launch).
 * Process-wide; for tests and measurements. */
gcr_status gcr_set_batch_shape(int32_t threads, int32_t grid);

/* Faults of the split sweep.  Its workgroups meet after every level (Sec.
 * 3.2: a level reads only earlier levels) at a device-scope counter; each
 * wait is bounded, and a wait that gives up (which co-residency of the
 * cooperative launch should prevent) sets a fault word of the batch, since
 * that call's fields, surface values and forces can then be wrong.
 * gcr_batch_status waits for the batch's gcr_batch_forward launches and
 * returns GCR_E_TIMEOUT if any of them gave up since the last query
 * (clearing the word), GCR_OK otherwise; it must not run concurrently with
 * forward calls on the same batch.  gcr_set_batch_spin sets the polls of a
 * wait before it gives up, process-wide (0: the default, 4M polls of about
 * 64 cycles); tests set 1 to make waits give up while every kernel still
 * ends. */
gcr_status gcr_batch_status(const gcr_batch* batch);
gcr_status gcr_set_batch_spin(int32_t polls);
/* Layering (Sec. 3.2).  At the default setting every instance is first
 * layered by one workgroup holding its counters and levels in LDS (up to
 * about 47,000 ghosts); a plan built alone that does not fit there and has
 * at least 65,536 interface cells is layered by the whole GPU (one
 * grid-wide round per level, then a stable counting sort by level); the
 * rest by one workgroup with its state in HBM.  A threshold set here
 * (`min_interface` > 0) sends every plan built alone with at least that
 * many interface cells to the whole GPU first, fitting LDS or not (for
 * tests and measurements).  A cycle or a graph deeper than 126 levels
 * hands an instance from the whole-GPU layering to the one-workgroup one,
 * so the result never depends on this setting.  0 restores the default.
 * Process-wide; applies to plans built afterwards. */
gcr_status gcr_set_wide_layering(int64_t min_interface);

/* The whole-GPU layering collects each round's newly placed ghosts in a
 * per-workgroup LDS buffer of `entries` slots (1..4096, default 4096; 0
 * restores it) and appends the overflow straight to the level's list.  The
 * result does not depend on it; a small buffer exercises the overflow (for
 * tests).  Else GCR_E_ARG.  Process-wide; applies to plans built
 * afterwards. */
gcr_status gcr_set_wide_buffer(int32_t entries);

/* When the Kahn layering of an instance stalls (its remaining ghosts read a
 * cycle), a remainder of at most `max_ghosts` ghosts is resolved by one
 * wave (closure by repeated squaring in registers, no workgroup barrier),
 * a larger one by the workgroup (trimming, closure, placement rounds).
 * Both give the same levels and units.  0..64, default 64 (0: always the
 * workgroup); else GCR_E_ARG.  Process-wide; applies to plans built
 * afterwards. */
gcr_status gcr_set_wave_residual(int32_t max_ghosts);

const char* gcr_status_str(gcr_status s);
const char* gcr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GCR_H */
