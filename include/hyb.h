/*
 * hyb.h -- C ABI of the MI355X domain-decomposition FEM/FDM wave solver
 * (L. Beilina, "Domain decomposition finite element/finite difference method
 * for the conductivity reconstruction in a hyperbolic equation",
 * arXiv 1509.01399).
 *
 * One context (hyb_ctx) owns all device state of one problem on one GPU:
 * the wavefields of the structured outer grid (finite differences) and of
 * the inner tetrahedral box (finite elements), the forward history or
 * checkpoints needed by the adjoint, the FP64 gradient accumulator and the
 * conjugate-gradient direction.  Every compute step runs in hand-written HIP
 * kernels for gfx950 on the context's stream.
 *
 * Conventions used by every call
 *  - Grid: n_cells[d] cells of size h per axis, (n_cells[d]+1) nodes, x
 *    fastest.  Faces are ordered x-, x+, y-, y+, z-, z+.  The backscattered
 *    trace (S_T of Sec. 5) is recorded on the z+ face, which is also the
 *    only face that may carry the plane-wave source.
 *  - FEM box: a tetrahedral mesh of a box of whole grid cells [o, o+C]
 *    (its bounding box: cubic, >= 5 cells wide, >= 1 cell to the outer
 *    boundary).  Two kinds (Sec. 1, Sec. 3, Sec. 7.2):
 *    structured: the split of every cube into the 6 tetrahedra sharing the
 *      cube diagonal; the P1 stiffness is then an edge-conductance stencil
 *      and the FEM rows run in grid-shaped tiles;
 *    general: any conforming mesh whose box surface carries exactly the grid
 *      nodes of the surface and in which every grid node of the inner box
 *      surface [o+2, o+C-2] is a mesh node (the overlap exchanges of
 *      Algorithm 1 need both); nodes elsewhere may lie anywhere.  The FEM
 *      rows then run on a sparse table of the assembled stiffness.
 *    A 6-tetrahedra split is treated as structured unless opts.fem_general
 *    asks for the general path.
 *  - Conductivity: a = 1 + sigma, sigma piecewise constant (a subspace of
 *    C_h, eq. (p0)), FP64.  Structured: one value per FEM cube, laid out
 *    [C_z][C_y][C_x] (x fastest); cubes within two cells of the FEM
 *    boundary are the overlap layer where a = 1 (condition (2.3)).  General:
 *    one value per tetrahedron in the mesh's order; a tetrahedron is free
 *    when all its vertices lie in the closed inner box [o+2, o+C-2]^3, and
 *    a = 1 on the others.  sigma outside the free cells is ignored and their
 *    gradient is 0.  Admissible values 0 <= sigma <= 4 (eq. (admpar)).
 *    hyb_fem_info gives the number of values.
 *  - Traces: obs / residual / data are FP64 device arrays
 *    [nt+1][(n_x+1)(n_y+1)] (level k = time k*dt; level 0 included).
 *  - Pointers named *_dev are device pointers owned by the caller; they must
 *    stay valid until the call's work has completed on the stream.  Pointers
 *    named *_host are host pointers.  Mesh arrays are host pointers that are
 *    copied during hyb_create.
 *  - Asynchrony: calls enqueue work on opts.hip_stream and return.  Calls
 *    that return a host scalar (J, gnorm) synchronise that stream.
 *  - Errors: argument, mesh and state errors are detected on the host before
 *    any work is enqueued and leave the context unchanged.  The CFL and
 *    non-finite sigma checks of a forward sweep run after the conductivity
 *    is loaded on the device: when they refuse, the previous sweeps of the
 *    context are no longer available (HYB_E_STATE until the next forward).
 *    Device errors are reported as HYB_E_DEVICE by the call that observes
 *    them.  hyb_last_error returns a text description of the last error.
 */
#ifndef HYB_H
#define HYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hyb_ctx hyb_ctx;

typedef enum {
    HYB_OK = 0,
    HYB_E_ARG = -1,          /* invalid argument (null, size, range)           */
    HYB_E_MESH = -2,         /* FEM mesh does not conform to the grid          */
    HYB_E_CFL = -3,          /* dt above the CFL bound tau <= h / sqrt(3 a)    */
    HYB_E_STATE = -4,        /* call out of order (e.g. adjoint before forward)*/
    HYB_E_OOM = -5,          /* device allocation failed                       */
    HYB_E_DEVICE = -6,       /* HIP runtime error                              */
    HYB_E_NONFINITE = -7,    /* NaN/Inf in an input                            */
    HYB_E_UNSUPPORTED = -8   /* valid but not supported by this build          */
} hyb_status;

/* Face conditions of the outer boundary.
 * ABC: first-order absorbing condition d_n u = -d_t u, discretised as in
 *      eq. (eq:abs2) (Sec. 7.4).
 * NEUMANN: d_n u = 0 (the lateral faces S_3 of Model Problems 1-2, Sec. 5).
 * SOURCE: z+ only; d_n u = p(t) while the pulse is on (S_{1,1}), absorbing
 *      afterwards (S_{1,2}), Model Problem 2 eq. (model2). */
typedef enum { HYB_BC_ABC = 0, HYB_BC_NEUMANN = 1, HYB_BC_SOURCE = 2 } hyb_bc;

typedef struct {
    int32_t n_cells[3];   /* cells per axis (>= 2)                                  */
    double h;             /* cell size, equal on all axes (> 0)                     */
    double origin[3];     /* coordinates of grid node (0,0,0)                       */
    int32_t face[6];      /* hyb_bc per face x-,x+,y-,y+,z-,z+                      */
} hyb_fd_grid;

typedef struct {
    int64_t n_nodes;      /* nodes; (C_x+1)(C_y+1)(C_z+1) for the structured split  */
    const double *xyz;    /* host [n_nodes][3] node coordinates                     */
    int64_t n_tets;       /* tetrahedra; 6 C_x C_y C_z for the structured split     */
    const int32_t *tet4;  /* host [n_tets][4] node ids (0-based, either orientation)*/
} hyb_fem_mesh;

typedef struct {
    int32_t width_cells;  /* overlap thickness; the method uses 2 (Sec. 3)          */
} hyb_overlap;

typedef struct {
    int32_t field_f32;    /* 0: FP64 wavefields; 1: FP32 wavefields (the gradient
                             integral, CG reductions and sigma stay FP64)           */
    int32_t store_mode;   /* forward states kept for the adjoint:
                             0: FEM-box history of every level;
                             1: sqrt(nt) checkpoints of the full state (field
                                precision) with segment recompute;
                             2: as 1, checkpoint increments in BF16;
                             3: as 1, checkpoint increments in 16-bit integers
                                with one FP32 scale per 64 values (kept to
                                1/65534 of each group's largest value).
                             2 and 3 need field_f32 = 1 (HYB_E_UNSUPPORTED) */
    double gamma;         /* Tikhonov regularisation parameter (eq. (functional))*/
    double alpha_rel;     /* CG: first trial step alpha_rel / max|d^m|          */
    void *hip_stream;     /* hipStream_t for all work; NULL = default stream      */
    int32_t fem_general;  /* 1: run a 6-tetrahedra split on the general path too
                             (one sigma per tetrahedron)                         */
    int32_t cg_max_trials;/* CG: trial steps per iteration (0: 8)               */
} hyb_opts;

typedef struct {
    int32_t kind;         /* 0: plane wave p(t) = sin(omega t) for
                                t < 2 pi / omega, then 0 (eq. (f));
                             1: flux table                                       */
    double omega;         /* kind 0: angular frequency (> 0)                     */
    const double *flux_dev; /* kind 1: device [nt][(n_x+1)(n_y+1)] flux d_n u   */
    int32_t k_on;         /* kind 1: steps k < k_on use the flux; afterwards the
                             z+ face is absorbing                                */
} hyb_source;

typedef struct {
    int32_t iter;         /* CG iterations done (0 before the first); set to 0 to
                             start a new run (beta^0 = 0)                        */
    double gnorm2_prev;   /* |g^{m-1}|^2_{L2} (host copy, informational)         */
    /* outputs of the last hyb_cg_step */
    double beta;          /* beta^m as computed (0 when m = 0)                   */
    double dmax;          /* max|d^m| of the direction searched (also read: the
                             next call starts its step search from twice
                             alpha * dmax)                                       */
    double alpha;         /* step taken (0 when no trial lowered J)              */
    double J_next;        /* J at the returned sigma                             */
    int32_t trials;       /* trial points evaluated, one forward sweep each      */
    int32_t restart;      /* 1: the direction restarted as -g^m                   */
    int32_t stalled;      /* 1: no trial lowered J; sigma unchanged, stop         */
    int32_t forwards;     /* forward sweeps the call ran                         */
} hyb_cg_state;

/* Create a context.  Validates the grid, the FEM mesh (see FEM box above;
 * HYB_E_MESH when it does not conform to the grid on the overlap, has two
 * nodes at one grid point, a degenerate tetrahedron or a node in no
 * tetrahedron) and the overlap width (must be 2), computes the P1 element
 * matrices and lumped masses of the mesh from its vertex coordinates and
 * allocates the wavefields.  opts may be NULL (FP64, history, gamma = 0.01,
 * alpha_rel = 0.25, default stream, structured path where possible).  fem
 * may be NULL for a pure finite-difference grid (no FEM box, no
 * conductivity).  On success *out owns the device state until hyb_destroy.
 * Errors: HYB_E_ARG, HYB_E_MESH, HYB_E_UNSUPPORTED, HYB_E_OOM, HYB_E_DEVICE. */
hyb_status hyb_create(const hyb_fd_grid *grid, const hyb_fem_mesh *fem,
                      const hyb_overlap *overlap, const hyb_opts *opts, hyb_ctx **out);

/* Release all device memory of the context (synchronises its stream). */
void hyb_destroy(hyb_ctx *ctx);

/* Forward solve (Algorithm 2, Sec. 7.5) for nt steps of size dt:
 * each step updates the FDM nodes with eq. (fdmschemeforward), the FEM nodes
 * with the lumped-mass scheme eq. (fem), the outer boundary with eq.
 * (eq:abs2) and the source of eq. (f), then copies the FEM values to the
 * FDM inner boundary omega_diamond and the FDM values to the FEM boundary
 * omega_o (Algorithm 1).  Zero initial data (Model Problem 2).
 * sigma_dev: device FP64 [n_params] (NULL = a = 1; must be NULL without FEM
 *            box).
 * obs_dev:   device FP64 [nt+1][face] receives the z+ trace (may be NULL).
 * Keeps what the adjoint needs according to opts.store_mode.
 * Errors: HYB_E_ARG (nt < 1, dt <= 0, source), HYB_E_CFL (structured: dt
 * above h/sqrt(3 max a); general: dt above h/sqrt(3), or dt^2 times the
 * Gershgorin bound max_n (|K_nn| + sum_m |K_nm|) / m_n of the FEM rows above
 * 4, a sufficient stability condition of the lumped-mass leapfrog),
 * HYB_E_NONFINITE (sigma not finite), HYB_E_OOM. */
hyb_status hyb_forward(hyb_ctx *ctx, const double *sigma_dev, const hyb_source *src,
                       int32_t nt, double dt, double *obs_dev);

/* Model Problem 1 initial data for the next hyb_forward (and only that one):
 * u0_dev, um1_dev are device FP64 [(n_z+1)(n_y+1)(n_x+1)] levels u^0 and
 * u^{-1} (NULL = zero).  Copied on the stream.  The FEM nodes take the values
 * of their grid nodes, so a general mesh with nodes off the grid returns
 * HYB_E_UNSUPPORTED.  Ends the Model Problem 1 data of
 * hyb_set_initial_taylor. */
hyb_status hyb_set_initial(hyb_ctx *ctx, const double *u0_dev, const double *um1_dev);

/* Model Problem 1 (eq. (model1), Sec. 5): initial data u(x,0) = f0,
 * u_t(x,0) = f1 for every later forward sweep of the context (those inside
 * hyb_cg_step included, so a CG run solves IP1), until the next call;
 * f0_dev = f1_dev = NULL returns to zero data (Model Problem 2, IP2).
 * f0_dev, f1_dev: device FP64 [(n_z+1)(n_y+1)(n_x+1)] full grid levels (NULL
 *   = 0 when the other is given); copied into the context on the stream (two
 *   grid levels of FP64 the context keeps until destroyed), so the caller may
 *   free them once the copy has run.
 * The paper gives the data, not the start.  The first level is the
 * second-order Taylor expansion u^1 = u^0 + dt f1 + (dt^2/2) A(u^0), with
 * A(u^0) the acceleration the scheme gives level 0: the leapfrog step from
 * the virtual level u^{-1} = f0 - dt f1 with dt^2 weighted by 1/2 in the
 * grid, FEM and ghost-node rows (the source flux at t = 0 included).  The
 * absorbing rows of eq. (eq:abs2) read levels 0 and 1 only and are
 * unchanged.  hyb_adjoint transposes that step, so the gradient's term of
 * step 0 carries the weight 1/2; hyb_get_wavefield(which = 1) returns the
 * cotangent of the level u^0 (with u^{-1} held fixed).
 * Replaces pending levels of hyb_set_initial, and hyb_set_initial replaces
 * these data.  Errors: HYB_E_UNSUPPORTED (general mesh with nodes off the
 * grid), HYB_E_STATE (context in a batch slot), HYB_E_OOM, HYB_E_DEVICE. */
hyb_status hyb_set_initial_taylor(hyb_ctx *ctx, const double *f0_dev, const double *f1_dev);

/* Variable wave speed: the coefficient 1/c^2 of the time derivative in
 * eq. (modelhyb), for every later sweep of the context until the next call
 * (NULL: c = 1, the model problems of Sec. 5).  Structured FEM boxes only.
 * eps_dev: device FP64 [C_z][C_y][C_x], 1/c^2 per FEM cube; used on the free
 *   cubes (c = 1 near and outside the FEM box, condition (coefic)), ignored
 *   elsewhere; copied into the context.  Values must be finite and > 0.
 * It weights the element mass matrices (M^K_ij = (phi_i/c^2, phi_j)_K,
 * Sec. 7.2), so after lumping the FEM row of node n divides by
 * m_n = sum_{K containing n} (1/c^2)_K |K| / 4; the 6-tetrahedra split gives
 * a cube's diagonal ends 1/4 of its volume and its other corners 1/12.  The
 * CFL check of hyb_forward becomes dt <= h sqrt(eps_min / (3 a_max)).
 * Synchronises the stream once (validation on the host); invalidates the
 * previous sweeps.  Errors: HYB_E_ARG (no FEM box, values not finite or
 * <= 0), HYB_E_UNSUPPORTED (general mesh), HYB_E_STATE (context in a batch
 * slot), HYB_E_OOM, HYB_E_DEVICE. */
hyb_status hyb_set_wave_speed(hyb_ctx *ctx, const double *eps_dev);

/* Derivative of the last adjoint's functional with respect to 1/c^2 per
 * cube, after hyb_adjoint (the exact derivative of the discrete scheme:
 * each FEM row's lumped mass is differentiated, using the second difference
 * of the node's forward levels k+1, k, k-1).
 * geps_dev: device FP64 [C_z][C_y][C_x]; mode 0 adjoint: the L2 density
 *   (1/h^3) dJ_misfit/d(1/c^2) (no regularisation term: the functional
 *   regularises a only); mode 1: the Euclidean dL/d(1/c^2).  0 on cubes that
 *   are not free.
 * Errors: HYB_E_ARG, HYB_E_STATE (no wave speed set, or no adjoint),
 * HYB_E_UNSUPPORTED (checkpoint store modes: the full FEM history is
 * needed). */
hyb_status hyb_gradient_eps(hyb_ctx *ctx, double *geps_dev);

/* Adjoint solve: the exact transpose of the last forward sweep, run backward
 * in time (in the interior it is eq. (fdmschemeadjoint) and the second line
 * of eq. (fem); boundary, source and exchange rows are transposed exactly).
 * residual_dev: device FP64 [nt+1][face].
 *   mode 0: residual = obs - data; the trace cotangent is
 *           tau * w_i * residual (trapezoid weights w_i on the z+ face,
 *           rectangle rule in time, z_delta = 1), i.e. the misfit part of
 *           eq. (functional);
 *   mode 1: residual is the raw cotangent dL/dobs (autograd).
 * Accumulates, fused with the FEM adjoint update, the FP64 time integral of
 * eq. (gradient1) per cube.  Requires a preceding hyb_forward (HYB_E_STATE).
 * Errors: HYB_E_ARG, HYB_E_STATE, HYB_E_OOM. */
hyb_status hyb_adjoint(hyb_ctx *ctx, const double *residual_dev, int32_t mode);

/* Finalise the gradient of the last adjoint into grad_dev (device FP64
 * [n_params]; 0 outside the free cells):
 *   mode 0: g_c = (1/|c|) dJ/dsigma_c + gamma * sigma_c, the L2 density of
 *           eq. (gradient1) for J of eq. (functional) (a_0 = 1), |c| the
 *           cell volume (h^3, or the tetrahedron's volume);
 *   mode 1: g_c = dL/dsigma_c (Euclidean, no regularisation).
 * J_host (nullable, mode 0 only): J = misfit + regularisation (synchronises).
 * Errors: HYB_E_ARG, HYB_E_STATE. */
hyb_status hyb_gradient(hyb_ctx *ctx, double *grad_dev, double *J_host);

/* hyb_gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same gradient of the last adjoint into grad_dev (device FP64 [n_params],
 * as hyb_gradient), and J (mode 0: misfit + regularisation; mode 1: 0) into
 * J_dev (device FP64 [1], nullable) instead of a host pointer, so nothing is
 * allocated and the stream is not synchronised.  The reduction scratch (one
 * partial sum per 256 parameters and the scalars) is a static device array
 * of 131 200 bytes that each GPU holds until the process ends; calls on one
 * GPU share it, so calls that overlap on one GPU (other streams, other
 * threads) race.  The context's own buffers must exist already (they do
 * after hyb_adjoint).
 * Errors: HYB_E_ARG, HYB_E_STATE (no adjoint), HYB_E_UNSUPPORTED (more than
 * 4 194 304 parameters: the scratch is full), HYB_E_DEVICE. */
hyb_status hyb_gradient_noalloc(hyb_ctx *ctx, double *grad_dev, double *J_dev);

/* One iteration m of Algorithm 3 (Sec. 8) at sigma^m = sigma_dev (device FP64
 * [n_params], updated in place to sigma^{m+1}), all in FP64 on the device:
 *   1. forward at sigma^m (skipped when the previous call's accepted trial
 *      was this sigma: same state, data_dev, source, nt, dt, and sigma_dev
 *      bitwise unchanged, which the call checks on the device), residual
 *      obs - data, adjoint, gradient g^m of eq. (gradient1) and J^m;
 *   2. beta^m = |g^m|^2 / |g^{m-1}|^2 (beta^0 = 0; L2 norms weighted by the
 *      cell volumes), d^m = -g^m + beta^m d^{m-1} on the free cells; when
 *      m > 0 and the slope sum |c| g_c d_c over the cells free to move (not
 *      held by a bound: sigma = 0 moving down, sigma = 4 moving up) is >= 0,
 *      d^m = -g^m (restart);
 *   3. step length (the paper refers to another work for it): trial steps
 *      alpha_t = 2^-t rho / max|d^m|, t = 0 .. opts.cg_max_trials - 1, with
 *      the first relative step (largest change of sigma) rho = alpha_rel at
 *      m = 0 and min(alpha_rel, 2 state->alpha state->dmax), twice the
 *      previous call's accepted one, afterwards (alpha_rel again after a
 *      stalled call);
 *      each trial point clip(sigma^m + alpha_t d^m, 0, 4) (free cells,
 *      eq. (admpar)) costs one forward sweep; the first with J < J^m becomes
 *      sigma^{m+1}.  When none lowers J, sigma stays, state->stalled = 1 and
 *      the run should stop.
 * The direction d lives in the context.  state (in/out): iter counts
 * iterations, the other fields report the call.  *gnorm_host (nullable)
 * receives |g^m|_{L2} for the stopping test, *J_host (nullable) J^m; the call
 * synchronises the stream once per trial.
 * Errors: as hyb_forward/hyb_adjoint; HYB_E_ARG for a null pointer. */
hyb_status hyb_cg_step(hyb_ctx *ctx, const double *data_dev, double *sigma_dev,
                       const hyb_source *src, int32_t nt, double dt, hyb_cg_state *state,
                       double *gnorm_host, double *J_host);

/* Device bytes a context with these arguments needs for nt steps (fields,
 * history or checkpoints, accumulators), without allocating anything.  Not
 * included: the buffers hyb_set_initial_taylor adds (two FP64 grid levels)
 * and those of hyb_set_wave_speed (per cube 8 bytes, per FEM node 8 bytes
 * plus one field element, one history level).
 * Errors: HYB_E_ARG, HYB_E_MESH, HYB_E_UNSUPPORTED. */
hyb_status hyb_footprint(const hyb_fd_grid *grid, const hyb_fem_mesh *fem,
                         const hyb_overlap *overlap, const hyb_opts *opts, int32_t nt,
                         size_t *bytes);

/* Wait for all work of the context; returns the first pending device error. */
hyb_status hyb_sync(hyb_ctx *ctx);

/* Text of the last error of ctx (or of the last failed hyb_create when ctx
 * is NULL).  The string is owned by the library. */
const char *hyb_last_error(const hyb_ctx *ctx);

/* Node counts used by the throughput metric: *fdm = nodes updated by the
 * finite-difference scheme or the outer boundary rows per step, *fem = FEM
 * nodes updated per step. */
hyb_status hyb_counts(const hyb_ctx *ctx, int64_t *fdm, int64_t *fem);

/* The FEM box of a context: *n_params = number of conductivity values
 * (cubes, or tetrahedra of a general mesh; 0 without FEM box), *general = 1
 * on the general path, *n_fem_nodes = FEM nodes (length of the FEM part of
 * hyb_get_wavefield).  Any pointer may be NULL. */
hyb_status hyb_fem_info(const hyb_ctx *ctx, int64_t *n_params, int32_t *general, int64_t *n_fem_nodes);

/* Average device time (ms) of one launch of the dominant kernel (the fused
 * FDM/FEM interior update of the forward sweep) over `reps` launches on the
 * context's stream, measured with HIP events around the launches, after the
 * given forward set-up (sigma_dev, dt).  The wavefield content is arbitrary
 * (the kernel's cost does not depend on values).  Synchronises.
 * Errors: HYB_E_ARG, HYB_E_STATE, HYB_E_DEVICE. */
hyb_status hyb_time_interior(hyb_ctx *ctx, const double *sigma_dev, double dt, int32_t reps,
                             double *ms_host);

/* Average device time (ms) of one launch of the FEM row kernel of a general
 * mesh (which 0: forward rows, which 1: adjoint rows with the gradient
 * accumulation) over `reps` launches, with HIP events on the context's
 * stream, at the conductivity and dt of the last forward.  Needs a previous
 * hyb_forward (and hyb_adjoint for which 1); the launches overwrite the
 * fields, so the sweeps are no longer available afterwards.  Synchronises.
 * Errors: HYB_E_ARG, HYB_E_STATE (no general mesh or no previous sweep),
 * HYB_E_DEVICE. */
hyb_status hyb_time_fem(hyb_ctx *ctx, int32_t which, int32_t reps, double *ms_host);

/* Copy the newest level of the last sweep to caller buffers (FP64, unpadded):
 *   which 0: u^{nt} of the last forward sweep;
 *   which 1: the multipliers of level 0 of the last adjoint sweep, i.e. the
 *            cotangent of u^0 (grid part; the FEM part is the cotangent of the
 *            FEM copy of u^0, to be added on the FEM box nodes).
 * Grid nodes strictly inside the hole (o+2, o+C-2)^3 belong to no grid row
 * (the FEM part holds the solution there) and are returned as 0.
 * u_dev: device [(n_z+1)(n_y+1)(n_x+1)] grid part (nullable);
 * v_dev: device [n_fem_nodes] FEM part in the mesh's node order (nullable;
 *        ignored without FEM box).
 * Errors: HYB_E_ARG, HYB_E_STATE (no such sweep yet). */
hyb_status hyb_get_wavefield(hyb_ctx *ctx, int32_t which, double *u_dev, double *v_dev);

/* ---------------------------------------------------------------------
 * Batched solves for request serving.  A batch advances many contexts at
 * once: every hyb_batch_tick performs one time step of every running slot,
 * and slots whose contexts have the same geometry (grid, FEM box, dt,
 * precision) run in the same kernel launches, each at its own step and
 * phase.  A slot runs one forward+adjoint+gradient solve: the forward sweep,
 * the residual obs - data, the adjoint sweep (mode 0) and the gradient of
 * hyb_gradient mode 0; results land in the caller's obs and grad buffers.
 * Each slot's arithmetic follows hyb_forward/hyb_adjoint/hyb_gradient step
 * for step; the batched kernels are separately compiled, so results agree
 * with those calls (and alone vs in a mix) to rounding, not bit for bit.
 */
typedef struct hyb_batch hyb_batch;

/* Create a batch of up to max_slots slots.  Each slot's work goes to the
 * stream of its context; slots on different streams run concurrently on the
 * device (a typical server gives each grid size its own stream), slots on
 * the same stream and geometry share launches.  hip_stream names the first
 * stream; pinned staging rings are allocated per stream.
 * Errors: HYB_E_ARG, HYB_E_OOM. */
hyb_status hyb_batch_create(int32_t max_slots, void *hip_stream, hyb_batch **out);

/* Release the batch (synchronises its stream; contexts stay with the caller). */
void hyb_batch_destroy(hyb_batch *b);

/* Start a solve on context ctx (structured FEM box required, full-history
 * store mode) in a free slot.  sigma_dev as in hyb_forward; sigma_max: the caller's
 * value of max(sigma) over the free cubes, used for the CFL check without a
 * device round trip; data_dev, obs_dev [nt+1][face] and grad_dev [C^3] are
 * device FP64 buffers owned by the caller and kept valid until the slot is
 * released.  *slot receives the slot number.
 * Errors: HYB_E_ARG, HYB_E_STATE (no free slot / context busy), HYB_E_CFL,
 * HYB_E_UNSUPPORTED (checkpoint store modes, general meshes), HYB_E_OOM. */
hyb_status hyb_batch_submit(hyb_batch *b, hyb_ctx *ctx, const double *sigma_dev, double sigma_max,
                            const hyb_source *src, int32_t nt, double dt, const double *data_dev,
                            double *obs_dev, double *grad_dev, int32_t *slot);

/* Up to `steps` ticks; each tick enqueues one time step of every running
 * slot (asynchronous).  Stops early when no slot is running.  *n_active
 * (nullable) receives the number of slots that stepped in the first tick.
 * The host plans up to 32 ticks at a time and ships their step arguments in
 * one copy per stream; it blocks only when it runs more than 16 such plans
 * ahead of the device. */
hyb_status hyb_batch_tick(hyb_batch *b, int32_t steps, int32_t *n_active);

/* State of a slot: -1 free, 0 running, 1 all work enqueued, 2 finished
 * (results valid; *J_host, nullable, receives J = misfit + regularisation),
 * 3 failed: sigma had non-finite entries, or its maximum on the device
 * exceeded the sigma_max given to hyb_batch_submit (the CFL check used that
 * value); hyb_batch_last_error names the reason.  Does not block. */
hyb_status hyb_batch_poll(hyb_batch *b, int32_t slot, int32_t *state, double *J_host);

/* hyb_batch_poll for every slot: state[max_slots], J[max_slots] (nullable). */
hyb_status hyb_batch_poll_all(hyb_batch *b, int32_t *state, double *J_host);

/* Free a slot whose work has been enqueued (waits for it to finish). */
hyb_status hyb_batch_release(hyb_batch *b, int32_t slot);

/* Text of the last batch error. */
const char *hyb_batch_last_error(const hyb_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* HYB_H */
