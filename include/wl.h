/*
 * wl.h - C ABI of the MI355X (gfx950) incompressible Navier-Stokes hot path.
 *
 * Method: Weymouth & Font, "WaterLily.jl: A differentiable fluid simulator in
 * Julia with fast heterogeneous execution" (arXiv 2304.08159), Sec. 2: a
 * uniform Cartesian grid, third-order finite-volume convection-diffusion with
 * explicit adaptive time stepping and implicit LES, Boundary Data Immersion
 * (BDIM) of a signed-distance body that also modifies the pressure-Poisson
 * matrix, and a geometric-multigrid (GMG) pressure solve followed by the
 * pressure-gradient update u[I,i] -= coeff[I,i]*(p[I]-p[I-del(i)]).
 * Sec. 3 (Tables 1-2) times the step simstep! and its routines convdiff!,
 * BDIM!, BC!, project! and CFL!.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Grid      : n[0] x n[1] x n[2] cells, spacing 1.  2D problems use
 *              ndim = 2 and n[2] = 1.  Cell I has centre I + 1/2.
 *  Layout    : every field is an interior-only, contiguous array of
 *              n[0]*n[1]*n[2] elements, x fastest (index x + n0*(y + n1*z)).
 *              Velocity component i sits on the LOWER i-face of each cell.
 *              In a non-periodic direction i the stored face with index 0 is
 *              the domain-boundary face; the upper x boundary face of an
 *              OUTFLOW boundary is a separate plane of n[1]*n[2] values
 *              (field WL_FIELD_UOUT, y fastest).
 *  Precision : WL_FP32 fields are float, WL_FP64 fields are double,
 *              WL_MIXED: float fields, FP32 V-cycles, FP64 outer
 *              defect-correction residual; Poisson x, b and coefficients are
 *              double in MIXED mode.
 *  Memory    : all array arguments are DEVICE pointers owned by the caller.
 *              The library never allocates device memory: each handle lives
 *              in a caller-supplied device workspace whose exact size the
 *              *_footprint call returns (host-only computation).  The library
 *              keeps the workspace and the stream given at creation, and no
 *              other pointer beyond a call.  Per handle it owns a 128-byte
 *              pinned host buffer (scalar results are read through it), a
 *              capture stream of default priority and at most two executable
 *              graphs, created on first use and released by *_destroy.
 *  Streams   : work is enqueued on the creation stream (a hipStream_t passed
 *              as void*, NULL = default stream).  Calls that return scalar
 *              results (residuals, V-cycle counts, dt) synchronise it.
 *  Errors    : every call returns a wl_status; negative values are errors and
 *              wl_last_error() gives a message (thread-local, valid until the
 *              next call on the same thread).  WL_ERR_NOT_CONVERGED leaves
 *              the last iterate in place with its residual reported; after
 *              any other error the outputs are unspecified and the handle
 *              remains usable unless the status is WL_ERR_HIP.
 *  Threads   : a handle must not be used from two threads at once.
 */
#ifndef WL_H
#define WL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WL_OK = 0,
    WL_ERR_INVALID_ARG = -1,
    WL_ERR_OUT_OF_MEMORY = -2,   /* workspace smaller than the footprint       */
    WL_ERR_NOT_CONVERGED = -3,   /* max V-cycles reached before the tolerance */
    WL_ERR_NONFINITE = -4,       /* NaN/Inf met in a residual norm            */
    WL_ERR_HIP = -5,             /* a HIP runtime call failed                 */
    WL_ERR_STATE = -6            /* call not valid in the handle's state      */
} wl_status;

typedef enum { WL_FP32 = 0, WL_FP64 = 1, WL_MIXED = 2 } wl_precision;

/* Domain-face boundary codes.  PERIODIC must be set on both faces of a
 * direction.  INFLOW only on the lower x face, OUTFLOW only on the upper x
 * face.  For the pressure every non-periodic face is homogeneous Neumann. */
typedef enum {
    WL_BC_PERIODIC = 0,
    WL_BC_INFLOW = 1,   /* velocity = U on the boundary face and its ghosts  */
    WL_BC_OUTFLOW = 2,  /* convective outflow plane with exit-flux balance   */
    WL_BC_WALL = 3      /* free-slip wall (zero normal velocity)             */
} wl_bc;

/* Body given by its signed-distance function (Sec. 2): kind 0 = none,
 * kind 1 = sphere (circle when ndim = 2) of the given centre and radius in
 * cell units, kind 2 = torus (the donut of Sec. 3; ndim = 3 only) whose axis
 * is the x direction through centre, with major radius `radius` (centre to
 * the tube's centre line) and minor radius `radius2` (the tube's), so that
 * d = sqrt(x^2 + (sqrt(y^2 + z^2) - radius)^2) - radius2 relative to centre.
 * eps is the BDIM kernel half-width (<= 0 selects 1 cell).  radius2 is read
 * for kind 2 only.  Drag and the adjoint step support kinds 0 and 1.
 *
 * Motion (Sec. 2: the body is its SDF composed with a coordinate map; here
 * the map of a rigid motion).  The centre follows
 *     X(t) = centre + velocity t + amplitude sin(omega t)
 * and the body spins at the constant angular velocity `spin` (kind 1 only:
 * the sphere's shape is unchanged by it; in 2D only spin[2], about z).  The
 * body velocity V_b(x, t) = dX/dt + spin x (x - X(t)) enters the BDIM blend,
 *     u* = mu0 f + (1 - mu0) V_b + (mu1 n) . (grad f - grad V_b),
 * and a moving body is measured again before every step at the time t + dt
 * the step advances to (moments, Poisson coefficients on every level, tile
 * classes).  All zero (the default of a zero-initialised struct): a body at
 * rest.  In 2D the z components of velocity and amplitude must be 0.  The
 * body must stay clear of periodic boundaries (its SDF is not wrapped).
 * Moving bodies are not supported by the adjoint step. */
typedef struct {
    int kind;
    double centre[3];
    double radius;
    double eps;
    double radius2;
    double velocity[3];   /* drift of the centre (cells per time unit)       */
    double amplitude[3];  /* oscillation amplitude of the centre (cells)     */
    double omega;         /* oscillation angular frequency (1 / time unit)    */
    double spin[3];       /* angular velocity of the body (1 / time unit)     */
} wl_body;

typedef struct {
    int ndim;             /* 2 or 3                                          */
    int n[3];             /* cells per direction (n[2] = 1 when ndim = 2)     */
    int bc_lo[3];         /* wl_bc per lower domain face                      */
    int bc_hi[3];         /* wl_bc per upper domain face                      */
    double U[3];          /* inflow / reference velocity, cells per time unit */
    double nu;            /* kinematic viscosity in grid units                */
    wl_body body;
    int prec;             /* wl_precision                                     */
    int mg_levels;        /* 0 = automatic coarsening                         */
    double tol;           /* pressure-solve tolerance, read per stop_rule     */
    int max_vcycles;      /* per pressure solve (<= 0 selects 100)            */
    int inner_vcycles;    /* MIXED: FP32 V-cycles per outer iteration (0: 3)  */
    double cfl;           /* CFL number of the adaptive time step (0: 0.5)    */
    int tape_steps;       /* steps the adjoint tape can hold (0: no adjoint)  */
    int stop_rule;        /* wl_stop_rule of the in-step pressure solves      */
} wl_sim_desc;

/* When an in-step pressure solve stops (tested before each V-cycle, on the
 * projection right-hand side sigma = div(u*)/(c dt) and the current pressure
 * iterate p of the stage, Sec. 2 project!):
 *  WL_STOP_DIVERGENCE: once the divergence the solve leaves in the projected
 *    velocity, c dt (sigma - A p), has RMS over the active cells <= tol.  For
 *    FP32 fields this is the usable rule: the rounding of an FP32 pressure
 *    alone floors ||sigma - A p|| / ||sigma|| near 1e-5 on large grids, while
 *    the divergence it leaves stays at the velocity's own rounding.
 *  WL_STOP_RELATIVE: once ||sigma - A p||_2 <= tol ||sigma||_2 (FP64 or MIXED
 *    fields, where the relative residual has no such floor). */
typedef enum { WL_STOP_DIVERGENCE = 0, WL_STOP_RELATIVE = 1 } wl_stop_rule;

typedef struct {
    double dt;            /* time step taken                                  */
    double t;             /* simulation time after the step                   */
    int vcycles[2];       /* V-cycles of the predictor and corrector solves   */
    double resid[2];      /* RMS divergence each solve leaves in the projected
                             velocity, c dt ||sigma - A p||_2 / sqrt(n_active) */
    double rel_resid[2];  /* relative residual each solve reached,
                             ||sigma - A p||_2 / ||sigma||_2 (sigma with
                             inactive cells dropped and the active mean removed;
                             0 when sigma is 0)                               */
} wl_step_stats;

/* Fields addressable by wl_set_field / wl_get_field. */
enum {
    WL_FIELD_U0 = 0, WL_FIELD_U1 = 1, WL_FIELD_U2 = 2,  /* velocity, r/w     */
    WL_FIELD_P = 3,                                     /* pressure, r/w     */
    WL_FIELD_UOUT = 4,     /* outflow plane (n1*n2), r/w                     */
    WL_FIELD_L0 = 5, WL_FIELD_L1 = 6, WL_FIELD_L2 = 7,  /* Poisson coeff, r  */
    WL_FIELD_MU0_0 = 8, WL_FIELD_MU0_1 = 9, WL_FIELD_MU0_2 = 10, /* mu0, r   */
    WL_FIELD_MU1N = 11,    /* (mu1 n)_ij, 9 consecutive fields i*3+j, r      */
    WL_FIELD_SIGMA = 20    /* projection RHS of the last stage, r            */
};

typedef struct wl_sim wl_sim;
typedef struct wl_poisson wl_poisson;

/* ---- Navier-Stokes simulation (the simstep! analogue, Sec. 2-3) -------- */

/* Exact workspace size in bytes for a simulation described by desc.
 * Host-only; validates desc (WL_ERR_INVALID_ARG on a bad description). */
wl_status wl_sim_footprint(const wl_sim_desc* desc, size_t* bytes);

/* Create a simulation in the caller's device workspace (>= footprint bytes,
 * 256-byte aligned).  Measures the body (BDIM moments and Poisson
 * coefficients on every multigrid level), sets u = U on every face (boundary
 * faces to their boundary values), p = 0, t = 0, and synchronises. */
wl_status wl_sim_create(const wl_sim_desc* desc, void* workspace, size_t ws_bytes,
                        void* hip_stream, wl_sim** out);
wl_status wl_sim_destroy(wl_sim* sim);

/* Copy one field from / to a caller device array in the layout above.
 * Writing U or UOUT invalidates the cached CFL maximum.  mu1n fields use
 * field WL_FIELD_MU1N + 3*i + j. */
wl_status wl_set_field(wl_sim* sim, int field, const void* src);
wl_status wl_get_field(const wl_sim* sim, int field, void* dst);
wl_status wl_set_time(wl_sim* sim, double t);

/* Checkpoint / restart of a simulation (the state simstep! carries from one
 * step to the next, Sec. 2-3): everything a later step reads, so that
 * restoring a snapshot and stepping on gives bitwise the results of never
 * having stopped.  The snapshot is one caller-owned DEVICE buffer of
 * wl_state_size bytes (256-byte aligned), laid out as
 *   bytes [0, 64)   : 8 doubles: format tag 1, time t, dt of the next
 *                     CFL-adaptive step (0 when it is not yet known), ndim,
 *                     n[0], n[1], n[2], precision;
 *   then, each section at the next 256-byte boundary (first at 256): the
 *   ndim velocity components (n cells each, sim dtype, wl_get_field layout),
 *   the outflow plane (OUTFLOW simulations only, n[1]*n[2] values), the
 *   pressure (n cells) and, for WL_MIXED, the FP64 pressure iterate the
 *   mixed-precision solve warm-starts from (n doubles).
 * Geometry, coefficients and the adjoint tape are not part of it (they are
 * fixed by the description or recorded anew).  Both calls synchronise the
 * stream.  wl_set_state returns WL_ERR_INVALID_ARG when the header does not
 * match this simulation (tag, grid or precision) and then changes nothing. */
wl_status wl_state_size(const wl_sim* sim, size_t* bytes);
wl_status wl_get_state(const wl_sim* sim, void* dst);
wl_status wl_set_state(wl_sim* sim, const void* src);

/* Advance one Heun step (predictor and corrector, each: convection-diffusion,
 * BDIM blend, boundary rules, divergence, GMG pressure solve, projection).
 * dt <= 0 selects the CFL-adaptive step from the current velocity.  stats
 * may be NULL.  Returns WL_ERR_NOT_CONVERGED when a solve hits max_vcycles
 * (the step is still completed with the last iterate). */
wl_status wl_step(wl_sim* sim, double dt, wl_step_stats* stats);

/* Advance CFL-adaptive steps in one call, as the paper's time loop does
 * (sim_step! to a target time, Sec. 2): at most nsteps steps, stopping once
 * the time reaches t_end (t_end <= 0: no time limit).  stats (may be NULL)
 * holds room for nsteps entries and receives one per step taken; *taken
 * (may be NULL) the number of steps taken.  Stops at the first step whose
 * status is not WL_OK and returns that status (a WL_ERR_NOT_CONVERGED step
 * is completed and counted).  WL_ERR_INVALID_ARG for nsteps < 0. */
wl_status wl_run(wl_sim* sim, int nsteps, double t_end, wl_step_stats* stats, int* taken);

/* ---- Adjoint of the step (the solver is differentiable, Sec. 2) --------- */

/* Pressure drag of the body from the current pressure (the corrector
 * pressure of the last step): F_x = -sum over active cells of
 * (p - mean p) n_x K(d) at cell centres, K the BDIM kernel, n = grad d. */
wl_status wl_drag(wl_sim* sim, double* Fx);

/* Start (on != 0) or stop recording an adjoint tape: while recording, each
 * wl_step stores its intermediate fields (state, stage fields, pressures,
 * dt) in the next free slot of the tape (at most desc.tape_steps slots,
 * carved from the workspace; steps taken once it is full are not recorded).
 * Starting clears the tape and the geometry adjoint accumulators.
 * WL_ERR_STATE when the simulation was created with tape_steps = 0. */
wl_status wl_tape_record(wl_sim* sim, int on);

/* Reverse one recorded step (the most recent one still on the tape), with dt
 * and the limiter / upwind branches frozen at their forward values and every
 * pressure solve treated as exact (its adjoint is the same GMG solve).
 * ubar_in: adjoint of the state after the step (ndim face arrays followed by
 * the outflow plane when there is one; sim dtype).  pbar_in (may be NULL =
 * zero): adjoint of the pressure after the step (the corrector's pressure,
 * n cells, sim dtype); the pressure is determined up to a constant, so the
 * part of pbar_in that is constant over the active cells (and its values on
 * inactive cells) does not contribute.  ubar_out: adjoint of the state
 * before it (same layout as ubar_in; may alias it).  The pressure before the
 * step is only the solves' starting guess, so it has no adjoint.
 * drag_weight: dJ/dF_x of the step's drag (added to pbar_in's effect).
 * g_params[4] (host, may be NULL) accumulates dJ/d(radius, centre x, y, z)
 * through the geometry (BDIM moments, Poisson coefficients, drag weights).
 * Synchronous on the simulation's stream.  WL_ERR_STATE when the tape is
 * empty. */
wl_status wl_step_adjoint(wl_sim* sim, const void* ubar_in, const void* pbar_in,
                          double drag_weight, void* ubar_out, double* g_params);

/* ---- Standalone pressure-Poisson GMG solve (project!, Sec. 2) ---------- */

/* Exact workspace size of a Poisson solver.  periodic[i] != 0 makes
 * direction i periodic, otherwise its faces are Neumann.  levels = 0 selects
 * automatic coarsening. */
wl_status wl_poisson_footprint(int ndim, const int n[3], const int periodic[3], int prec,
                               int levels, size_t* bytes);
wl_status wl_poisson_create(int ndim, const int n[3], const int periodic[3], int prec,
                            int levels, void* workspace, size_t ws_bytes, void* hip_stream,
                            wl_poisson** out);

/* Solve A x = b with A the coefficient-weighted 2d-point operator
 *   (A x)(I) = sum_i L_i(I+delta_i)(x(I+delta_i)-x(I)) - L_i(I)(x(I)-x(I-delta_i)).
 * coeffs: ndim consecutive face arrays L_0, L_1[, L_2] (lower faces, layout
 * above); the lower face of a non-periodic direction is treated as zero.
 * Pass NULL to reuse the coefficients of the previous call.  x: initial guess
 * in, solution out.  b is read only: the solver uses b with inactive cells
 * (all face coefficients zero) dropped and the active mean removed.  V-cycles
 * run until ||b - A x|| <= tol ||b|| (tested before each cycle) or
 * max_vcycles.  vcycles_out / rel_resid_out may be NULL. */
wl_status wl_poisson_solve(wl_poisson* ps, const void* coeffs, void* x, const void* b,
                           double tol, int max_vcycles, int* vcycles_out,
                           double* rel_resid_out);
wl_status wl_poisson_destroy(wl_poisson* ps);

/* ---- Batched small Poisson solves (serving) ------------------------------ */

/* One Poisson problem of a batch: the same operator, method and stopping rule
 * as wl_poisson_solve (Sec. 2, project!).  coeffs: ndim face arrays of
 * double (layout above; zero faces are walls / solid); x: initial guess in,
 * solution out (double); b: right-hand side (double, projected onto the
 * active cells and made mean-free there by the solver, not modified).  All
 * device pointers owned by the caller.  mixed = 0: FP64 V-cycles; mixed = 1:
 * FP32 V-cycles (three per outer iteration, from zero, on FP32 copies of the
 * coefficients) with the FP64 defect correction x += e around them, as
 * WL_MIXED (the residual test and x stay FP64).  At most 262144 cells; the
 * coarsest multigrid level (every direction halved while all are even and
 * >= 8) must have at most 1024 cells. */
typedef struct {
    int ndim;
    int n[3];
    int periodic[3];
    const void* coeffs;
    void* x;
    const void* b;
    double tol;           /* stop once ||b - A x|| <= tol ||b||              */
    int max_vcycles;      /* mixed: inner FP32 V-cycles in total             */
    int mixed;
} wl_batch_request;

typedef struct {
    int status;           /* WL_OK, WL_ERR_NOT_CONVERGED or WL_ERR_NONFINITE  */
    int vcycles;
    double rel_resid;
} wl_batch_result;

/* Exact device workspace for wl_poisson_batch_solve on these requests (host
 * only; pointers may be NULL here).  WL_ERR_INVALID_ARG names the first
 * request that is malformed or too large. */
wl_status wl_poisson_batch_footprint(const wl_batch_request* reqs, int count, size_t* bytes);

/* Solves count requests with one persistent kernel on hip_stream: its
 * workgroups (at most one per compute unit) take requests from a device work
 * queue until it is empty, one request per workgroup at a time.  Every
 * reduction is a fixed-order workgroup sum, so each request's result is
 * bitwise independent of the batch it is in.  workspace: >= the footprint,
 * 256-byte aligned.  results: count entries (host), filled on return
 * (synchronises the stream).  Returns WL_OK when every request converged,
 * else the first failing request's status. */
wl_status wl_poisson_batch_solve(const wl_batch_request* reqs, int count, void* workspace,
                                 size_t ws_bytes, void* hip_stream, wl_batch_result* results);

/* wl_poisson_batch_solve for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same requests, method, kernel and results (bitwise), with no workspace
 * argument.  The batch's device scratch (request table, results, queue head
 * and every request's multigrid level arrays, wl_poisson_batch_footprint
 * bytes) lives in a 32 MiB array of device memory that the library holds per
 * GPU for the life of the process; the host side uses fixed tables.  The call
 * makes no device or pinned allocation.  Limits: at most 256 requests, and a
 * footprint of at most 32 MiB (e.g. 64 requests of 128^2 cells); larger
 * batches return WL_ERR_INVALID_ARG with a message naming the size.  Every
 * call on one GPU uses that GPU's single scratch array: calls that overlap on
 * the same GPU (from several threads or streams) race and must be
 * serialised by the caller; this process serialises the host part itself.
 * Synchronises hip_stream; results as wl_poisson_batch_solve. */
wl_status wl_poisson_batch_solve_noalloc(const wl_batch_request* reqs, int count,
                                         void* hip_stream, wl_batch_result* results);

/* ---- Batched small Navier-Stokes runs (serving) ------------------------- */

/* One small simulation of a batch: `steps` CFL-adaptive Heun steps (Sec. 3
 * simstep!: convection-diffusion, BDIM, boundary rules, GMG projection, CFL)
 * of the flow described as in wl_sim_desc, with FP32 fields and each pressure
 * solve in FP32 V-cycles with an FP64 defect correction to the relative
 * residual tol (the method and readings of WL_MIXED with WL_STOP_RELATIVE).
 * The body (kinds 0-2) must be at rest.  u: ndim face arrays of float
 * (layout above), the state in and out; uout: the outflow plane (float,
 * n[1]*n[2]; OUTFLOW requests only, else NULL); p: the pressure (double,
 * n cells), the solves' warm start in and the last solve's result out.  All
 * device pointers owned by the caller.  At most 262144 cells; the coarsest
 * multigrid level (every direction halved while all are even and >= 8) must
 * have at most 1024 cells. */
typedef struct {
    int ndim;
    int n[3];
    int bc_lo[3];
    int bc_hi[3];
    double U[3];
    double nu;
    wl_body body;
    double tol;           /* relative residual of every pressure solve       */
    int max_vcycles;      /* inner FP32 V-cycles per solve (<= 0: 100)        */
    int steps;
    double cfl;           /* <= 0: 0.5                                        */
    void* u;
    void* uout;
    void* p;
} wl_ns_request;

typedef struct {
    int status;           /* WL_OK, WL_ERR_NOT_CONVERGED (some solve hit
                             max_vcycles; the run still completes),
                             WL_ERR_NONFINITE or WL_ERR_INVALID_ARG (a time
                             step that is not positive)                      */
    int vcycles;          /* inner V-cycles of all its solves                 */
    double t;             /* simulated time                                   */
    double dt;            /* last time step                                   */
} wl_ns_result;

/* Exact device workspace for wl_ns_batch_run on these requests (host only;
 * the requests' device pointers may be NULL here).  WL_ERR_INVALID_ARG names
 * the first request that is malformed or too large. */
wl_status wl_ns_batch_footprint(const wl_ns_request* reqs, int count, size_t* bytes);

/* Runs count requests with one persistent kernel on hip_stream: its
 * workgroups (at most one per compute unit) take requests from a device work
 * queue until it is empty; a request's whole run is taken by one workgroup,
 * every phase of a step a loop over its cells followed by a barrier, every
 * reduction a fixed-order workgroup sum, so each result is bitwise
 * independent of the batch it is in.  workspace: >= the footprint, 256-byte
 * aligned.  results: count entries (host), filled on return (synchronises
 * the stream).  Returns WL_OK when every request completed cleanly, else the
 * first failing request's status. */
wl_status wl_ns_batch_run(const wl_ns_request* reqs, int count, void* workspace, size_t ws_bytes,
                          void* hip_stream, wl_ns_result* results);

/* BDIM-modified Poisson coefficients of a body (Sec. 2): L_i = mu0 of the
 * signed distance at every lower i-face centre (cosine kernel of half-width
 * body->eps, <= 0 selects 1 cell), zero on non-periodic lower boundary faces;
 * body->kind == 0 gives L = 1.  L_out receives ndim consecutive face arrays
 * (layout above) of float (prec WL_FP32) or double (WL_FP64, WL_MIXED).
 * Enqueued on hip_stream and synchronised before returning. */
wl_status wl_body_coeffs(const wl_body* body, int ndim, const int n[3], const int periodic[3],
                         int prec, void* L_out, void* hip_stream);

/* ---- Execution ----------------------------------------------------------- */

/* Repeated solve bodies (one V-cycle with its residual norm; one
 * mixed-precision outer iteration) are captured once per solver and solution
 * array, on a private stream of default priority, and replayed as HIP graphs
 * on the caller's stream from their second use on (default, enable != 0).
 * enable = 0 launches every kernel individually.  Results are bitwise the
 * same either way.  Process-wide; bodies are launched individually while any
 * multigrid kernel class is timed (wl_profile_enable). */
wl_status wl_set_graphs(int enable);

/* Each pre- and post-smoothing pair of damped-Jacobi sweeps (Sec. 2's GMG
 * smoother) on a uniform, fully periodic 3D level whose x and y extents are
 * multiples of 8 runs as one kernel that keeps the intermediate iterate on
 * chip; the V-cycle then also checks the residual with a measuring pass that
 * writes nothing, and a simulation's divergence kernel takes each solve's
 * first check.  Levels with face coefficients or walls are fused too from
 * 2^22 cells up.  The coarse end of each V-cycle (the levels of at most 16^3
 * cells, with a coarsest level of at most 128 cells) runs as one
 * one-workgroup launch.  Iterates are bitwise the same as with separate
 * sweeps and per-level launches (the reported residual norms agree to
 * rounding).  mode 0: separate sweeps and per-level launches everywhere; 1
 * (default) and 2: fused (1 honours the minimum level sizes; 2 fuses every
 * eligible level).  Process-wide; a solver or simulation takes the mode in
 * force when it is created.  WL_ERR_INVALID_ARG for another mode. */
wl_status wl_set_fused_sweeps(int mode);

/* Smoother of the multigrid levels (every level but the coarsest, which is
 * solved exactly).  WL_SMOOTH_JACOBI (default): damped Jacobi,
 * w = 2d/(2d+1), two sweeps before and two after the coarse correction.
 * WL_SMOOTH_CG: the conjugate-gradient smoothing Sec. 2 names for the GMG
 * levels: each smoothing step is a fresh run of two Jacobi-preconditioned CG
 * iterations on the level's system from the current iterate, with the
 * residual kept mean-free over the active cells; every dot product is a
 * fixed-order FP64 device reduction and no scalar returns to the host, so
 * results are deterministic and the V-cycle can be replayed as a graph.
 * CG smoothing needs four more arrays per level (residual, direction, M p,
 * inverse diagonal) and turns off the fused Jacobi sweep pairs.
 * Process-wide; a solver or simulation takes the smoother in force when its
 * footprint is computed and when it is created (keep it unchanged between
 * the two).  The batched solver (wl_poisson_batch_solve) always uses Jacobi.
 * WL_ERR_INVALID_ARG for another kind. */
enum { WL_SMOOTH_JACOBI = 0, WL_SMOOTH_CG = 1 };
wl_status wl_set_smoother(int kind);

/* ---- Kernel timing (measurement support) -------------------------------- */

/* Kernels whose launches can be bracketed by HIP events, to turn algorithmic
 * bytes into achieved bandwidth without an external profiler.  Fine level
 * means the caller's grid (level 0 of the multigrid hierarchy). */
enum {
    WL_PROF_SMOOTH_FINE = 0,     /* plain damped-Jacobi sweep, fine level     */
    WL_PROF_SMOOTH_NORM = 1,     /* sweep fused with the residual norm        */
    WL_PROF_PROLONG_FINE = 2,    /* prolongation added in place, fine level   */
    WL_PROF_RESTRICT_FINE = 3,   /* residual + restriction, fine level        */
    WL_PROF_MOMENTUM = 4,        /* convection-diffusion stage update         */
    WL_PROF_DIVERGENCE = 5,      /* projection right-hand side                */
    WL_PROF_PROJECT = 6,         /* pressure-gradient update (+ CFL)          */
    WL_PROF_NORM_FINE = 7,       /* residual norm only, fine level            */
    WL_PROF_PAIR_FINE = 8,       /* two sweeps fused, fine level              */
    WL_PROF_PAIR_PROLONG_FINE = 9, /* post-smoothing pair (after the
                                      prolongation), fine level            */
    WL_PROF_COUNT = 10
};

/* Enable event timing for the kernels in mask (bit k = kernel k); 0 turns it
 * off.  Events are recorded on the stream each kernel is launched on. */
wl_status wl_profile_enable(unsigned mask);
/* Clear accumulated timings. */
wl_status wl_profile_reset(void);
/* Synchronise the recorded events and return the total time in ms, the
 * number of timed launches and the grid cells each launch covered (last). */
wl_status wl_profile_read(int kernel, double* total_ms, long long* launches,
                          long long* cells_per_launch);

/* ---- Misc --------------------------------------------------------------- */

/* Message of the last error on this thread ("" when none). */
const char* wl_last_error(void);

/* Library version string. */
const char* wl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WL_H */
