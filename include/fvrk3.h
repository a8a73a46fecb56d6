/*
 * fvrk3.h -- C ABI of the MI355X (gfx950) finite-volume RHS / TVD-RK3 library.
 *
 * The library evaluates the explicit finite-volume right-hand side of the
 * compressible Navier-Stokes equations on a uniform Cartesian grid
 * (arXiv:2402.05193, Sec. 3.2 Eq. (FVD)) and the third-order TVD Runge-Kutta
 * update that consumes it (Sec. 3.4), for three models:
 *   FV_EULER  single-phase inviscid       (Sec. 2.1, 3.5)
 *   FV_NS     single-phase viscous        (Sec. 2.1 dissipative fluxes, Sec. 2.5)
 *   FV_DIM    five-equation diffuse-interface two-phase model (Sec. 2.3, 3.7)
 * with WENO5-Z or TENO6-A reconstruction of primitive or characteristic
 * variables, the HLLC flux, 4th-order central viscous fluxes and, optionally
 * (default for FV_DIM), the interpolation and flux positivity limiters of
 * Sec. 3.3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays: device pointers to contiguous structure-of-arrays storage
 *   [ncomp][nz][ny][nx], x fastest, element type cfg->dtype (double or
 *   float), base address aligned to 16 bytes.  ncomp = 5 for FV_EULER/FV_NS
 *   (U = rho, rho u, rho v, rho w, E; W = rho, u, v, w, p) and 7 for FV_DIM
 *   (U = a1 rho1, a2 rho2, rho u, rho v, rho w, E, a1;
 *    W = a1 rho1, a2 rho2, u, v, w, p, a1), the state vectors of Sec. 2.1 / 2.3.
 *   Only interior cells are stored; boundary conditions are applied while
 *   the kernels read neighbours.
 * Ownership: the caller owns every buffer (states, workspace, outputs).  The
 *   library allocates no device memory and keeps no device state.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   All calls are asynchronous and stream-ordered unless stated otherwise.
 * Errors: every function returns FV_OK (0) or a negative fv_status.  Nothing
 *   throws or aborts.  last_error() returns a thread-local message describing
 *   the last failure of the calling thread.
 * Re-entrancy: calls on different streams with disjoint buffers may run
 *   concurrently.
 */
#ifndef FVRK3_H
#define FVRK3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FV_ABI_VERSION 3

enum fv_model { FV_EULER = 0, FV_NS = 1, FV_DIM = 2 };
enum fv_dtype { FV_F64 = 0, FV_F32 = 1 };
/* Boundary conditions by index mapping (Sec. 3.1): periodic wrap, zero
 * gradient (first-order extrapolation), symmetry (mirror with the normal
 * momentum negated; needs at least 3 cells along that axis).  Periodic must
 * be set on both faces of an axis. */
enum fv_bc { FV_PERIODIC = 0, FV_ZERO_GRADIENT = 1, FV_SYMMETRY = 2 };

enum fv_status {
    FV_OK = 0,
    FV_EINVAL = -1,        /* invalid configuration or argument value      */
    FV_ENULL = -2,         /* a required pointer is NULL                    */
    FV_EALIGN = -3,        /* a device pointer is not 16-byte aligned       */
    FV_EUNSUPPORTED = -4,  /* valid request that the library does not serve */
    FV_EHIP = -5,          /* a HIP runtime call or kernel launch failed    */
    FV_EINADMISSIBLE = -6, /* check_state found an inadmissible cell        */
    FV_ENONFINITE = -7     /* check_state found a NaN or Inf                */
};

/* Initial conditions served by init_state (parameters in `params`). */
enum fv_case {
    FV_CASE_UNIFORM = 0, /* params: the primitive state W (ncomp values)                    */
    FV_CASE_TGV = 1,     /* Taylor-Green vortex on [0,2pi)^3 (cfg dx = 2pi/nx ...):
                            params: Ma, rho0, noise amplitude (seeded +-noise on u, v, w)   */
    FV_CASE_RIEMANN = 2, /* planar two-state problem: params: axis, x0 (fraction of the
                            domain along axis), W_left (ncomp), W_right (ncomp)            */
    FV_CASE_SBI = 3,     /* shock-bubble: params: x_shock, x_c, y_c, z_c, radius, eps_alpha,
                            W_postshock_air (rho, u, p), W_air (rho, p), rho_bubble;
                            fluid 1 = bubble gas, fluid 2 = air; coordinates in metres     */
    FV_CASE_GAUSS_WAVE = 4, /* the convergence test's density wave (Sec. 5.1): params: axis,
                            u, p; rho = 1 + 5 exp(-200 (s - 0.5)^2) + 5 exp(-200 (s - 1.5)^2)
                            along the axis (s = cell coordinate from 0; [0, 2) with
                            periodic ends for the paper's test) as exact cell averages,
                            velocity u along the axis, pressure p; single phase            */
    FV_CASE_ISENTROPIC_VORTEX = 5 /* Shu's isentropic vortex, z-invariant: params: strength,
                            x_c, y_c, u_inf, v_inf; rho_inf = p_inf = 1, T = p / rho,
                            u = u_inf - strength/(2 pi) exp((1 - r^2)/2) (y - y_c),
                            v = v_inf + strength/(2 pi) exp((1 - r^2)/2) (x - x_c),
                            T = 1 - (gamma-1) strength^2/(8 gamma pi^2) exp(1 - r^2),
                            rho = T^(1/(gamma-1)); conservative cell averages by 5 x 5
                            Gauss-Legendre points; single phase                            */
};

/* Problem description, passed by pointer to every call and copied into
 * kernel arguments.  Zero tolerances select the per-precision defaults of
 * Sec. 3.3 (FP64: eps_rho 1e-12, eps_rhoc2 1e-10, eps_alpha 1e-12;
 * FP32: 1e-10, 1e-8, 1e-10); weno_eps 0 selects 1e-40 (FP64) / 1e-30 (FP32). */
typedef struct fv_config {
    int32_t abi_version; /* must be FV_ABI_VERSION                         */
    int32_t nx, ny, nz;  /* interior cells, each >= 1                      */
    int32_t model;       /* fv_model                                       */
    int32_t dtype;       /* fv_dtype of every array                        */
    int32_t bc[6];       /* fv_bc for x-, x+, y-, y+, z-, z+               */
    int32_t positivity;  /* 1: limiters on, 0: off, -1: default (on for DIM) */
    int32_t recon;       /* reconstruction variables: 0 primitive (Sec. 3.2 as read
                            here), 1 characteristic (Sec. 3.2 steps 1-4, frozen face
                            state = mean of the two cells, appendix eigenvectors);
                            the adjoint takes 0 only                            */
    double dx, dy, dz;   /* uniform cell sizes, > 0                        */
    double gamma1, pinf1;/* stiffened gas of fluid 1 (the only fluid for EULER/NS) */
    double gamma2, pinf2;/* stiffened gas of fluid 2 (FV_DIM)              */
    double mu;           /* constant dynamic viscosity (FV_NS), >= 0       */
    double prandtl;      /* Prandtl number (FV_NS), > 0                    */
    double eps_rho, eps_rhoc2, eps_alpha; /* limiter tolerances (0: default) */
    double weno_eps;     /* WENO-Z epsilon (0: default)                    */
    double cfl;          /* CFL number used by advance/compute_dt, > 0     */
    int32_t visc_law;    /* dynamic viscosity (Sec. 2.5), FV_NS only: 0 constant mu;
                            1 power law mu (T/T_ref)^0.7; 2 Sutherland
                            mu (T/T_ref)^1.5 (T_ref + C)/(T + C); mu = the value at
                            T_ref.  Faces use the temperature interpolated to the face;
                            conductivity from the constant Prandtl number          */
    int32_t scheme;      /* reconstruction scheme (Sec. 3.2 step 3): 0 WENO5-Z; 1 TENO6-A
                            (stencils of the reconstruction schematic, Jiang-Shu
                            indicators, adaptive cut-off; the six cells i-2..i+3
                            of a face for both states); the adjoint takes 0 only */
    double T_ref;        /* reference temperature of the law, > 0 when visc_law != 0 */
    double sutherland;   /* Sutherland's constant C, >= 0                  */
    double gas_R;        /* specific gas constant in T = p / (rho R); 0 selects 1 */
    int32_t visc_order;  /* central viscous stencils (FV_NS): 0 or 4 -- 4th order inside
                            the fused stage; 6 -- 6th order (the paper's single-phase
                            simulation setup), computed by separate passes into the workspace
                            (rhs_ws, rk3_stage3_cfl, rk3_step, advance; not rhs,
                            rk3_stage or batches)                               */
    int32_t thinc;       /* FV_DIM: 1 replaces the volume fraction and partial densities of
                            the face states of interface cells by the THINC profile
                            (Sec. 3.2; eps 1e-4, beta 1; profile centre from the cell
                            average); 0 off                                     */
} fv_config;

/* Result of check_state. */
typedef struct fv_report {
    int32_t status;         /* FV_OK, FV_ENONFINITE or FV_EINADMISSIBLE    */
    int32_t bad_count_clamped; /* number of bad cells, saturated at 2^31-1  */
    int64_t first_bad_cell; /* smallest flat index of a bad cell, -1 if none */
} fv_report;

/* Number of components for cfg->model (5 or 7), or a negative status. */
int32_t fv_ncomp(const fv_config* cfg);

/* Bytes of workspace needed by rhs_ws / rk3_step / advance / compute_dt /
 * check_state: two extra state arrays plus 256 bytes of device scalars; with
 * visc_order 6 also the viscous passes' fields, 13 (nx+6)(ny+6)(nz+6) + 4 nx ny nz
 * values (each block aligned to 256 bytes). */
int workspace_bytes(const fv_config* cfg, size_t* out);

/* Analytic initial condition written as conservative variables U
 * (compute_initial_condition of the paper's API, introduction of Sec. 6): values at
 * cell centres, except the cell averages of FV_CASE_GAUSS_WAVE and
 * FV_CASE_ISENTROPIC_VORTEX.
 * Seeded noise uses splitmix64 keyed by (seed, 3*flat_index + component). */
int init_state(const fv_config* cfg, int32_t case_id, const double* params, int32_t nparams,
               uint64_t seed, void* U, void* stream);

/* U = L_{W->U}(W) (Sec. 2.1/2.3 state vectors, Sec. 2.4 EOS). */
int prim_to_cons(const fv_config* cfg, const void* W, void* U, void* stream);

/* W = L_{U->W}(U). */
int cons_to_prim(const fv_config* cfg, const void* U, void* W, void* stream);

/* R = R_NSE(U), Eq. (FVD) plus the DIM volume-fraction source (Sec. 3.7).
 * dt is used only by the flux limiter's admissibility test (ignored when the
 * limiters are off).  U and R must not overlap. */
int rhs(const fv_config* cfg, const void* U, void* R, double dt, void* stream);

/* rhs with a workspace of workspace_bytes(cfg) bytes (required for
 * visc_order 6, whose viscous passes keep their intermediate fields there;
 * otherwise the same as rhs).  The workspace contents are overwritten. */
int rhs_ws(const fv_config* cfg, const void* U, void* R, double dt, void* ws, void* stream);

/* Workgroups of the problem's share of a batched stage launch; a measure of how
 * much of the GPU the problem fills (each CU holds two FP64 or three FP32 stage
 * workgroups at a time).  A single-problem launch has as many, except that the
 * five-equation model may take fewer, longer z chunks alone when they still give
 * every CU its full share. */
int stage_workgroups(const fv_config* cfg, int32_t* out);

/* Bytes of the limiter decision record of rhs_flags: one byte per cell face,
 * (nx+1) ny nz + nx (ny+1) nz + nx ny (nz+1). */
int limiter_flag_bytes(const fv_config* cfg, size_t* out);

/* rhs plus the decisions of the positivity limiters of Sec. 3.3 at every face
 * (the interpolation limiter's switch of each reconstructed state to its cell
 * state, item 1, and the flux limiter's switch to the first-order HLLC flux,
 * item 2).  R is the same as rhs (and rhs_ws) computes.
 * flags: device buffer of limiter_flag_bytes(cfg) bytes, written in full: the
 *   x faces first, [k][j][i] with i = 0..nx the face between cells i-1 and i
 *   (i fastest), then the y faces [k][j = 0..ny][i], then the z faces
 *   [k = 0..nz][j][i].  Bit 0: the left state was replaced, bit 1: the right
 *   state, bit 2: the flux limiter tripped.  With the limiters off every byte is 0.
 * ws: workspace of workspace_bytes(cfg) for visc_order 6 (NULL otherwise). */
int rhs_flags(const fv_config* cfg, const void* U, void* R, double dt, uint8_t* flags, void* ws, void* stream);

/* One TVD-RK3 stage (Sec. 3.4), the benchmarked unit:
 *   stage 1: Uout = Un + dt R(Un)                        (Uk must equal Un)
 *   stage 2: Uout = 3/4 Un + 1/4 Uk + 1/4 dt R(Uk)
 *   stage 3: Uout = 1/3 Un + 2/3 Uk + 2/3 dt R(Uk)
 * dt_dev: optional device pointer to a double holding dt (then `dt` is
 * ignored).  Uout must not overlap Uk; in stage 3 Uout may equal Un. */
int rk3_stage(const fv_config* cfg, int32_t stage, const void* Un, const void* Uk, void* Uout,
              double dt, const double* dt_dev, void* stream);

/* Stage 3 of rk3_stage fused with the CFL reduction of its output:
 * Uout = 1/3 Un + 2/3 Uk + 2/3 dt R(Uk) with dt = *dt_dev, then
 * *dt_next = cfg->cfl * min(min_d dx_d / (|u_d| + c), (3/14) rho dx_min^2 / mu)
 * over Uout (the time step of the next step, as compute_dt would give it,
 * without another pass over the state).  dt_next may equal dt_dev.  ws: the
 * workspace of workspace_bytes() (its scalar area holds the reduction). */
int rk3_stage3_cfl(const fv_config* cfg, const void* Un, const void* Uk, void* Uout, const double* dt_dev,
                   double* dt_next, void* ws, void* stream);

/* One full TVD-RK3 step in place: U <- I_RK3(U, R, dt).  ws: workspace of
 * workspace_bytes(). */
int rk3_step(const fv_config* cfg, void* U, double dt, void* ws, void* stream);

/* dt = cfg->cfl * min(min_d dx_d / (|u_d| + c), (3/14) rho dx_min^2 / mu),
 * written to the device double *dt_dev.  ws as for rk3_step. */
int compute_dt(const fv_config* cfg, const void* U, double* dt_dev, void* ws, void* stream);

/* Advance nsteps TVD-RK3 steps in place (the feedforward of the paper's API,
 * introduction of Sec. 6).  dt > 0: fixed step; dt <= 0: CFL step recomputed on the device
 * before every step.  t_inout (host, optional): incremented by the simulated
 * time; the only host synchronisation of this call happens when it is given. */
int advance(const fv_config* cfg, void* U, int32_t nsteps, double dt, double* t_inout, void* ws,
            void* stream);

/* Size of the fixed device array that advance_noalloc uses as its workspace
 * (one per device, held until the process ends): 64 MiB, e.g. a 64^3 FP64
 * single-phase (42 MB) or five-equation problem (59 MB). */
#define FV_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* advance without any device allocation, for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same TVD-RK3 steps as advance(cfg, U, nsteps, dt, NULL,
 * ws, stream), bit for bit, with ws taken from the library's fixed array of
 * FV_NOALLOC_SCRATCH_BYTES bytes on the current device instead of the caller's
 * workspace.  Problems whose workspace_bytes(cfg) exceed it are rejected with
 * FV_EINVAL.  No simulated-time read-back (t_inout of advance).  Every call on a
 * device shares that device's array: calls that overlap in time on one device
 * (different streams or host threads) race and must not be issued; calls in one
 * stream order are safe.  The first call on a device looks up the array's
 * address there (once per device). */
int advance_noalloc(const fv_config* cfg, void* U, int32_t nsteps, double dt, void* stream);

/* Discrete adjoint (the reverse-mode derivative the paper takes by automatic
 * differentiation of the solver, Sec. 6): the vector-Jacobian product
 *   Ubar = (dR/dU)^T Rbar
 * of rhs() at U, overwriting Ubar.  Covers the single-phase Euler model in
 * FP64 with the positivity limiters off (other configurations return
 * FV_EUNSUPPORTED); all boundary conditions.  Non-differentiable points take
 * |x|' = sgn(x) with sgn(0) = 0, an even split at ties of min/max, and a zero
 * derivative of the HLLC upwind switch.  Contributions are accumulated with
 * atomic adds: reproducible to round-off, not bitwise.  ws is unused (may be
 * NULL).  Ubar must not overlap U or Rbar.
 * Conditioning: at a constant reconstruction stencil (uniform regions,
 * zero-gradient halos) the smoothness indicators are round-off and the
 * derivative of the WENO-Z weights scales like 1/(beta + weno_eps)^2; with the
 * default epsilon 1e-40 it is then set by rounding.  Reproducible gradients of
 * such fields need a larger epsilon (e.g. 1e-6, the same in the forward). */
int rhs_adjoint(const fv_config* cfg, const void* U, const void* Rbar, void* Ubar, void* ws,
                void* stream);

/* Bytes of workspace for rk3_step_adjoint: five state arrays. */
int adjoint_workspace_bytes(const fv_config* cfg, size_t* out);

/* Reverse sweep of one TVD-RK3 step at a fixed dt (Sec. 3.4): on entry Ubar
 * holds the cotangent of U^{n+1} = I_RK3(U^n); on return the cotangent of U^n
 * (dt is a constant of the step, not differentiated).  The stage states are
 * recomputed from Un.  aws: adjoint_workspace_bytes() of device memory.  Same
 * coverage as rhs_adjoint. */
int rk3_step_adjoint(const fv_config* cfg, const void* Un, void* Ubar, double dt, void* aws, void* stream);

/* rk3_step_adjoint with the step's stage states given instead of recomputed
 * (Sec. 3.4): U1 = U^(1) and U2 = U^(2) of the forward step from Un at the same
 * dt, as rk3_stage writes them (stage 1 from Un, stage 2 from Un and U1), device
 * arrays of the state layout, read only.  Ubar (in place, as for
 * rk3_step_adjoint) must not overlap Un, U1 or U2.  aws: adjoint_workspace_bytes()
 * of device memory.  Same coverage and errors as rk3_step_adjoint. */
int rk3_step_adjoint_stages(const fv_config* cfg, const void* Un, const void* U1, const void* U2, void* Ubar,
                            double dt, void* aws, void* stream);

/* Scan U for NaN/Inf and for cells outside the admissible set of Sec. 3.3
 * (rho > 0 and rho c^2 > 0; DIM: 0 <= a1 <= 1, a_k rho_k > 0).  Synchronises
 * the stream.  Returns the status also stored in out->status. */
int check_state(const fv_config* cfg, const void* U, void* ws, fv_report* out, void* stream);

/* Simulated time accumulated in a workspace by advance (CFL mode, when
 * t_inout is given) or by the batched steps below, copied to the host double
 * *t.  Synchronises the stream. */
int workspace_time(const fv_config* cfg, const void* ws, double* t, void* stream);

/* ---------------------------------------------------------------------------
 * Batched time stepping of many independent problems (continuous batching).
 *
 * Each member is one problem: its fv_config, its state U and its workspace ws
 * (workspace_bytes(cfg), exactly as for advance).  Members may differ in grid,
 * model, precision, boundary conditions, parameters and options (reconstruction
 * variables and scheme, THINC, viscosity law; not visc_order 6, which needs its
 * separate passes).  Every RK stage of a batched step is one launch per group of
 * members sharing (model, precision, limiter setting, reconstruction variables and
 * scheme, viscosity law or THINC on/off), at most 16 groups per batch, whose
 * workgroups are spread over the group's members through a device table, so
 * small problems fill the GPU together.  Time stepping is in CFL mode: each
 * member keeps its own dt, recomputed on the device from its own state (the
 * reduction fused into its third stage), and its own simulated time.  A
 * member's arithmetic does not depend on the other members: its result is
 * bitwise that of advance(cfg, U, nsteps, 0, ...) run alone.
 * ------------------------------------------------------------------------- */
typedef struct fv_batch fv_batch; /* opaque host-side handle */

/* Device bytes of the request table of a batch of up to `capacity` members. */
int batch_table_bytes(int32_t capacity, size_t* out);

/* Create a batch handle.  table: caller-owned device buffer of at least
 * batch_table_bytes(capacity) bytes, 256-byte aligned, used only by this
 * handle.  The handle allocates pinned host staging memory (no device memory). */
int batch_create(int32_t capacity, void* table, size_t table_bytes, fv_batch** out);

/* Release the handle (waits for its pending table uploads). */
int batch_destroy(fv_batch* b);

/* Set the members: n <= capacity problems, arrays of n configs, states and
 * workspaces.  fresh (optional, n flags): members whose time stepping starts
 * now: their first dt is computed from U and their simulated time set to 0.
 * The table upload is stream-ordered: work enqueued earlier still runs on the
 * previous membership.  Captured graphs stay valid (they read the membership
 * from the table).  FV_EUNSUPPORTED for a member with visc_order 6; FV_EINVAL when
 * the members form more than 16 groups. */
int batch_set(fv_batch* b, int32_t n, const fv_config* cfgs, void* const* U, void* const* ws, const int32_t* fresh,
              void* stream);

/* nsteps TVD-RK3 steps (Sec. 3.4) of every member, CFL mode.  A group with a
 * single member runs the single-problem stage kernel with that member's
 * arguments (the same arithmetic). */
int batch_step(fv_batch* b, int32_t nsteps, void* stream);

/* As batch_step, through a HIP graph of nsteps steps.  The graph's kernels read
 * the membership from the device table, and their grids are the groups'
 * workgroup counts rounded up to a multiple of an eighth of their power-of-two
 * floor (spare workgroups return at once), so one captured graph serves every
 * membership with the same groups and rounded grids:
 * graphs are cached per batch under that key, nsteps and the stream (at most 16,
 * least recently used dropped) and captured on a miss.  stream must not be the
 * default (NULL) stream; the graph runs on the stream it was captured on.  When
 * every group has a single member the steps run as batch_step (no graph). */
int batch_step_graph(fv_batch* b, int32_t nsteps, void* stream);

/* Number of step graphs the batch holds (diagnostics). */
int batch_graph_count(const fv_batch* b);

/* Thread-local message of the last failure ("" if none). */
const char* last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FVRK3_H */
