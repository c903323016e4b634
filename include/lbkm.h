/*
 * lbkm.h -- C ABI of the MI355X (gfx950) implementation of the two-dimensional
 * multiple-relaxation-time lattice Boltzmann kinetic model for combustion
 * (Xu, Lin, Zhang, Li, arXiv:1411.6697).
 *
 * One time step advances the 24 discrete distribution functions f_i of the
 * D2V24 model and the reaction progress lambda on a cell-centred Nx x Ny grid:
 *
 *   f_i^{n+1} = f_i^n + dt [ -v_i . grad_NND f_i
 *                            - M^-1_il ( R_l (f_hat_l - f_hat^eq_l) - A_hat_l )
 *                            + C_i ]                       (Sec. II, Eq. Boltzmann_chemical)
 *   lambda^{n+1} = lambda^n + dlambda_chem - dt u . grad_NND lambda
 *                                                           (Sec. II, Eq. lambda_equation)
 *
 * with f_hat = M f (rows m_1..m_24 of Sec. II), f_hat^eq the 24 closed forms of
 * Sec. II (entries 14 and 16 carry the factor T that Eq. moment7 requires),
 * A_hat_8, A_hat_9 of Eqs. ArtificialA8/ArtificialA9 entering with the
 * moment-space sign of Eq. CE_LB, C_i of Eq. C_i with F = dlambda_chem / dt,
 * the Cochran rate integrated exactly over the step with p frozen, and the NND
 * scheme (Zhang 1988, flux-split minmod) upwinded by the sign of v_i (of u for
 * lambda).  Time integration is forward Euler.  Delta_k = f_hat_k - f_hat^eq_k
 * (Sec. VI) with Delta_1..4 = 0.
 *
 * Conventions
 *  - Every function returns lbkm_status; no exception crosses the ABI.  A
 *    human-readable message for the last failure on a context is available
 *    from lbkm_last_error (valid until the next call on that context).
 *  - All field pointers are DEVICE pointers to float64 data unless stated
 *    otherwise.  The caller owns every field and state buffer and keeps it
 *    alive while bound; the library never frees them.  The library owns only
 *    its constant tables and reduction scratch (freed by lbkm_destroy).
 *  - Layouts: a scalar field is [ny][nx] dense (row pitch nx) unless a
 *    pitch is given.  The distribution buffers are structure-of-arrays
 *    f[24][ny][pitch] with pitch >= nx, velocity i = 8 g + d in group
 *    g = 0 (v_a), 1 (v_b), 2 (v_c) and unit direction d of
 *    (1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).  lambda buffers
 *    are [ny][pitch].
 *  - Work is enqueued on the HIP stream given at creation (NULL = the null
 *    stream).  Functions that return values in host memory synchronise that
 *    stream; all others are asynchronous.
 *  - A context is not thread-safe; calls on one context must be serialised.
 */
#ifndef LBKM_H
#define LBKM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbkm_ctx lbkm_ctx;

typedef enum {
    LBKM_OK = 0,
    LBKM_EINVAL = -1,      /* invalid argument or parameter                         */
    LBKM_ESINGULAR = -2,   /* moment matrix M singular or too ill-conditioned       */
    LBKM_ENOMEM = -3,      /* device or host allocation failed                      */
    LBKM_EDEVICE = -4,     /* HIP runtime error (message holds the HIP error string) */
    LBKM_ESTATE = -5,      /* call out of order (e.g. step before set_params)       */
    LBKM_ENONFINITE = -6   /* lbkm_check found NaN/Inf, rho <= 0 or T <= 0          */
} lbkm_status;

typedef enum { LBKM_BC_PERIODIC = 0, LBKM_BC_OUTFLOW = 1 } lbkm_bc;

/* D2V24 velocity model (Sec. II): group speeds and internal-dof parameters. */
typedef struct { double va, vb, vc, eta_a, eta_b, eta_c; } lbkm_dvm;

/* Grid and time step.  Ghost cells are implicit: periodic wrap, or
 * zero-gradient outflow (both ghosts copy the edge cell). */
typedef struct {
    int32_t nx, ny;
    double dx, dy, dt;
    int32_t bc_x, bc_y;           /* lbkm_bc */
    lbkm_dvm dvm;
} lbkm_grid;

/* Cochran rate of Eq. lambda_equation: d lambda/dt = omega1 p^m (1-lambda)
 * + omega2 p^n lambda (1-lambda), active only where T > T_ig. */
typedef struct { double omega1, omega2, m, n, T_ig; } lbkm_rates;

/* ---- single-grid context ------------------------------------------------ */

/* Create a context for one grid; validates the grid and the velocity model and
 * builds M and its block inverse on the host (LBKM_ESINGULAR if M is singular
 * or its condition number exceeds 1e12).  hip_stream is a hipStream_t or NULL.
 * No device work happens here (device tables are allocated by lbkm_bind_buffers).
 * The kernels address the 24 planes of one state with 32-bit byte offsets, so
 * 24 * nx * ny doubles must stay within 4 GiB (about 22.3 million cells; a larger
 * domain is split into several grids): LBKM_EINVAL otherwise.
 * On failure *out may still hold a context for lbkm_last_error; destroy it. */
lbkm_status lbkm_create(const lbkm_grid* grid, void* hip_stream, lbkm_ctx** out);

/* Bind caller-owned device buffers: f_a, f_b of 24*ny*pitch doubles and
 * lam_a, lam_b of ny*pitch doubles (pitch >= nx elements).  The state lives in
 * the "a" buffers after init_fields/set_state and ping-pongs between a and b.
 * LBKM_EINVAL for NULL or equal buffers, pitch < nx, or 24*ny*pitch doubles
 * beyond 4 GiB (checked before any device work). */
lbkm_status lbkm_bind_buffers(lbkm_ctx* ctx, double* f_a, double* f_b,
                              double* lam_a, double* lam_b, int64_t pitch);

/* Relaxation rates and physics (Sec. II-III).  S holds R_1..R_24 (host array).
 * gamma = (D+I+2)/(D+I) gives I = 2/(gamma-1) - 2 (snapped to the nearest
 * integer when within 1e-9).  If Pr > 0 the library requires R_5 = R_6 = R_7
 * and sets R_8 = R_9 = Pr R_5 (Pr = R_kappa / R_mu, Sec. III); if Pr <= 0, S is
 * used as given.  Q is the heat release (Eq. chemical_energy).
 * LBKM_EINVAL if gamma <= 1 or I <= 0, any R_k <= 0, R_k dt >= 2 for k >= 5,
 * T_ig < 0, m or n < 0, omega1 or omega2 < 0, or a non-finite value. */
lbkm_status lbkm_set_params(lbkm_ctx* ctx, const double S[24], double gamma, double Pr,
                            double Q, const lbkm_rates* rates);

/* Initial state f = M^-1 f_hat^eq(rho, u, T) and lambda (Eq. moment12).  Inputs are
 * dense [ny][nx] device arrays.  LBKM_EINVAL is not raised for rho <= 0 or T <= 0
 * in the data (that would need a device sync); lbkm_check reports them. */
lbkm_status lbkm_init_fields(lbkm_ctx* ctx, const double* rho, const double* ux,
                             const double* uy, const double* T, const double* lambda);

/* Advance n >= 0 time steps on the bound stream (asynchronous).  One step is one launch
 * of the fused step kernel (forward Euler, Eq. Boltzmann_chemical with the readings of the
 * library), or 2 / 3 launches for the Runge-Kutta schemes of lbkm_set_time_scheme; with
 * wall sides (lbkm_set_boundary) each launch is preceded by the fill of the ghost layers.
 * The library allocates, on first need and for the life of the context, the velocity planes
 * of the modification term, the third Runge-Kutta state and the ghost layers.  On grids of
 * at most 262144 cells a call with n >= 64 replays a HIP graph of the launches of 64 steps,
 * captured once per buffer parity and launch configuration on a library stream (the same
 * kernels: results are bitwise those of n single steps).  Errors:
 * EINVAL for n < 0; ESTATE before buffers, parameters and fields are set; EDEVICE for a
 * failed launch or allocation. */
lbkm_status lbkm_step(lbkm_ctx* ctx, int64_t n);

/* Macroscopic readout rho, u_x, u_y, T, p = rho T, lambda into dense [ny][nx]
 * device arrays; any pointer may be NULL (asynchronous). */
lbkm_status lbkm_get_moments(lbkm_ctx* ctx, double* rho, double* ux, double* uy,
                             double* T, double* p, double* lambda);

/* TNE readout (Sec. VI): delta[20][ny][nx] holds Delta_5..Delta_24 and d[ny][nx]
 * holds sqrt(sum_k Delta_k^2); either may be NULL (asynchronous). */
lbkm_status lbkm_get_tne(lbkm_ctx* ctx, double* delta, double* d);

/* Deterministic grid reductions into host memory (synchronises):
 * out[0..7] = sum rho, sum rho u_x, sum rho u_y, sum E (E = f_hat_4 / 2, total energy
 * density), sum_cells sum_k Delta_k^2, (dx/ny) sum |Delta_5| (row-averaged global TNE
 * area, Sec. VI B), min lambda, max lambda. */
lbkm_status lbkm_reduce(lbkm_ctx* ctx, double out[8]);

/* Health check (synchronises): LBKM_ENONFINITE if any cell holds NaN/Inf in f or
 * lambda, rho <= 0 or T <= 0; LBKM_OK otherwise. */
lbkm_status lbkm_check(lbkm_ctx* ctx);

/* Ignition margin of the current state (synchronises): *margin (host) receives the
 * minimum of |T - T_ig| over the cells with lambda < 1, +infinity when there is none.
 * The ignition test T > T_ig (Sec. II, the rate law) is the one discontinuity of the
 * step; a margin far above rounding shows that no cell sits on it, so implementations
 * that round differently still take the same branch everywhere.  EINVAL for a NULL
 * margin; ESTATE before buffers, parameters and fields are set. */
lbkm_status lbkm_ignition_margin(lbkm_ctx* ctx, double* margin);

/* Copy the current state out to / in from caller device buffers f[24][ny][nx]
 * and lam[ny][nx] (dense, asynchronous).  set_state marks the fields as set. */
lbkm_status lbkm_get_state(lbkm_ctx* ctx, double* f, double* lam);
lbkm_status lbkm_set_state(lbkm_ctx* ctx, const double* f, const double* lam);

/* Launch shape of the step kernel: a work-group updates a tile_x x tile_y tile.  lds
 * selects the kernel: 0 collides first and then reads the stencil through the caches;
 * 1 collides first and stages each plane's tile and stencil halo in LDS; 2 streams first
 * (each input value is read once: the streamed values wait in LDS while the cell collides
 * from its centre values); 3 collides first with the tile's centre values shared in LDS
 * (the streaming reads in-tile neighbours from LDS and neighbouring lanes, and loads only
 * the halo).  Compiled shapes: (64,4,0), (256,2,0), (256,1,0), (64,4,1), (32,8,1),
 * (128,2,1), (64,4,2), (32,8,2), (128,2,2), (256,1,2), (64,4,3) (default), (128,2,3);
 * LBKM_EINVAL for any other.  Results do not depend on the launch shape (bitwise). */
lbkm_status lbkm_set_tile(lbkm_ctx* ctx, int32_t tile_x, int32_t tile_y, int32_t lds);

/* Order in which the tiles are dealt to the eight XCDs: vertical = 1 (the default) gives
 * each XCD a contiguous band of tile columns (used only when their number divides by
 * eight, else bands of tile rows), vertical = 0 a band of tile rows.  Results do not
 * depend on it. */
lbkm_status lbkm_set_tile_order(lbkm_ctx* ctx, int32_t vertical);

/* Collision form of the single-grid step (Sec. V, Eq. SRT).  tau > 0: the
 * single-relaxation-time form, -(f_i - M^-1_il f_hat^eq_l) / tau + C_i, with one
 * relaxation time tau for all 24 distribution functions and no modification term
 * (R_1..R_24 and Pr of lbkm_set_params are then unused).  tau = 0 (the state after
 * lbkm_create): the multiple-relaxation-time form of Eq. Boltzmann_chemical.  Errors:
 * EINVAL if tau < 0, not finite, or dt / tau >= 2 (forward Euler relaxation unstable);
 * ESTATE on a batched context.  lbkm_adjoint_step refuses a context in the SRT form
 * (ESTATE).  Takes effect from the next step (the constants are uploaded, and the stream
 * waited for, once buffers and parameters are set). */
lbkm_status lbkm_set_srt(lbkm_ctx* ctx, double tau);

/* Wall boundary of one side of the grid (Sec. IV C shock reflection, Sec. IV D Couette
 * flow), overriding the axis rule of lbkm_grid.bc_x / bc_y on that side.  side: 0 = x low,
 * 1 = x high, 2 = y low, 3 = y high.  The wall lies on the face between the edge cells and
 * two ghost layers whose distributions the library fills before every step (and every
 * Runge-Kutta stage) from the current state:
 *   type 0: none (the axis rule: periodic wrap or zero-gradient outflow);
 *   type 1: reflecting (specular) wall: ghost layer k holds the edge layer k with the
 *           velocities mirrored across the wall, lambda alike; no mass, energy or
 *           tangential momentum crosses it;
 *   type 2: Dirichlet: both layers hold the discrete equilibrium M^-1 f_hat^eq of
 *           state = {rho, T, u_x, u_y, lambda} (inflow, far field);
 *   type 3: non-equilibrium extrapolation: both layers hold the equilibrium at the edge
 *           cell's density and the wall's T = state[1], u = (state[2], state[3]) plus the
 *           edge cell's non-equilibrium part f - f^eq; lambda copies the edge cell.
 * state: host array of 5 doubles (used by types 2 and 3; may be NULL for 0 and 1).  A wall
 * needs bc = LBKM_BC_OUTFLOW on its axis (the opposite side keeps that rule unless it is a
 * wall too).  With a wall the step uses the 64 x 4 shared-centre launch shape.  Errors: EINVAL
 * for a bad side, type, axis rule or state (non-finite, rho <= 0 or T <= 0), or when the
 * library-owned ghost layers (27 * 8 * max(nx, ny) doubles) would exceed 4 GiB; ESTATE on
 * a batched context.  lbkm_adjoint_step refuses a context with walls (ESTATE). */
lbkm_status lbkm_set_boundary(lbkm_ctx* ctx, int32_t side, int32_t type, const double* state);

/* Time integration of the single-grid step.  order = 1: forward Euler (the default, the
 * reading of Eq. Boltzmann_chemical's time derivative used throughout); order = 2: the
 * two-stage and order = 3: the three-stage strong-stability-preserving Runge-Kutta schemes
 * of Shu and Osher (1988), whose stages are forward-Euler updates of the whole right-hand
 * side (streaming, collision, C_i, and the lambda equation with its Cochran increment as
 * the rate times dt) combined with f^n:
 *   RK2: g1 = E(f^n);  f^{n+1} = f^n/2 + E(g1)/2
 *   RK3: g1 = E(f^n);  g2 = 3/4 f^n + 1/4 E(g1);  f^{n+1} = 1/3 f^n + 2/3 E(g2).
 * One lbkm_step advances one full step (2 or 3 kernel launches).  RK3 allocates a third
 * state (library-owned, freed by lbkm_destroy).  Errors: EINVAL for another order; ESTATE on
 * a batched context.  lbkm_adjoint_step refuses order != 1 (ESTATE). */
lbkm_status lbkm_set_time_scheme(lbkm_ctx* ctx, int32_t order);

/* Autotuner of the launch shape: times every compiled (tile, lds) shape in both tile
 * orders for a few steps from the current state (two passes, the better trial of each
 * candidate counts), keeps the fastest, and restores the state and the step count (the
 * trial steps run on the bound buffers; a temporary copy of the state is allocated).
 * Row bands (vertical = 0) must be faster than column bands by more than 2 % to be kept:
 * they give each XCD a band of rows, so work that later gathers in some rows (a layer
 * that ignites) would load some XCDs more than others, which the trial cannot see.  With wall sides there is one shape (64 x 4, shared centres) and
 * only the two tile orders are timed.  Needs parameters and fields.  choice (host, 4 ints, may be NULL)
 * receives tile_x, tile_y, lds, vertical.  Synchronous. */
lbkm_status lbkm_autotune(lbkm_ctx* ctx, int32_t* choice);

/* Host copies of the dense 24x24 moment matrix M (row k = moment m_{k+1}, column i =
 * velocity i) and of M^-1, both row-major, reassembled from the symmetry blocks the
 * kernels use; *cond (may be NULL) receives ||M||_inf ||M^-1||_inf.  Needs no device. */
lbkm_status lbkm_get_matrices(lbkm_ctx* ctx, double* M, double* Minv, double* cond);

/* Number of steps taken since init_fields / set_state. */
lbkm_status lbkm_get_step_count(lbkm_ctx* ctx, int64_t* out);

/* Discrete adjoint of one step (the transpose of the step's Jacobian).
 * Given the level-n state (f_n [24][ny][nx], lam_n [ny][nx], dense device arrays)
 * and the adjoint of the level-(n+1) state (af_np1, alam_np1, same layout), write
 * the adjoint of the level-n state into af_n, alam_n and ADD this step's parameter
 * gradient contributions to grad_params (device array of 27 doubles:
 * d/dR_1..R_24, d/dQ, d/domega1, d/domega2).  R_8, R_9 are treated as independent
 * parameters.  Asynchronous.  Branches (minmod selections, the ignition test)
 * are frozen at the level-n values. */
lbkm_status lbkm_adjoint_step(lbkm_ctx* ctx, const double* f_n, const double* lam_n,
                              const double* af_np1, const double* alam_np1,
                              double* af_n, double* alam_n, double* grad_params);

/* Adjoint of lbkm_init_fields: given a_f = dL/df (dense [24][ny][nx]) and the
 * initial macroscopic fields, write dL/d(rho, u_x, u_y, T) (dense [ny][nx]).
 * Asynchronous. */
lbkm_status lbkm_adjoint_init(lbkm_ctx* ctx, const double* rho, const double* ux,
                              const double* uy, const double* T, const double* af,
                              double* arho, double* aux, double* auy, double* aT);

/* Loss L = sum_cells sum_{k=5..24} Delta_k^2 of a dense state f[24][ny][nx]
 * (into *loss_dev, device) and its gradient dL/df into grad_f (dense, may be
 * NULL).  Asynchronous. */
lbkm_status lbkm_tne_loss(lbkm_ctx* ctx, const double* f, double* loss_dev, double* grad_f);

/* lbkm_tne_loss for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): the same kernels and the same result, bitwise, but the
 * per-work-group partial sums live in a fixed library array in device memory (512 KiB per
 * GPU, held until the process ends) instead of the context's lazily allocated adjoint
 * scratch, and the call makes no hipMalloc/hipFree or other allocating call.  Arguments,
 * layout and ownership as lbkm_tne_loss; asynchronous on the context's stream.  Errors: as
 * lbkm_tne_loss, plus LBKM_EINVAL when ceil(nx/256) * ny > 65536 (more partial sums than
 * the array holds).  Every call on one GPU shares that array: calls that overlap in time on
 * one GPU (other streams, other threads) race and must be ordered by the caller. */
lbkm_status lbkm_tne_loss_noalloc(lbkm_ctx* ctx, const double* f, double* loss_dev, double* grad_f);

/* Plain streaming copy of n doubles src -> dst (device pointers, 16-byte aligned) on
 * hip_stream; a bandwidth reference for the step kernel's roofline (asynchronous). */
lbkm_status lbkm_copy_kernel(const double* src, double* dst, int64_t n, void* hip_stream);

const char* lbkm_last_error(const lbkm_ctx* ctx);
lbkm_status lbkm_destroy(lbkm_ctx* ctx);

/* ---- batched 1D instances ------------------------------------------------ */
/* Many independent 1D runs of ragged lengths nx[k] (Ny = 1, zero-gradient outflow at
 * both ends, as the 1D problems of Sec. IV), sharing dx, dt, the velocity model
 * (Sec. III), gamma, Q and the rate law (Eq. for F, Sec. II), each with its own
 * R_1..R_24 (and Prandtl number).  The library owns the packed state: f[24][P] and
 * lambda[P], P = sum(nx) rounded up to 64, instances back to back.  Two launch modes
 * (lbkm_batch_set_launch, lbkm_batch_autotune), with bitwise identical results:
 *  - persistent (the default, 2 work-groups per CU): one lbkm_batch_step call replays a
 *    captured HIP graph holding one kernel launch that advances every instance n steps;
 *    neighbouring work-groups synchronise through per-work-group step counters, every
 *    wait is bounded, and a wait that runs out (work-groups not co-resident) sets a
 *    sticky error that lbkm_batch_status reports;
 *  - one launch per step: each step is one launch over all packed cells (64-cell waves,
 *    each taking the instances it overlaps one at a time), replayed from captured graphs
 *    of 64 launches and one of the remainder; no waits, no co-residency needed.
 * Calls on one context are ordered on its stream; two contexts may run concurrently.
 * Errors: LBKM_EINVAL for bad sizes or rates (checked per instance, message names it),
 * LBKM_ESTATE for calls out of order, LBKM_EDEVICE for HIP failures. */

/* n_inst >= 1 instances, nx: host [n_inst], every nx[k] >= 1, sum(nx) < 2^28 and the
 * state within 4 GiB.  common supplies dx, dy, dt and the velocity model; its nx, ny,
 * bc_x and bc_y are ignored.  Allocates the state on the current device. */
lbkm_status lbkm_batch_create(int32_t n_inst, const int32_t* nx, const lbkm_grid* common,
                              void* hip_stream, lbkm_ctx** out);

/* S: host [n_inst][24] rates; Pr: host [n_inst] or NULL (same meaning as in
 * lbkm_set_params, per instance); gamma, Q and rates shared.  Synchronous. */
lbkm_status lbkm_batch_set_params(lbkm_ctx* ctx, const double* S, const double* Pr,
                                  double gamma, double Q, const lbkm_rates* rates);

/* Initial fields, packed back to back: rho, ux, uy, T, lambda of sum(nx) doubles
 * each (device pointers, read on the stream).  Clears the step count and the error. */
lbkm_status lbkm_batch_init_fields(lbkm_ctx* ctx, const double* rho, const double* ux,
                                   const double* uy, const double* T, const double* lambda);

/* Autotuner: times a few steps of one launch per step and of the persistent kernel at
 * each candidate number of work-groups per compute unit (within the occupancy the device
 * reports) and keeps the fastest.  The state and the step count are saved and restored
 * around the trials.  If never called, the persistent kernel at two work-groups per
 * compute unit is used.  *cells_per_wg (host, may be NULL) receives the resulting cells
 * per work-group (256 with one launch per step).  Synchronous. */
lbkm_status lbkm_batch_autotune(lbkm_ctx* ctx, int32_t* cells_per_wg);

/* Fix the launch instead of autotuning: wgs_per_cu = 0 for one launch per step, 1..16 for
 * the persistent kernel with that many work-groups per compute unit.  LBKM_EINVAL outside
 * 0..16, or if the persistent kernel's occupancy does not allow that many (the shape then
 * falls back to the largest allowed).  Synchronous. */
lbkm_status lbkm_batch_set_launch(lbkm_ctx* ctx, int32_t wgs_per_cu);

/* Advance every instance n steps, 0 <= n < 2^31 (asynchronous; replays a captured
 * graph, one per buffer parity and n). */
lbkm_status lbkm_batch_step(lbkm_ctx* ctx, int64_t n);

/* Packed macroscopic readout (sum(nx) doubles each, device, NULL allowed). */
lbkm_status lbkm_batch_get_moments(lbkm_ctx* ctx, double* rho, double* ux, double* uy,
                                   double* T, double* p, double* lambda);

/* Total number of cells sum(nx) (host). */
lbkm_status lbkm_batch_total_cells(lbkm_ctx* ctx, int64_t* out);

/* Synchronises the stream; LBKM_EDEVICE if a neighbour wait of any launch since the
 * last init ran out (the results are then invalid).  wgs, wgs_per_cu (host, may be
 * NULL) receive the current launch shape: work-groups per launch, and work-groups per
 * compute unit (0 with one launch per step). */
lbkm_status lbkm_batch_status(lbkm_ctx* ctx, int32_t* wgs, int32_t* wgs_per_cu);

#ifdef __cplusplus
}
#endif

#endif /* LBKM_H */
