// C ABI of liblbkm: context management, parameter validation and kernel launches.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lbkm.h"
#include "lbkm_abi_internal.h"
#include "lbkm_kernels.h"

using namespace lbkm;

namespace lbkm {

lbkm_status fail(lbkm_ctx* ctx, lbkm_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

lbkm_status hip_fail(lbkm_ctx* ctx, hipError_t e, const char* what) {
    return fail(ctx, LBKM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// I = 2/(gamma-1) - D, snapped to an integer within 1e-9 (gamma = (D+I+2)/(D+I), Sec. III)
double internal_dof(double gamma) {
    double I = 2.0 / (gamma - 1.0) - 2.0;
    const double r = std::nearbyint(I);
    if (std::fabs(I - r) <= 1e-9) I = r;
    return I;
}

// Validate one rate set and write the physics part of the constants.  Shared by the
// single-grid and the batched contexts.
lbkm_status fill_physics(lbkm_ctx* ctx, Consts* c, const double S[24], double gamma, double Pr,
                         double Q, const lbkm_rates* rates, double dt) {
    if (!S || !rates) return fail(ctx, LBKM_EINVAL, "S and rates must not be NULL");
    if (!std::isfinite(gamma) || !(gamma > 1.0))
        return fail(ctx, LBKM_EINVAL, "gamma must be finite and > 1");
    const double I = internal_dof(gamma);
    if (!(I > 0.0)) return fail(ctx, LBKM_EINVAL, "gamma >= 2 gives I <= 0; C_i divides by I");
    double R[24];
    std::memcpy(R, S, sizeof(R));
    if (!finite_all(R, 24)) return fail(ctx, LBKM_EINVAL, "non-finite relaxation rate");
    if (std::isfinite(Pr) && Pr > 0.0) {
        if (!(R[4] == R[5] && R[5] == R[6]))
            return fail(ctx, LBKM_EINVAL, "Pr > 0 requires R_5 = R_6 = R_7");
        R[7] = R[8] = Pr * R[4];
    } else if (!std::isfinite(Pr)) {
        return fail(ctx, LBKM_EINVAL, "Pr must be finite (<= 0 means: use S as given)");
    }
    for (int k = 0; k < 24; ++k) {
        if (!(R[k] > 0.0)) return fail(ctx, LBKM_EINVAL, "R_" + std::to_string(k + 1) + " must be > 0");
        if (k >= 4 && !(R[k] * dt < 2.0))
            return fail(ctx, LBKM_EINVAL, "R_" + std::to_string(k + 1) +
                                              " dt >= 2: forward Euler relaxation is unstable");
    }
    const double vals[] = {Q, rates->omega1, rates->omega2, rates->m, rates->n, rates->T_ig};
    if (!finite_all(vals, 6)) return fail(ctx, LBKM_EINVAL, "non-finite Q or rate constant");
    if (rates->omega1 < 0 || rates->omega2 < 0 || rates->m < 0 || rates->n < 0)
        return fail(ctx, LBKM_EINVAL, "omega1, omega2, m, n must be >= 0");
    if (rates->T_ig < 0) return fail(ctx, LBKM_EINVAL, "T_ig must be >= 0");
    std::memcpy(c->R, R, sizeof(R));
    c->I = I;
    c->DI = 2.0 + I;
    c->Q = Q;
    c->w1 = rates->omega1;
    c->w2 = rates->omega2;
    c->pm = rates->m;
    c->pn = rates->n;
    c->m_is_one = rates->m == 1.0;
    c->n_is_one = rates->n == 1.0;
    c->Tig = rates->T_ig;
    c->a8c = (R[4] - R[7]) / R[4];
    c->a9c = (R[6] - R[8]) / R[6];
    c->amod = (c->a8c != 0.0 || c->a9c != 0.0) ? 1 : 0;
    c->chem = (rates->omega1 > 0.0 || rates->omega2 > 0.0) ? 1 : 0;
    return LBKM_OK;
}

lbkm_status validate_grid_common(lbkm_ctx* ctx, const lbkm_grid* g) {
    const double v[] = {g->dx, g->dy, g->dt, g->dvm.va, g->dvm.vb, g->dvm.vc,
                        g->dvm.eta_a, g->dvm.eta_b, g->dvm.eta_c};
    if (!finite_all(v, 9)) return fail(ctx, LBKM_EINVAL, "non-finite grid or velocity parameter");
    if (!(g->dx > 0 && g->dy > 0 && g->dt > 0)) return fail(ctx, LBKM_EINVAL, "dx, dy, dt must be > 0");
    if (!(g->dvm.va > 0 && g->dvm.vb > 0 && g->dvm.vc > 0))
        return fail(ctx, LBKM_EINVAL, "group speeds must be > 0");
    if (g->dvm.eta_a < 0 || g->dvm.eta_b < 0 || g->dvm.eta_c < 0)
        return fail(ctx, LBKM_EINVAL, "eta parameters must be >= 0");
    return LBKM_OK;
}

lbkm_status build_tables(lbkm_ctx* ctx, const lbkm_grid* g) {
    const double dvm[6] = {g->dvm.va, g->dvm.vb, g->dvm.vc, g->dvm.eta_a, g->dvm.eta_b, g->dvm.eta_c};
    std::memset(&ctx->h, 0, sizeof(Consts));
    if (build_moment_blocks(dvm, &ctx->h, &ctx->cond) != 0) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "moment matrix singular or ill-conditioned (cond_inf = %.3g)", ctx->cond);
        return fail(ctx, LBKM_ESINGULAR, buf);
    }
    Consts& c = ctx->h;
    c.dt = g->dt;
    c.inv_dx = 1.0 / g->dx;
    c.inv_dy = 1.0 / g->dy;
    c.half_inv_dx = 1.0 / (2.0 * g->dx);
    c.half_inv_dy = 1.0 / (2.0 * g->dy);
    for (int k = 0; k < 3; ++k) {
        c.cx[k] = c.dt * c.vg[k] * c.inv_dx;
        c.cy[k] = c.dt * c.vg[k] * c.inv_dy;
    }
    c.nx = g->nx;
    c.ny = g->ny;
    c.bc_x = g->bc_x;
    c.bc_y = g->bc_y;
    c.gL = g->nx > g->ny ? g->nx : g->ny;
    return LBKM_OK;
}

lbkm_status ensure_device_tables(lbkm_ctx* ctx) {
    if (ctx->d) return LBKM_OK;
    hipError_t e = hipMalloc((void**)&ctx->d, sizeof(Consts));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->partials, sizeof(double) * 8 * kReduceBlocks);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->out8, sizeof(double) * 8);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->flag, sizeof(int));
    if (e == hipSuccess) e = setup_noalloc_scratch();   // lbkm_tne_loss_noalloc's scratch on this device
    if (e != hipSuccess) return hip_fail(ctx, e, "allocation of library tables");
    return LBKM_OK;
}

lbkm_status upload_consts(lbkm_ctx* ctx) {
    lbkm_status st = ensure_device_tables(ctx);
    if (st != LBKM_OK) return st;
    hipError_t e = hipMemcpyAsync(ctx->d, &ctx->h, sizeof(Consts), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "upload of constants");
    e = hipStreamSynchronize(ctx->stream);   // the host copy may change before the next launch
    if (e != hipSuccess) return hip_fail(ctx, e, "upload of constants");
    return LBKM_OK;
}

}  // namespace lbkm

extern "C" {

static void drop_step_graphs(lbkm_ctx* ctx);

lbkm_status lbkm_create(const lbkm_grid* grid, void* hip_stream, lbkm_ctx** out) {
    if (!grid || !out) return LBKM_EINVAL;
    *out = nullptr;
    lbkm_ctx* ctx = new (std::nothrow) lbkm_ctx();
    if (!ctx) return LBKM_ENOMEM;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->grid = *grid;
    lbkm_status st = LBKM_OK;
    if (grid->nx < 1 || grid->ny < 1) st = fail(ctx, LBKM_EINVAL, "nx and ny must be >= 1");
    if (st == LBKM_OK && (int64_t)NV * grid->nx * grid->ny * 8 > 0xFFFFFFFFll)
        st = fail(ctx, LBKM_EINVAL, "24 nx ny doubles exceed 4 GiB (the kernels use 32-bit plane offsets)");
    if (st == LBKM_OK && ((grid->bc_x != LBKM_BC_PERIODIC && grid->bc_x != LBKM_BC_OUTFLOW) ||
                          (grid->bc_y != LBKM_BC_PERIODIC && grid->bc_y != LBKM_BC_OUTFLOW)))
        st = fail(ctx, LBKM_EINVAL, "unknown boundary condition");
    if (st == LBKM_OK) st = validate_grid_common(ctx, grid);
    if (st == LBKM_OK) st = build_tables(ctx, grid);
    if (st != LBKM_OK) {
        // keep the context so that lbkm_last_error can report; caller must destroy it
        *out = ctx;
        return st;
    }
    *out = ctx;
    return LBKM_OK;
}

lbkm_status lbkm_bind_buffers(lbkm_ctx* ctx, double* f_a, double* f_b, double* lam_a, double* lam_b,
                              int64_t pitch) {
    if (!ctx) return LBKM_EINVAL;
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "bind_buffers is not used by batched contexts");
    if (!f_a || !f_b || !lam_a || !lam_b) return fail(ctx, LBKM_EINVAL, "NULL buffer");
    if (f_a == f_b || lam_a == lam_b) return fail(ctx, LBKM_EINVAL, "the two buffers of a pair must differ");
    if (pitch < ctx->grid.nx) return fail(ctx, LBKM_EINVAL, "pitch < nx");
    if ((int64_t)NV * pitch * ctx->grid.ny * 8 > 0xFFFFFFFFll)
        return fail(ctx, LBKM_EINVAL, "24 pitch ny doubles exceed 4 GiB (the kernels use 32-bit plane offsets)");
    drop_step_graphs(ctx);             // replayed graphs hold the old buffer addresses
    ctx->f[0] = f_a;
    ctx->f[1] = f_b;
    ctx->lam[0] = lam_a;
    ctx->lam[1] = lam_b;
    ctx->cur = 0;
    ctx->pitch = pitch;
    ctx->h.pitch = pitch;
    ctx->h.plane = pitch * (int64_t)ctx->grid.ny;
    ctx->fields = false;
    ctx->u_valid = false;
    lbkm_status st = ensure_device_tables(ctx);
    if (st != LBKM_OK) return st;
    ctx->bound = true;
    return ctx->params ? upload_consts(ctx) : LBKM_OK;
}

lbkm_status lbkm_set_params(lbkm_ctx* ctx, const double S[24], double gamma, double Pr, double Q,
                            const lbkm_rates* rates) {
    if (!ctx) return LBKM_EINVAL;
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "use lbkm_batch_set_params on a batched context");
    Consts trial = ctx->h;
    lbkm_status st = fill_physics(ctx, &trial, S, gamma, Pr, Q, rates, ctx->grid.dt);
    if (st != LBKM_OK) return st;
    ctx->h = trial;
    ctx->params = true;
    return ctx->bound ? upload_consts(ctx) : LBKM_OK;
}

static lbkm_status ready(lbkm_ctx* ctx, bool need_fields) {
    if (!ctx) return LBKM_EINVAL;
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "not available on a batched context");
    if (!ctx->bound) return fail(ctx, LBKM_ESTATE, "buffers not bound");
    if (!ctx->params) return fail(ctx, LBKM_ESTATE, "parameters not set");
    if (need_fields && !ctx->fields) return fail(ctx, LBKM_ESTATE, "fields not initialised");
    return LBKM_OK;
}

lbkm_status lbkm_init_fields(lbkm_ctx* ctx, const double* rho, const double* ux, const double* uy,
                             const double* T, const double* lambda) {
    lbkm_status st = ready(ctx, false);
    if (st != LBKM_OK) return st;
    if (!rho || !ux || !uy || !T || !lambda) return fail(ctx, LBKM_EINVAL, "NULL field");
    ctx->cur = 0;
    hipError_t e = launch_init(ctx->d, ctx->grid.nx, ctx->grid.ny, rho, ux, uy, T, lambda, ctx->f[0],
                               ctx->lam[0], ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "init kernel");
    ctx->fields = true;
    ctx->steps = 0;
    ctx->u_valid = false;
    return LBKM_OK;
}

// The velocity planes that A_hat reads: allocated on first use, computed from the current
// state when they are not current (after init, set_state, a step without A_hat, ...).
static lbkm_status velocity_ready(lbkm_ctx* ctx) {
    const int64_t plane = ctx->pitch * (int64_t)ctx->grid.ny;
    if (!ctx->u[0] || ctx->u_plane != plane) {
        for (int i = 0; i < 2; ++i) {
            if (ctx->u[i]) (void)hipFree(ctx->u[i]);
            ctx->u[i] = nullptr;
        }
        for (int i = 0; i < 2; ++i) {
            hipError_t e = hipMalloc((void**)&ctx->u[i], sizeof(double) * 2 * plane);
            if (e != hipSuccess) return hip_fail(ctx, e, "allocation of the velocity planes");
        }
        ctx->u_plane = plane;
        ctx->u_valid = false;
    }
    if (!ctx->u_valid) {
        hipError_t e = launch_velocity(ctx->d, ctx->grid.nx, ctx->grid.ny, ctx->f[ctx->cur], ctx->u[ctx->cur],
                                       ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "velocity kernel");
        ctx->u_valid = true;
    }
    return LBKM_OK;
}

// The third state of SSP-RK3 (f, lambda and, with A_hat, velocity planes), library-owned.
static lbkm_status rk3_ready(lbkm_ctx* ctx, bool amod) {
    const int64_t plane = ctx->pitch * (int64_t)ctx->grid.ny;
    if (ctx->rk3_plane != plane) {
        for (double** p : {&ctx->f3, &ctx->lam3, &ctx->u3}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        ctx->rk3_plane = 0;
        hipError_t e = hipMalloc((void**)&ctx->f3, sizeof(double) * NV * plane);
        if (e == hipSuccess) e = hipMalloc((void**)&ctx->lam3, sizeof(double) * plane);
        if (e != hipSuccess) return hip_fail(ctx, e, "allocation of the third Runge-Kutta state");
        ctx->rk3_plane = plane;
    }
    if (amod && !ctx->u3) {
        hipError_t e = hipMalloc((void**)&ctx->u3, sizeof(double) * 2 * plane);
        if (e != hipSuccess) return hip_fail(ctx, e, "allocation of the third Runge-Kutta state");
    }
    return LBKM_OK;
}

static bool any_wall(const lbkm_ctx* ctx) {
    for (int k = 0; k < 4; ++k)
        if (ctx->h.wall[k] != kWallNone) return true;
    return false;
}

// ghost buffer of the wall sides, library-owned
static lbkm_status ghost_ready(lbkm_ctx* ctx) {
    const int64_t n = (int64_t)kGhostPlanes * 8 * ctx->h.gL;
    if (ctx->gbuf) return LBKM_OK;
    hipError_t e = hipMalloc((void**)&ctx->gbuf, sizeof(double) * n);
    if (e != hipSuccess) return hip_fail(ctx, e, "allocation of the ghost layers");
    return LBKM_OK;
}

// Grids up to kGraphCells cells are launch-bound: a call of at least kGraphSteps steps
// replays a captured graph of kGraphSteps steps (an even number, so a replay ends on the
// buffer parity it starts from) instead of launching every kernel from the host.
constexpr int64_t kGraphSteps = 64;
constexpr int64_t kGraphCells = 1 << 18;

static void drop_step_graphs(lbkm_ctx* ctx) {
    for (int p = 0; p < 2; ++p) {
        if (ctx->step_exec[p]) (void)hipGraphExecDestroy(ctx->step_exec[p]);
        ctx->step_exec[p] = nullptr;
        ctx->step_key[p] = -1;
    }
}

lbkm_status lbkm_step(lbkm_ctx* ctx, int64_t n) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    if (n < 0) return fail(ctx, LBKM_EINVAL, "n must be >= 0");
    if (n == 0) return LBKM_OK;
    const int flags = step_flags(ctx->h);
    const bool amod = (flags & 1) != 0;
    if (amod) {
        st = velocity_ready(ctx);
        if (st != LBKM_OK) return st;
    }
    if (ctx->rk == 3) {
        st = rk3_ready(ctx, amod);
        if (st != LBKM_OK) return st;
    }
    const bool walls = any_wall(ctx);
    if (walls) {
        st = ghost_ready(ctx);
        if (st != LBKM_OK) return st;
    }
    const int nx = ctx->grid.nx, ny = ctx->grid.ny, var = ctx->step_variant, ord = ctx->tile_order;
    double* gb = walls ? ctx->gbuf : nullptr;
    // one stage: the ghost layers of its input state (wall sides), then the step kernel
    auto stage = [&](const double* fi, double* fo, const double* li, double* lo, const double* ui, double* uo,
                     const Blend* bl) {
        if (walls) {
            hipError_t e = launch_ghost(ctx->d, nx, ny, fi, li, gb, ctx->stream);
            if (e != hipSuccess) return e;
        }
        return launch_step(ctx->d, var, flags, nx, ny, fi, fo, li, lo, ui, uo, ord, ctx->stream, bl, gb);
    };
    // `count` steps from buffer parity `a0` enqueued on stream `s`; returns the final parity
    auto issue = [&](int64_t count, int a0, hipStream_t s, int& a_end) {
        hipStream_t keep = ctx->stream;
        ctx->stream = s;
        hipError_t e = hipSuccess;
        int a = a0;
        for (int64_t k = 0; k < count && e == hipSuccess; ++k) {
            const int b = 1 - a;
            double *fa = ctx->f[a], *fb = ctx->f[b], *la = ctx->lam[a], *lb = ctx->lam[b];
            double *ua = ctx->u[a], *ub = ctx->u[b];
            // forward Euler, and the first stage of both Runge-Kutta schemes: state b = E(state a)
            e = stage(fa, fb, la, lb, ua, ub, nullptr);
            if (e == hipSuccess && ctx->rk == 2) {
                // f^{n+1} = f^n / 2 + E(g_1) / 2, written over f^n
                const Blend bl{nullptr, nullptr, 0.5, 0.5};
                e = stage(fb, fa, lb, la, ub, ua, &bl);
            } else if (e == hipSuccess && ctx->rk == 3) {
                // g_2 = 3/4 f^n + 1/4 E(g_1); f^{n+1} = 1/3 f^n + 2/3 E(g_2), written over f^n
                const Blend b2{fa, la, 0.75, 0.25};
                e = stage(fb, ctx->f3, lb, ctx->lam3, ub, ctx->u3, &b2);
                const Blend b3{nullptr, nullptr, 1.0 / 3.0, 2.0 / 3.0};
                if (e == hipSuccess) e = stage(ctx->f3, fa, ctx->lam3, la, ctx->u3, ua, &b3);
            }
            if (ctx->rk == 1) a = b;
        }
        ctx->stream = keep;
        a_end = a;
        return e;
    };
    hipError_t e = hipSuccess;
    int64_t done = 0;
    if ((int64_t)nx * ny <= kGraphCells && n >= kGraphSteps) {
        const int p = ctx->cur;
        const int64_t key = ((((int64_t)var * 2 + ord) * 64 + flags) * 4 + ctx->rk) * 2 + (walls ? 1 : 0);
        if (ctx->step_key[p] != key) {
            if (ctx->step_exec[p]) (void)hipGraphExecDestroy(ctx->step_exec[p]);
            ctx->step_exec[p] = nullptr;
            ctx->step_key[p] = -1;
            if (!ctx->step_cap) e = hipStreamCreateWithFlags(&ctx->step_cap, hipStreamNonBlocking);
            hipGraph_t g = nullptr;
            if (e == hipSuccess) e = hipStreamBeginCapture(ctx->step_cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                int a_end = p;
                const hipError_t le = issue(kGraphSteps, p, ctx->step_cap, a_end);
                e = hipStreamEndCapture(ctx->step_cap, &g);
                if (e == hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ctx->step_exec[p], g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(ctx, e, "step graph capture");
            ctx->step_key[p] = key;
        }
        for (; done + kGraphSteps <= n && e == hipSuccess; done += kGraphSteps)
            e = hipGraphLaunch(ctx->step_exec[p], ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "step graph launch");
    }
    int a_end = ctx->cur;
    e = issue(n - done, ctx->cur, ctx->stream, a_end);
    if (e != hipSuccess) return hip_fail(ctx, e, "step kernel");
    ctx->cur = a_end;
    ctx->steps += n;
    ctx->u_valid = amod;            // a step without A_hat does not write the velocity planes
    return LBKM_OK;
}

lbkm_status lbkm_get_moments(lbkm_ctx* ctx, double* rho, double* ux, double* uy, double* T, double* p,
                             double* lambda) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    hipError_t e = launch_moments(ctx->d, ctx->grid.nx, ctx->grid.ny, ctx->f[ctx->cur], ctx->lam[ctx->cur],
                                  rho, ux, uy, T, p, lambda, ctx->stream);
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "moments kernel");
}

lbkm_status lbkm_get_tne(lbkm_ctx* ctx, double* delta, double* d) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    hipError_t e = launch_tne(ctx->d, ctx->grid.nx, ctx->grid.ny, ctx->f[ctx->cur], delta, d, ctx->stream);
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "tne kernel");
}

lbkm_status lbkm_reduce(lbkm_ctx* ctx, double out[8]) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    if (!out) return fail(ctx, LBKM_EINVAL, "NULL output");
    const int64_t cells = (int64_t)ctx->grid.nx * ctx->grid.ny;
    int nb = (int)((cells + 255) / 256);
    if (nb > kReduceBlocks) nb = kReduceBlocks;
    hipError_t e = launch_reduce(ctx->d, ctx->f[ctx->cur], ctx->lam[ctx->cur], ctx->partials, nb, ctx->out8,
                                 ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, ctx->out8, 8 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduction");
    out[5] *= ctx->grid.dx / ctx->grid.ny;
    return LBKM_OK;
}

lbkm_status lbkm_ignition_margin(lbkm_ctx* ctx, double* margin) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    if (!margin) return fail(ctx, LBKM_EINVAL, "NULL output");
    const int64_t cells = (int64_t)ctx->grid.nx * ctx->grid.ny;
    int nb = (int)((cells + 255) / 256);
    if (nb > kReduceBlocks) nb = kReduceBlocks;
    hipError_t e = launch_margin(ctx->d, ctx->f[ctx->cur], ctx->lam[ctx->cur], ctx->partials, nb, ctx->out8,
                                 ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(margin, ctx->out8, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "ignition margin");
    return LBKM_OK;
}

lbkm_status lbkm_check(lbkm_ctx* ctx) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    int flag = 0;
    hipError_t e = launch_check(ctx->d, ctx->grid.nx, ctx->grid.ny, ctx->f[ctx->cur], ctx->lam[ctx->cur],
                                ctx->flag, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "check");
    if (flag) return fail(ctx, LBKM_ENONFINITE, "non-finite value, rho <= 0 or T <= 0 in the state");
    return LBKM_OK;
}

lbkm_status lbkm_get_state(lbkm_ctx* ctx, double* f, double* lam) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    hipError_t e = hipSuccess;
    if (f) e = launch_copy_state(ctx->d, ctx->grid.nx, ctx->grid.ny, ctx->f[ctx->cur], f, 24, 1, ctx->stream);
    if (e == hipSuccess && lam)
        e = launch_copy_state(ctx->d, ctx->grid.nx, ctx->grid.ny, ctx->lam[ctx->cur], lam, 1, 1, ctx->stream);
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "get_state");
}

lbkm_status lbkm_set_state(lbkm_ctx* ctx, const double* f, const double* lam) {
    lbkm_status st = ready(ctx, false);
    if (st != LBKM_OK) return st;
    if (!f || !lam) return fail(ctx, LBKM_EINVAL, "NULL state");
    ctx->cur = 0;
    hipError_t e = launch_copy_state(ctx->d, ctx->grid.nx, ctx->grid.ny, f, ctx->f[0], 24, 0, ctx->stream);
    if (e == hipSuccess)
        e = launch_copy_state(ctx->d, ctx->grid.nx, ctx->grid.ny, lam, ctx->lam[0], 1, 0, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "set_state");
    ctx->fields = true;
    ctx->steps = 0;
    ctx->u_valid = false;
    return LBKM_OK;
}

lbkm_status lbkm_set_tile(lbkm_ctx* ctx, int32_t tile_x, int32_t tile_y, int32_t lds) {
    if (!ctx) return LBKM_EINVAL;
    for (int v = 0; v < kNumStepVariants; ++v)
        if (kStepVariants[v][0] == tile_x && kStepVariants[v][1] == tile_y && kStepVariants[v][2] == lds) {
            ctx->step_variant = v;
            return LBKM_OK;
        }
    return fail(ctx, LBKM_EINVAL, "unsupported step tile shape");
}

lbkm_status lbkm_set_srt(lbkm_ctx* ctx, double tau) {
    if (!ctx) return LBKM_EINVAL;
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "not available on a batched context");
    if (!std::isfinite(tau) || tau < 0.0) return fail(ctx, LBKM_EINVAL, "tau must be finite and >= 0");
    if (tau > 0.0 && !(ctx->grid.dt / tau < 2.0))
        return fail(ctx, LBKM_EINVAL, "dt / tau >= 2: forward Euler relaxation is unstable");
    ctx->h.srt = tau > 0.0 ? 1 : 0;
    ctx->h.inv_tau = tau > 0.0 ? 1.0 / tau : 0.0;
    ctx->u_valid = false;
    return ctx->bound && ctx->params ? upload_consts(ctx) : LBKM_OK;
}

lbkm_status lbkm_set_boundary(lbkm_ctx* ctx, int32_t side, int32_t type, const double* state) {
    if (!ctx) return LBKM_EINVAL;
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "not available on a batched context");
    if (side < 0 || side > 3) return fail(ctx, LBKM_EINVAL, "side must be 0..3 (x_lo, x_hi, y_lo, y_hi)");
    if (type < kWallNone || type > kWallNee) return fail(ctx, LBKM_EINVAL, "unknown boundary type");
    const int axis_bc = side < 2 ? ctx->grid.bc_x : ctx->grid.bc_y;
    if (type != kWallNone && axis_bc != LBKM_BC_OUTFLOW)
        return fail(ctx, LBKM_EINVAL, "a wall side needs the outflow rule on its axis (the other side keeps it)");
    if (type != kWallNone && (int64_t)kGhostPlanes * 8 * ctx->h.gL * 8 > 0xFFFFFFFFll)
        return fail(ctx, LBKM_EINVAL, "ghost layers beyond 4 GiB (the longer grid side is too long for walls)");
    double v[5] = {0, 0, 0, 0, 0};
    if (type == kWallDirichlet || type == kWallNee) {
        if (!state) return fail(ctx, LBKM_EINVAL, "this boundary type needs a state");
        std::memcpy(v, state, sizeof(v));
        if (!finite_all(v, 5)) return fail(ctx, LBKM_EINVAL, "non-finite boundary state");
        if (!(v[1] > 0.0) || (type == kWallDirichlet && !(v[0] > 0.0)))
            return fail(ctx, LBKM_EINVAL, "boundary density and temperature must be > 0");
    }
    ctx->h.wall[side] = type;
    std::memcpy(ctx->h.wall_state[side], v, sizeof(v));
    return ctx->bound && ctx->params ? upload_consts(ctx) : LBKM_OK;
}

lbkm_status lbkm_set_time_scheme(lbkm_ctx* ctx, int32_t order) {
    if (!ctx) return LBKM_EINVAL;
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "not available on a batched context");
    if (order < 1 || order > 3) return fail(ctx, LBKM_EINVAL, "order must be 1, 2 or 3");
    ctx->rk = order;
    return LBKM_OK;
}

lbkm_status lbkm_set_tile_order(lbkm_ctx* ctx, int32_t vertical) {
    if (!ctx) return LBKM_EINVAL;
    if (vertical != 0 && vertical != 1) return fail(ctx, LBKM_EINVAL, "vertical must be 0 or 1");
    ctx->tile_order = vertical;
    return LBKM_OK;
}

lbkm_status lbkm_autotune(lbkm_ctx* ctx, int32_t* choice) {
    lbkm_status st = ready(ctx, true);
    if (st != LBKM_OK) return st;
    // wall sides run one shape (kWallTile): only the tile order is tuned
    int v_lo = 0, v_hi = kNumStepVariants;
    if (any_wall(ctx))
        for (int v = 0; v < kNumStepVariants; ++v)
            if (kStepVariants[v][0] == kWallTile[0] && kStepVariants[v][1] == kWallTile[1] &&
                kStepVariants[v][2] == kWallTile[2]) {
                v_lo = v;
                v_hi = v + 1;
            }
    const int64_t cells = ctx->pitch * (int64_t)ctx->grid.ny;
    const int cur = ctx->cur;
    const int64_t steps0 = ctx->steps;
    double* save = nullptr;
    hipError_t e = hipMalloc((void**)&save, sizeof(double) * 25 * cells);
    if (e == hipSuccess)
        e = hipMemcpyAsync(save, ctx->f[cur], sizeof(double) * 24 * cells, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(save + 24 * cells, ctx->lam[cur], sizeof(double) * cells, hipMemcpyDeviceToDevice,
                           ctx->stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    int best_v = ctx->step_variant, best_o = ctx->tile_order;
    // Every candidate is timed in two passes and keeps the better trial, so that one noisy
    // trial does not decide (the closest shapes differ by about 1 %).
    const int trial = 8, passes = 2;
    float t_ms[kNumStepVariants][2];
    for (int v = 0; v < kNumStepVariants; ++v) t_ms[v][0] = t_ms[v][1] = 1e30f;
    for (int pass = 0; pass < passes && st == LBKM_OK && e == hipSuccess; ++pass)
        for (int v = v_lo; v < v_hi && st == LBKM_OK && e == hipSuccess; ++v)
            for (int o = 0; o < 2 && e == hipSuccess; ++o) {
                ctx->step_variant = v;
                ctx->tile_order = o;
                st = lbkm_step(ctx, 1);                    // warm-up of this shape
                if (st != LBKM_OK) break;
                e = hipEventRecord(t0, ctx->stream);
                if (e == hipSuccess) st = lbkm_step(ctx, trial);
                if (st != LBKM_OK) break;
                e = hipEventRecord(t1, ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                if (e == hipSuccess && ms < t_ms[v][o]) t_ms[v][o] = ms;
            }
    // Row bands give each XCD a contiguous band of rows.  Where the work per cell varies
    // along y and moves with the flow (a reacting layer that ignites later), one XCD then
    // carries more of it, which a trial on the present state cannot see; column bands
    // spread any such layer over all XCDs.  So row bands are chosen only when they are
    // faster by more than 2 %.
    float best_ms = 1e30f;
    for (int v = v_lo; v < v_hi; ++v)
        for (int o = 0; o < 2; ++o) {
            const float ms = o == 0 ? 1.02f * t_ms[v][0] : t_ms[v][1];
            if (ms < best_ms) {
                best_ms = ms;
                best_v = v;
                best_o = o;
            }
        }
    ctx->step_variant = best_v;
    ctx->tile_order = best_o;
    ctx->cur = cur;
    ctx->steps = steps0;
    ctx->u_valid = false;          // the trial steps overwrote the velocity planes
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->f[cur], save, sizeof(double) * 24 * cells, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->lam[cur], save + 24 * cells, sizeof(double) * cells, hipMemcpyDeviceToDevice,
                           ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (save) (void)hipFree(save);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
    if (st != LBKM_OK) return st;
    if (choice) {
        choice[0] = kStepVariants[best_v][0];
        choice[1] = kStepVariants[best_v][1];
        choice[2] = kStepVariants[best_v][2];
        choice[3] = best_o;
    }
    return LBKM_OK;
}

lbkm_status lbkm_get_matrices(lbkm_ctx* ctx, double* M, double* Minv, double* cond) {
    if (!ctx || !M || !Minv) return LBKM_EINVAL;
    dense_from_blocks(&ctx->h, M, Minv);
    if (cond) *cond = ctx->cond;
    return LBKM_OK;
}

lbkm_status lbkm_get_step_count(lbkm_ctx* ctx, int64_t* out) {
    if (!ctx || !out) return LBKM_EINVAL;
    *out = ctx->steps;
    return LBKM_OK;
}

lbkm_status lbkm_copy_kernel(const double* src, double* dst, int64_t n, void* hip_stream) {
    if (!src || !dst || n < 0 || (n / 2 + 255) / 256 > INT32_MAX) return LBKM_EINVAL;
    return launch_copy(src, dst, n, (hipStream_t)hip_stream) == hipSuccess ? LBKM_OK : LBKM_EDEVICE;
}

const char* lbkm_last_error(const lbkm_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

lbkm_status lbkm_destroy(lbkm_ctx* ctx) {
    if (!ctx) return LBKM_EINVAL;
    drop_step_graphs(ctx);
    if (ctx->step_cap) (void)hipStreamDestroy(ctx->step_cap);
    destroy_extras(ctx);
    if (ctx->d) (void)hipFree(ctx->d);
    if (ctx->partials) (void)hipFree(ctx->partials);
    if (ctx->out8) (void)hipFree(ctx->out8);
    if (ctx->flag) (void)hipFree(ctx->flag);
    if (ctx->adj_scratch) (void)hipFree(ctx->adj_scratch);
    for (int i = 0; i < 2; ++i)
        if (ctx->u[i]) (void)hipFree(ctx->u[i]);
    for (double* p : {ctx->f3, ctx->lam3, ctx->u3, ctx->gbuf})
        if (p) (void)hipFree(p);
    delete ctx;
    return LBKM_OK;
}

}  // extern "C"
