// Context structure behind the opaque lbkm_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbkm.h"
#include "lbkm_internal.h"

namespace lbkm {
constexpr int kReduceBlocks = 1024;   // per-work-group partials of lbkm_reduce
struct BatchState;                    // batched contexts (batch.hip)
}

struct lbkm_ctx {
    lbkm_grid grid{};
    hipStream_t stream = nullptr;
    int batched = 0;
    double* f[2] = {nullptr, nullptr};
    double* lam[2] = {nullptr, nullptr};
    int64_t pitch = 0;
    int cur = 0;
    int step_variant = 10;             // launch shape of the step kernel (kStepVariants): 64x4, collide first,
                                       // centre values shared in LDS (the fastest on MI355X at 2048^2)
    int tile_order = 1;                // 1: bands of tile columns per XCD, 0: bands of tile rows
    bool bound = false, params = false, fields = false;
    int64_t steps = 0;
    double cond = 0.0;
    lbkm::Consts h{};                  // host copy of the device constants
    lbkm::Consts* d = nullptr;         // device constants
    double* partials = nullptr;        // reduction scratch
    double* out8 = nullptr;
    int* flag = nullptr;
    lbkm::BatchState* batch = nullptr;
    double* u[2] = {nullptr, nullptr}; // velocity planes [2][plane] of f[0], f[1] (inputs of A_hat)
    int64_t u_plane = 0;
    bool u_valid = false;              // u[cur] holds the velocity of f[cur]
    int rk = 1;                        // time scheme: 1 forward Euler, 2 SSP-RK2, 3 SSP-RK3
    double* f3 = nullptr;              // third state for SSP-RK3 (library-owned): f, lambda, u
    double* lam3 = nullptr;
    double* u3 = nullptr;
    int64_t rk3_plane = 0;
    double* gbuf = nullptr;            // ghost layers of the wall sides [27][4][2][max(nx, ny)]
    double* adj_scratch = nullptr;     // adjoint step: U, W planes and parameter partials
    int64_t adj_scratch_n = 0;
    // small grids: the launches of kGraphSteps steps captured once per buffer parity and
    // launch configuration (step_key) and replayed by lbkm_step
    hipGraphExec_t step_exec[2] = {nullptr, nullptr};
    int64_t step_key[2] = {-1, -1};
    hipStream_t step_cap = nullptr;
    std::string err;
};

namespace lbkm {
lbkm_status fail(lbkm_ctx* ctx, lbkm_status st, const std::string& msg);
lbkm_status hip_fail(lbkm_ctx* ctx, hipError_t e, const char* what);
lbkm_status fill_physics(lbkm_ctx* ctx, Consts* c, const double S[24], double gamma, double Pr, double Q,
                         const lbkm_rates* rates, double dt);
lbkm_status validate_grid_common(lbkm_ctx* ctx, const lbkm_grid* g);
lbkm_status build_tables(lbkm_ctx* ctx, const lbkm_grid* g);
lbkm_status upload_consts(lbkm_ctx* ctx);
lbkm_status ensure_device_tables(lbkm_ctx* ctx);
void destroy_extras(lbkm_ctx* ctx);
hipError_t setup_noalloc_scratch();   // adjoint.hip: scratch address of lbkm_tne_loss_noalloc
}  // namespace lbkm
