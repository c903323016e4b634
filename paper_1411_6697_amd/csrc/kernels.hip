// HIP kernels of the single-grid MRT-LBKM path (gfx950, float64) and their launchers.
//
// Initialisation, readouts, reductions and copies.  State layout (structure of arrays):
// f[24][ny][pitch], lambda[ny][pitch].  The step kernel lives in step.hip.

#include <hip/hip_runtime.h>

#include "lbkm_device.h"
#include "lbkm_kernels.h"

namespace lbkm {

namespace {

__device__ __forceinline__ void load_cell(const double* __restrict__ f, int64_t plane, int64_t at,
                                          double v[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = f[i * plane + at];
}

// f = M^-1 f_hat^eq(rho, u, T) (Eq. moment12), lambda copied; inputs dense [ny][nx]
__global__ __launch_bounds__(256) void k_init(const Consts* __restrict__ c, const double* __restrict__ rho,
                                              const double* __restrict__ ux, const double* __restrict__ uy,
                                              const double* __restrict__ T, const double* __restrict__ lam,
                                              double* __restrict__ f, double* __restrict__ lout) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t dn = (int64_t)y * c->nx + x, at = (int64_t)y * c->pitch + x;
    Blocks e, s;
    equilibrium(rho[dn], ux[dn], uy[dn], T[dn], c->I, e);
    inverse(c, e, s);
    double v[NV];
    from_combos(s, v);
#pragma unroll
    for (int i = 0; i < NV; ++i) f[i * c->plane + at] = v[i];
    lout[at] = lam[dn];
}

__device__ __forceinline__ void natural_delta(const Blocks& h, const Blocks& e, double dk[NV]) {
#pragma unroll
    for (int r = 0; r < NEE; ++r) dk[EE_M[r]] = h.ee[r] - e.ee[r];
#pragma unroll
    for (int r = 0; r < NOE; ++r) dk[OE_M[r]] = h.oe[r] - e.oe[r];
#pragma unroll
    for (int r = 0; r < NEO; ++r) dk[EO_M[r]] = h.eo[r] - e.eo[r];
#pragma unroll
    for (int r = 0; r < NOO; ++r) dk[OO_M[r]] = h.oo[r] - e.oo[r];
}

__global__ __launch_bounds__(256) void k_moments(const Consts* __restrict__ c, const double* __restrict__ f,
                                                 const double* __restrict__ lam, double* rho, double* ux,
                                                 double* uy, double* T, double* p, double* lout) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t dn = (int64_t)y * c->nx + x, at = (int64_t)y * c->pitch + x;
    double v[NV];
    load_cell(f, c->plane, at, v);
    Blocks s, h;
    to_combos(v, s);
    forward(c, s, h);
    const Macro m = macro_of(h, c->DI);
    if (rho) rho[dn] = m.rho;
    if (ux) ux[dn] = m.ux;
    if (uy) uy[dn] = m.uy;
    if (T) T[dn] = m.T;
    if (p) p[dn] = m.rho * m.T;
    if (lout) lout[dn] = lam[at];
}

__global__ __launch_bounds__(256) void k_tne(const Consts* __restrict__ c, const double* __restrict__ f,
                                             double* delta, double* dist) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t dn = (int64_t)y * c->nx + x, at = (int64_t)y * c->pitch + x;
    const int64_t cells = (int64_t)c->nx * c->ny;
    double v[NV];
    load_cell(f, c->plane, at, v);
    Blocks s, h, e;
    to_combos(v, s);
    forward(c, s, h);
    const Macro m = macro_of(h, c->DI);
    equilibrium(m.rho, m.ux, m.uy, m.T, c->I, e);
    double dk[NV];
    natural_delta(h, e, dk);
    double ss = 0.0;
#pragma unroll
    for (int k = 4; k < NV; ++k) {
        if (delta) delta[(k - 4) * cells + dn] = dk[k];
        ss = fma(dk[k], dk[k], ss);
    }
    if (dist) dist[dn] = sqrt(ss);
}

// wave64 + work-group reduction of 8 values (sum x6, min, max); deterministic order
__device__ __forceinline__ void block_reduce8(double v[8], double* sh /*[4][8]*/) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] += __shfl_xor(v[k], off, 64);
        v[6] = fmin(v[6], __shfl_xor(v[6], off, 64));
        v[7] = fmax(v[7], __shfl_xor(v[7], off, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 8; ++k) sh[wave * 8 + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            for (int k = 0; k < 6; ++k) v[k] += sh[w * 8 + k];
            v[6] = fmin(v[6], sh[w * 8 + 6]);
            v[7] = fmax(v[7], sh[w * 8 + 7]);
        }
    }
}

// per-work-group partial reductions over a grid-stride range of cells
__global__ __launch_bounds__(256) void k_reduce_partial(const Consts* __restrict__ c,
                                                        const double* __restrict__ f,
                                                        const double* __restrict__ lam,
                                                        double* __restrict__ partials) {
    __shared__ double sh[4 * 8];
    const int64_t cells = (int64_t)c->nx * c->ny;
    double v[8] = {0, 0, 0, 0, 0, 0, INFINITY, -INFINITY};
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < cells;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(q / c->nx), x = (int)(q % c->nx);
        const int64_t at = (int64_t)y * c->pitch + x;
        double fv[NV];
        load_cell(f, c->plane, at, fv);
        Blocks s, h, e;
        to_combos(fv, s);
        forward(c, s, h);
        const Macro m = macro_of(h, c->DI);
        equilibrium(m.rho, m.ux, m.uy, m.T, c->I, e);
        double dk[NV];
        natural_delta(h, e, dk);
        double ss = 0.0;
#pragma unroll
        for (int k = 4; k < NV; ++k) ss = fma(dk[k], dk[k], ss);
        v[0] += h.ee[0];
        v[1] += h.oe[0];
        v[2] += h.eo[0];
        v[3] += 0.5 * h.ee[1];
        v[4] += ss;
        v[5] += fabs(dk[4]);
        const double l = lam[at];
        v[6] = fmin(v[6], l);
        v[7] = fmax(v[7], l);
    }
    block_reduce8(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) partials[blockIdx.x * 8 + k] = v[k];
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partials, int n,
                                                      double* __restrict__ out) {
    __shared__ double sh[4 * 8];
    double v[8] = {0, 0, 0, 0, 0, 0, INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
        for (int k = 0; k < 6; ++k) v[k] += partials[b * 8 + k];
        v[6] = fmin(v[6], partials[b * 8 + 6]);
        v[7] = fmax(v[7], partials[b * 8 + 7]);
    }
    block_reduce8(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) out[k] = v[k];
}

// ignition margin: per-work-group minima of |T - T_ig| over the cells with lambda < 1
__global__ __launch_bounds__(256) void k_margin_partial(const Consts* __restrict__ c,
                                                        const double* __restrict__ f,
                                                        const double* __restrict__ lam,
                                                        double* __restrict__ partials) {
    __shared__ double sh[4];
    const int64_t cells = (int64_t)c->nx * c->ny;
    double v = INFINITY;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < cells;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(q / c->nx), x = (int)(q % c->nx);
        const int64_t at = (int64_t)y * c->pitch + x;
        if (!(lam[at] < 1.0)) continue;
        double fv[NV];
        load_cell(f, c->plane, at, fv);
        Blocks s, h;
        to_combos(fv, s);
        forward(c, s, h);
        const Macro m = macro_of(h, c->DI);
        v = fmin(v, fabs(m.T - c->Tig));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmin(v, sh[w]);
        partials[blockIdx.x] = v;
    }
}

__global__ __launch_bounds__(256) void k_min_final(const double* __restrict__ partials, int n,
                                                   double* __restrict__ out) {
    __shared__ double sh[4];
    double v = INFINITY;
    for (int b = threadIdx.x; b < n; b += blockDim.x) v = fmin(v, partials[b]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmin(v, sh[w]);
        out[0] = v;
    }
}

// health check: NaN/Inf anywhere in f or lambda, rho <= 0 or T <= 0
__global__ __launch_bounds__(256) void k_check(const Consts* __restrict__ c, const double* __restrict__ f,
                                               const double* __restrict__ lam, int* flag) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t at = (int64_t)y * c->pitch + x;
    double v[NV];
    load_cell(f, c->plane, at, v);
    bool bad = !isfinite(lam[at]);
#pragma unroll
    for (int i = 0; i < NV; ++i) bad |= !isfinite(v[i]);
    Blocks s, h;
    to_combos(v, s);
    forward(c, s, h);
    const Macro m = macro_of(h, c->DI);
    bad |= !(m.rho > 0.0) || !(m.T > 0.0);
    if (bad) atomicOr(flag, 1);
}

// velocity of every cell in plane order (the same operations the step uses when it writes
// a new state), for A_hat of the next step
__global__ __launch_bounds__(256) void k_velocity(const Consts* __restrict__ c, const double* __restrict__ f,
                                                  double* __restrict__ u) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t at = (int64_t)y * c->pitch + x;
    VelAcc va;
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
        for (int d = 0; d < 8; ++d) vel_add(va, c, g, d, f[(int64_t)(8 * g + d) * c->plane + at]);
    u[at] = va.jx / va.r;
    u[c->plane + at] = va.jy / va.r;
}

// Ghost layers of the wall sides (Sec. IV C, IV D name the boundaries without formulas):
//   reflect:   layer k holds interior layer k with mirrored velocities, lambda alike;
//   dirichlet: both layers hold the discrete equilibrium of the given state and lambda;
//   nee:       both layers hold f^eq(rho_edge, wall T and u) + (f - f^eq) of the edge cell,
//              lambda copies the edge cell;
// and the velocity planes hold the velocity moment of the ghost distributions.
// One thread per (side, position along the side).
__global__ __launch_bounds__(256) void k_ghost(const Consts* __restrict__ c, const double* __restrict__ f,
                                               const double* __restrict__ lam, double* __restrict__ gb) {
    const int side = blockIdx.y;
    const int type = c->wall[side];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = c->nx, ny = c->ny;
    if (type == kWallNone || j >= (side < 2 ? ny : nx)) return;
    const int64_t L = c->gL, gplane = 8 * L;
    // mirror of direction d across a wall normal to x (sides 0, 1) or to y (sides 2, 3)
    constexpr int kMirrorX[8] = {2, 1, 0, 3, 5, 4, 7, 6};
    constexpr int kMirrorY[8] = {0, 3, 2, 1, 7, 6, 5, 4};
    auto cell = [&](int k) -> int64_t {                 // interior layer k from the edge
        int x, y;
        if (side < 2) {
            const int kk = k < nx ? k : nx - 1;
            x = side == 0 ? kk : nx - 1 - kk;
            y = j;
        } else {
            const int kk = k < ny ? k : ny - 1;
            y = side == 2 ? kk : ny - 1 - kk;
            x = j;
        }
        return (int64_t)y * c->pitch + x;
    };
    auto put = [&](int layer, int p, double v) { gb[p * gplane + (side * 2 + layer) * L + j] = v; };
    double g[NV];
    for (int layer = 0; layer < 2; ++layer) {
        if (type == kWallReflect || layer == 0) {
            const int64_t at = cell(type == kWallReflect ? layer : 0);
            double fc[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) fc[i] = f[i * c->plane + at];
            const double lc = lam[at];
            if (type == kWallReflect) {
#pragma unroll
                for (int gg = 0; gg < 3; ++gg)
#pragma unroll
                    for (int d = 0; d < 8; ++d) g[8 * gg + d] = fc[8 * gg + (side < 2 ? kMirrorX[d] : kMirrorY[d])];
                put(layer, NV, lc);
            } else {
                const double* st = c->wall_state[side];
                double feqw[NV];
                Blocks e, se;
                if (type == kWallDirichlet) {
                    equilibrium(st[0], st[2], st[3], st[1], c->I, e);
                    inverse(c->mat, e, se);
                    from_combos(se, g);
                    put(0, NV, st[4]);
                } else {
                    const Macro m = macro_sums(c, fc);
                    equilibrium(m.rho, m.ux, m.uy, m.T, c->I, e);
                    inverse(c->mat, e, se);
                    double feq0[NV];
                    from_combos(se, feq0);
                    equilibrium(m.rho, st[2], st[3], st[1], c->I, e);
                    inverse(c->mat, e, se);
                    from_combos(se, feqw);
#pragma unroll
                    for (int i = 0; i < NV; ++i) g[i] = feqw[i] + (fc[i] - feq0[i]);
                    put(0, NV, lc);
                }
            }
        } else {
            put(1, NV, gb[NV * gplane + (side * 2) * L + j]);   // the second layer repeats the first
        }
        VelAcc va;
#pragma unroll
        for (int gg = 0; gg < 3; ++gg)
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                put(layer, 8 * gg + d, g[8 * gg + d]);
                vel_add(va, c, gg, d, g[8 * gg + d]);
            }
        put(layer, NV + 1, va.jx / va.r);
        put(layer, NV + 2, va.jy / va.r);
    }
}

// pitched <-> dense copies of the state
__global__ __launch_bounds__(256) void k_copy_state(const Consts* __restrict__ c, const double* __restrict__ src,
                                                    double* __restrict__ dst, int planes, int to_dense) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t cells = (int64_t)c->nx * c->ny;
    const int64_t dn = (int64_t)y * c->nx + x, at = (int64_t)y * c->pitch + x;
    for (int i = 0; i < planes; ++i) {
        if (to_dense)
            dst[i * cells + dn] = src[i * c->plane + at];
        else
            dst[i * c->plane + at] = src[i * cells + dn];
    }
}

__global__ void k_fill_int(int* p, int v) { *p = v; }

// plain streaming copy (bandwidth calibration): one 16-byte access per thread
__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                              int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n2) dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------- launchers

static dim3 row_grid(int nx, int ny) { return dim3((nx + 255) / 256, ny); }

hipError_t launch_init(const Consts* dc, int nx, int ny, const double* rho, const double* ux,
                       const double* uy, const double* T, const double* lam, double* f, double* lout,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_init, row_grid(nx, ny), dim3(256), 0, st, dc, rho, ux, uy, T, lam, f, lout);
    return hipGetLastError();
}

hipError_t launch_moments(const Consts* dc, int nx, int ny, const double* f, const double* lam,
                          double* rho, double* ux, double* uy, double* T, double* p, double* lout,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_moments, row_grid(nx, ny), dim3(256), 0, st, dc, f, lam, rho, ux, uy, T, p, lout);
    return hipGetLastError();
}

hipError_t launch_tne(const Consts* dc, int nx, int ny, const double* f, double* delta, double* dist,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_tne, row_grid(nx, ny), dim3(256), 0, st, dc, f, delta, dist);
    return hipGetLastError();
}

hipError_t launch_margin(const Consts* dc, const double* f, const double* lam, double* partials,
                         int nblocks, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_margin_partial, dim3(nblocks), dim3(256), 0, st, dc, f, lam, partials);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(256), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_reduce(const Consts* dc, const double* f, const double* lam, double* partials,
                         int nblocks, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partial, dim3(nblocks), dim3(256), 0, st, dc, f, lam, partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_check(const Consts* dc, int nx, int ny, const double* f, const double* lam, int* flag,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, st, flag, 0);
    hipLaunchKernelGGL(k_check, row_grid(nx, ny), dim3(256), 0, st, dc, f, lam, flag);
    return hipGetLastError();
}

hipError_t launch_velocity(const Consts* dc, int nx, int ny, const double* f, double* u, hipStream_t st) {
    hipLaunchKernelGGL(k_velocity, row_grid(nx, ny), dim3(256), 0, st, dc, f, u);
    return hipGetLastError();
}

hipError_t launch_ghost(const Consts* dc, int nx, int ny, const double* f, const double* lam, double* gb,
                        hipStream_t st) {
    const int len = nx > ny ? nx : ny;
    hipLaunchKernelGGL(k_ghost, dim3((len + 255) / 256, 4), dim3(256), 0, st, dc, f, lam, gb);
    return hipGetLastError();
}

hipError_t launch_copy_state(const Consts* dc, int nx, int ny, const double* src, double* dst, int planes,
                             int to_dense, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_state, row_grid(nx, ny), dim3(256), 0, st, dc, src, dst, planes, to_dense);
    return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st) {
    const int64_t n2 = n / 2;
    if (n2 > 0)
        hipLaunchKernelGGL(k_copy, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, (const double2*)src,
                           (double2*)dst, n2);
    if (n & 1) (void)hipMemcpyAsync(dst + n - 1, src + n - 1, sizeof(double), hipMemcpyDeviceToDevice, st);
    return hipGetLastError();
}

}  // namespace lbkm
