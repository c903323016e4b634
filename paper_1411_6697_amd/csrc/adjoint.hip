// Discrete adjoint (reverse mode, written by hand) of one step of the MRT-LBKM scheme, of
// the initialisation f = M^-1 f_hat^eq, and of the non-equilibrium loss
// L = sum_cells sum_{k=5..24} Delta_k^2 (Sec. VI).  Every branch of the forward step (the
// minmod selections of the NND scheme, the upwind side of lambda, the ignition test) is
// taken as the forward step takes it from the level-n state, so the result is the exact
// derivative of the discrete map on the branch that the run follows.
//
// One adjoint step is three passes over the grid (all arrays dense [plane][ny][nx]):
//   k_adj_macro   rho, u_x, u_y of every cell (the neighbours' values are needed twice)
//   k_adj_local   the transposed Jacobian of everything that is local to a cell:
//                 collision (M, f_hat^eq, R, A_hat), chemistry (Cochran step and
//                 C_i), the velocity factor of the lambda advection; parameter gradients
//                 (per work-group partial sums); the adjoints of the velocity gradients
//                 inside A_hat, which belong to the neighbours (3 values per cell)
//   k_adj_stream  the identity of the Euler step, the transposed NND streaming of f and
//                 lambda (a gather over the cells whose stencil reaches this cell, boundary
//                 rules included) and the neighbours' A_hat terms
// followed by a fixed-order reduction of the parameter partials.

#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "lbkm_abi_internal.h"
#include "lbkm_device.h"
#include "lbkm_kernels.h"

namespace lbkm {

namespace {

constexpr int kAdjThreads = 256;
constexpr int kNumGrad = 27;      // d/dR_1..R_24, d/dQ, d/domega_1, d/domega_2
constexpr int kNumLds = 23;       // the ones a cell can touch: R_5..R_24, Q, omega_1, omega_2

// y = A^T x for a block stored column-major (At[k][r] = A[r][k]): y_k = sum_r At[k][r] x_r.
// Each stored column is read through the constant address space just before its dot
// product: the copy of its address is tied to the previous result, so the compiler does
// not hoist all N*N scalar loads to the top (which runs out of scalar registers).
template <int N>
__device__ __forceinline__ void matvec_t(const double (*At)[N], const double* x, double* y) {
    typedef const __attribute__((address_space(4))) double cdouble;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double* col = At[k];
        if (k == 0)
            asm volatile("" : "+s"(col) : "v"(x[N - 1]));
        else
            asm volatile("" : "+s"(col) : "v"(y[k - 1]));
        cdouble* A = (cdouble*)(const void*)col;
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) s = fma(A[r], x[r], s);
        y[k] = s;
    }
}

// M^T hb (moment adjoints in block order -> velocity order).  M = B P with P the
// symmetric combinations, and P^T is the recombination from_combos.
__device__ __forceinline__ void forward_t(const Mats& M, const Blocks& hb, double fb[NV]) {
    Blocks s;
    matvec_t<NEE>(M.BEE, hb.ee, s.ee);
    matvec_t<NOE>(M.BOE, hb.oe, s.oe);
    matvec_t<NEO>(M.BEO, hb.eo, s.eo);
    matvec_t<NOO>(M.BOO, hb.oo, s.oo);
    from_combos(s, fb);
}

// M^-T x (velocity order -> block order).  M^-1 = P^T C, so M^-T = C^T P.
__device__ __forceinline__ void inverse_t(const Mats& M, const double x[NV], Blocks& y) {
    Blocks s;
    to_combos(x, s);
    matvec_t<NEE>(M.CEE, s.ee, y.ee);
    matvec_t<NOE>(M.COE, s.oe, y.oe);
    matvec_t<NEO>(M.CEO, s.eo, y.eo);
    matvec_t<NOO>(M.COO, s.oo, y.oo);
}

__device__ __forceinline__ void zero(Blocks& b) {
#pragma unroll
    for (int r = 0; r < NEE; ++r) b.ee[r] = 0.0;
#pragma unroll
    for (int r = 0; r < NOE; ++r) b.oe[r] = 0.0;
#pragma unroll
    for (int r = 0; r < NEO; ++r) b.eo[r] = 0.0;
#pragma unroll
    for (int r = 0; r < NOO; ++r) b.oo[r] = 0.0;
}

// Adjoint of the closed forms of f_hat^eq (Sec. II, factor T in entries 14 and 16):
// (rb, xb, yb, Tb) += J^T eb with J = d f_hat^eq / d(rho, u_x, u_y, T).  Each entry is
// rho * phi_k(u_x, u_y, T); the partial derivatives of phi_k are written out below.
__device__ __forceinline__ void equilibrium_t(double rho, double x, double y, double T, double I,
                                              const Blocks& eb, double& rb, double& xb, double& yb,
                                              double& Tb) {
    const double D = 2.0, DI = D + I;
    const double u2 = x * x + y * y;
    const double a2 = (DI + 2.0) * T + u2;
    const double a4 = (DI + 4.0) * T + u2;
    const double k10 = 2.0 * D + I + 8.0;
    const double c10 = u2 * u2 + (D + 2.0) * (DI + 4.0) * T * T + k10 * u2 * T;
    const double c10x = 4.0 * x * u2 + 2.0 * k10 * x * T;
    const double c10y = 4.0 * y * u2 + 2.0 * k10 * y * T;
    const double c10T = 2.0 * (D + 2.0) * (DI + 4.0) * T + k10 * u2;
    const double k11 = D + 3.0 * I + 2.0;
    const double c11 = u2 + k11 * T;
    double pr = 0.0, px = 0.0, py = 0.0, pT = 0.0;
    auto acc = [&](double w, double phi, double fx, double fy, double fT) {
        pr = fma(w, phi, pr);
        px = fma(w, fx, px);
        py = fma(w, fy, py);
        pT = fma(w, fT, pT);
    };
    // EE: m1 m4 m5 m7 m14 m16 m17 m19 m20
    acc(eb.ee[0], 1.0, 0.0, 0.0, 0.0);
    acc(eb.ee[1], DI * T + u2, 2.0 * x, 2.0 * y, DI);
    acc(eb.ee[2], T + x * x, 2.0 * x, 0.0, 1.0);
    acc(eb.ee[3], T + y * y, 0.0, 2.0 * y, 1.0);
    acc(eb.ee[4], a2 * T + x * x * a4, 2.0 * x * T + 2.0 * x * a4 + 2.0 * x * x * x, 2.0 * y * T + 2.0 * x * x * y,
        a2 + (DI + 2.0) * T + (DI + 4.0) * x * x);
    acc(eb.ee[5], a2 * T + y * y * a4, 2.0 * x * T + 2.0 * x * y * y, 2.0 * y * T + 2.0 * y * a4 + 2.0 * y * y * y,
        a2 + (DI + 2.0) * T + (DI + 4.0) * y * y);
    acc(eb.ee[6], I * T * T + I * x * x * T, 2.0 * I * x * T, 0.0, 2.0 * I * T + I * x * x);
    acc(eb.ee[7], I * T * T + I * y * y * T, 0.0, 2.0 * I * y * T, 2.0 * I * T + I * y * y);
    acc(eb.ee[8], I * T * (u2 + (D + 3.0 * I) * T), 2.0 * I * x * T, 2.0 * I * y * T,
        I * u2 + 2.0 * I * (D + 3.0 * I) * T);
    // OE: m2 m8 m10 m12 m21 m23
    acc(eb.oe[0], x, 1.0, 0.0, 0.0);
    acc(eb.oe[1], x * a2, a2 + 2.0 * x * x, 2.0 * x * y, (DI + 2.0) * x);
    acc(eb.oe[2], 3.0 * x * T + x * x * x, 3.0 * T + 3.0 * x * x, 0.0, 3.0 * x);
    acc(eb.oe[3], x * T + x * y * y, T + y * y, 2.0 * x * y, x);
    acc(eb.oe[4], x * c10, c10 + x * c10x, x * c10y, x * c10T);
    acc(eb.oe[5], I * T * x * c11, I * T * c11 + 2.0 * I * T * x * x, 2.0 * I * T * x * y,
        I * x * c11 + I * T * x * k11);
    // EO: m3 m9 m11 m13 m22 m24
    acc(eb.eo[0], y, 0.0, 1.0, 0.0);
    acc(eb.eo[1], y * a2, 2.0 * x * y, a2 + 2.0 * y * y, (DI + 2.0) * y);
    acc(eb.eo[2], y * T + x * x * y, 2.0 * x * y, T + x * x, y);
    acc(eb.eo[3], 3.0 * y * T + y * y * y, 0.0, 3.0 * T + 3.0 * y * y, 3.0 * y);
    acc(eb.eo[4], y * c10, y * c10x, c10 + y * c10y, y * c10T);
    acc(eb.eo[5], I * T * y * c11, 2.0 * I * T * x * y, I * T * c11 + 2.0 * I * T * y * y,
        I * y * c11 + I * T * y * k11);
    // OO: m6 m15 m18
    acc(eb.oo[0], x * y, y, x, 0.0);
    acc(eb.oo[1], x * y * a4, y * a4 + 2.0 * x * x * y, x * a4 + 2.0 * x * y * y, (DI + 4.0) * x * y);
    acc(eb.oo[2], I * x * y * T, I * y * T, I * x * T, I * x * y);
    rb += pr;
    xb += rho * px;
    yb += rho * py;
    Tb += rho * pT;
}

// Adjoint of rho = h_1, u = (h_2, h_3)/rho, T = (h_4/rho - u^2)/(D+I): adds to hb.
__device__ __forceinline__ void macro_t(const Blocks& h, const Macro& m, double DI, double rb, double xb,
                                        double yb, double Tb, Blocks& hb) {
    hb.ee[1] += Tb / (DI * m.rho);
    rb -= Tb * h.ee[1] / (DI * m.rho * m.rho);
    xb -= 2.0 * m.ux * Tb / DI;
    yb -= 2.0 * m.uy * Tb / DI;
    hb.oe[0] += xb / m.rho;
    rb -= xb * m.ux / m.rho;
    hb.eo[0] += yb / m.rho;
    rb -= yb * m.uy / m.rho;
    hb.ee[0] += rb;
}

// Derivative of minmod(a, b) = median(a, b, 0) with respect to (a, b): the selected
// argument gets 1, a tie between equal arguments splits it in halves, the zero branch
// gets nothing.
__device__ __forceinline__ void minmod_sel(double a, double b, double& sa, double& sb) {
    // branch-free: selects only
    const bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
    const bool a_smaller = fabs(a) < fabs(b);
    const double wa = a == b ? 0.5 : (a_smaller ? 1.0 : 0.0);
    sa = same ? wa : 0.0;
    sb = same ? 1.0 - wa : 0.0;
}

// Stencil bookkeeping of the transposed NND operator along one axis for the cell at
// position x (extent n, boundary rule bc).  With G(k) = a_k +- mm(a_k - a_{k-1},
// a_{k+1} - a_k)/2 the interface value, the forward derivative at cell j is
// (G(j) - G(j-1))/h for a positive speed and (G(j+1) - G(j))/h for a negative one, so
// this cell receives adjoint through the interfaces k = x-1, x, x+1 and their three
// slots k-1, k, k+1 (positions mapped by the boundary rule).
struct AxisAdj {
    int pos[5];        // cell index of offsets -2..2 under the boundary rule
    double val[5];     // 1 if offset t is a real cell (periodic: always), else 0
    double mk[3][3];   // interface x-1+q reaches this cell through slot t (-1, 0, 1)
};

__device__ __forceinline__ AxisAdj axis_adj(int x, int n, int bc) {
    AxisAdj A;
#pragma unroll
    for (int t = -2; t <= 2; ++t) {
        A.pos[t + 2] = wrap(x + t, n, bc);
        A.val[t + 2] = (bc == 0 || (x + t >= 0 && x + t < n)) ? 1.0 : 0.0;
    }
    // periodic with n < 3: x-1, x, x+1 are not distinct interfaces; count each once
    const bool c0 = bc != 0 || n >= 2, c2 = bc != 0 || n >= 3;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const bool cand = q == 1 || (q == 0 ? c0 : c2);
#pragma unroll
        for (int t = 0; t < 3; ++t) A.mk[q][t] = (cand && A.pos[q + t] == x) ? 1.0 : 0.0;
    }
    return A;
}

// Transposed NND derivative for one plane along one axis.  av[t] holds the adjoint of the
// derivative D at offset t - 2 (zero outside the grid), fv[t] the level-n values.
// sgn = +1: the upwind side is j-2..j+1 (G = a + mm/2); sgn = -1: j-1..j+2 (G = a - mm/2).
__device__ __forceinline__ double nnd_t(const AxisAdj& A, const double fv[5], const double av[5], int sgn) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double sa, sb;
        minmod_sel(fv[q + 1] - fv[q], fv[q + 2] - fv[q + 1], sa, sb);
        const double h = 0.5 * sgn;
        const double w0 = -h * sa, w1 = 1.0 + h * (sa - sb), w2 = h * sb;
        // interface x-1+q feeds the cells x-1+q (+) and x+q (-) for sgn > 0, and
        // x-2+q (+) and x-1+q (-) for sgn < 0
        const double Gb = sgn > 0 ? av[q + 1] - av[q + 2] : av[q] - av[q + 1];
        acc = fma(Gb, A.mk[q][0] * w0 + A.mk[q][1] * w1 + A.mk[q][2] * w2, acc);
    }
    return acc;
}

__device__ __forceinline__ void block_reduce_grad(double v[kNumGrad], double* sh /*[4][kNumGrad]*/) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < kNumGrad; ++k) v[k] += __shfl_xor(v[k], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < kNumGrad; ++k) sh[wave * kNumGrad + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            for (int k = 0; k < kNumGrad; ++k) v[k] += sh[w * kNumGrad + k];
}

__device__ __forceinline__ void load_dense(const double* __restrict__ f, int64_t plane, int64_t at, double v[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = f[i * plane + at];
}

__global__ __launch_bounds__(kAdjThreads) void k_adj_macro(const Consts* __restrict__ c,
                                                           const double* __restrict__ f, double* __restrict__ U) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= c->nx) return;
    const int64_t plane = (int64_t)c->nx * c->ny, at = (int64_t)y * c->nx + x;
    double v[NV];
    load_dense(f, plane, at, v);
    Blocks s, h;
    to_combos(v, s);
    forward(c->mat, s, h);
    const Macro m = macro_of(h, c->DI);
    U[at] = m.rho;
    U[plane + at] = m.ux;
    U[2 * plane + at] = m.uy;
}

// Register pressure: the parameter gradients of each thread are kept in LDS (not in
// registers); the collision part's contribution M^T h_bar (moments 5..24) is written out as
// soon as it is known; the equilibrium adjoint is folded into (rho, u, T) adjoints right
// after the collision part and again after the chemistry part; f_hat^eq is evaluated a
// second time inside the chemistry branch instead of being kept alive.  The adjoints of the
// conserved moments h_1..h_4 are handed to k_adj_stream (4 planes of W), which adds their
// closed-form transpose M^T h_bar = h_1 + v_x h_2 + v_y h_3 + (v^2 + eta^2) h_4 together
// with the identity term of the Euler step and the neighbours' contributions.
__global__ __launch_bounds__(kAdjThreads) void k_adj_local(const Consts* __restrict__ c,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ lam,
                                                           const double* __restrict__ af1,
                                                           const double* __restrict__ al1,
                                                           const double* __restrict__ U,
                                                           double* __restrict__ af0, double* __restrict__ al0,
                                                           double* __restrict__ Wout, double* __restrict__ part) {
    __shared__ double sg[kNumLds][kAdjThreads];           // per-thread parameter gradients
    const int nx = ro(c->nx), ny = ro(c->ny);
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    const int tid = (int)threadIdx.x;
    const int64_t plane = (int64_t)nx * ny;
#pragma unroll
    for (int k = 0; k < kNumLds; ++k) sg[k][tid] = 0.0;

    if (x < nx) {
        const int64_t at = (int64_t)y * nx + x;
        const double dt = ro(c->dt), I = ro(c->I), DI = ro(c->DI), D = 2.0;
        // Every load of the cell is issued first, in one burst: at one wave per SIMD each
        // separate wait would be exposed in full.
        const int bcx = ro(c->bc_x), bcy = ro(c->bc_y);
        const int xp = wrap(x + 1, nx, bcx), xm = wrap(x - 1, nx, bcx);
        const int yp = wrap(y + 1, ny, bcy), ym = wrap(y - 1, ny, bcy);
        const int xp2 = wrap(x + 2, nx, bcx), xm2 = wrap(x - 2, nx, bcx);
        const int yp2 = wrap(y + 2, ny, bcy), ym2 = wrap(y - 2, ny, bcy);
        const int64_t row = (int64_t)y * nx;
        const double* Ux = U + plane;
        const double* Uy = U + 2 * plane;
        double v[NV], sbar[NV];
        load_dense(f, plane, at, v);
        load_dense(af1, plane, at, sbar);
        const double lm = lam[at];
        const double beta = al1[at];
        const double ux_xp = Ux[row + xp], ux_xm = Ux[row + xm], uy_xp = Uy[row + xp], uy_xm = Uy[row + xm];
        const double ux_yp = Ux[(int64_t)yp * nx + x], ux_ym = Ux[(int64_t)ym * nx + x];
        const double uy_yp = Uy[(int64_t)yp * nx + x], uy_ym = Uy[(int64_t)ym * nx + x];
        const double l_m2 = lam[row + xm2], l_m1 = lam[row + xm], l_p1 = lam[row + xp], l_p2 = lam[row + xp2];
        const double b_m2 = lam[(int64_t)ym2 * nx + x], b_m1 = lam[(int64_t)ym * nx + x];
        const double b_p1 = lam[(int64_t)yp * nx + x], b_p2 = lam[(int64_t)yp2 * nx + x];
        __builtin_amdgcn_sched_barrier(0);

        Blocks h;
        {
            Blocks sb;
            to_combos(v, sb);
            forward(c->mat, sb, h);
        }
        const Macro m = macro_of(h, DI);
        const double h4 = h.ee[1];

        // velocity gradients (central differences over the boundary rule)
        const double dux_dx = (ux_xp - ux_xm) * ro(c->half_inv_dx);
        const double duy_dx = (uy_xp - uy_xm) * ro(c->half_inv_dx);
        const double dux_dy = (ux_yp - ux_ym) * ro(c->half_inv_dy);
        const double duy_dy = (uy_yp - uy_ym) * ro(c->half_inv_dy);

        // NND derivatives of lambda at this cell, upwind by the sign of u (forward values)
        const double dlx = nnd_upwind(m.ux > 0.0, l_m2, l_m1, lm, l_p1, l_p2) * ro(c->inv_dx);
        const double dly = nnd_upwind(m.uy > 0.0, b_m2, b_m1, lm, b_p1, b_p2) * ro(c->inv_dy);

        // ---- reverse sweep --------------------------------------------------------
#pragma unroll
        for (int i = 0; i < NV; ++i) sbar[i] *= dt;                // adjoint of the source term
        double rb = 0.0, xb = 0.0, yb = 0.0, Tb = 0.0;
        double lamb = beta, dlamb = beta;
        // lambda^{n+1} = lambda + dlambda - dt (u_x D_x lambda + u_y D_y lambda)
        xb -= dt * beta * dlx;
        yb -= dt * beta * dly;

        Blocks hb;
        zero(hb);
        double A8b, A9b;
        {
            // src = -M^-1 g:  g_bar = -M^-T src_bar;  g_k = R_k (h_k - e_k) - A_hat_k, k >= 5
            Blocks gb, e, eb;
            inverse_t(c->mat, sbar, gb);
            equilibrium(m.rho, m.ux, m.uy, m.T, I, e);
            zero(eb);
            const double* R = c->R;
#pragma unroll
            for (int r = 2; r < NEE; ++r) {                            // skip m1, m4
                const double g = -gb.ee[r], d = h.ee[r] - e.ee[r];
                sg[EE_M[r] - 4][tid] = g * d;
                hb.ee[r] = ro(R[EE_M[r]]) * g;
                eb.ee[r] = -ro(R[EE_M[r]]) * g;
            }
#pragma unroll
            for (int r = 1; r < NOE; ++r) {                            // skip m2
                const double g = -gb.oe[r], d = h.oe[r] - e.oe[r];
                sg[OE_M[r] - 4][tid] = g * d;
                hb.oe[r] = ro(R[OE_M[r]]) * g;
                eb.oe[r] = -ro(R[OE_M[r]]) * g;
            }
#pragma unroll
            for (int r = 1; r < NEO; ++r) {                            // skip m3
                const double g = -gb.eo[r], d = h.eo[r] - e.eo[r];
                sg[EO_M[r] - 4][tid] = g * d;
                hb.eo[r] = ro(R[EO_M[r]]) * g;
                eb.eo[r] = -ro(R[EO_M[r]]) * g;
            }
#pragma unroll
            for (int r = 0; r < NOO; ++r) {
                const double g = -gb.oo[r], d = h.oo[r] - e.oo[r];
                sg[OO_M[r] - 4][tid] = g * d;
                hb.oo[r] = ro(R[OO_M[r]]) * g;
                eb.oo[r] = -ro(R[OO_M[r]]) * g;
            }
            A8b = gb.oe[1];          // g_8 = ... - A_8, so A_bar_8 = -g_bar_8 = gb.oe[1]
            A9b = gb.eo[1];
            equilibrium_t(m.rho, m.ux, m.uy, m.T, I, eb, rb, xb, yb, Tb);
        }
        {
            double fb[NV];
            forward_t(c->mat, hb, fb);                       // h_bar_1..4 are still zero here
#pragma unroll
            for (int i = 0; i < NV; ++i) af0[i * plane + at] = fb[i];
        }

        // A_hat_8, A_hat_9 (Eqs. ArtificialA8/ArtificialA9), always differentiated: their
        // derivative with respect to R_8, R_9 does not vanish at R_8 = R_5, R_9 = R_7
        double GX, GY, S_b;
        {
            const double iDI = 1.0 / DI;
            const double X8 = dux_dx - dux_dx * iDI - duy_dy * iDI;
            const double X9 = duy_dy - dux_dx * iDI - duy_dy * iDI;
            const double Sg = duy_dx + dux_dy;
            const double P8 = 4.0 * m.ux * X8 + 2.0 * m.uy * Sg;
            const double P9 = 4.0 * m.uy * X9 + 2.0 * m.ux * Sg;
            const double rT = m.rho * m.T;
            const double a8c = ro(c->a8c), a9c = ro(c->a9c);
            rb += m.T * (A8b * a8c * P8 + A9b * a9c * P9);
            Tb += m.rho * (A8b * a8c * P8 + A9b * a9c * P9);
            const double a8cb = A8b * rT * P8, a9cb = A9b * rT * P9;
            const double P8b = A8b * rT * a8c, P9b = A9b * rT * a9c;
            xb += 4.0 * X8 * P8b + 2.0 * Sg * P9b;
            yb += 2.0 * Sg * P8b + 4.0 * X9 * P9b;
            const double X8b = 4.0 * m.ux * P8b, X9b = 4.0 * m.uy * P9b;
            S_b = 2.0 * m.uy * P8b + 2.0 * m.ux * P9b;
            GX = X8b * (1.0 - iDI) - X9b * iDI;                 // adjoint of d u_x / dx
            GY = -X8b * iDI + X9b * (1.0 - iDI);                // adjoint of d u_y / dy
            // a8c = (R_5 - R_8)/R_5, a9c = (R_7 - R_9)/R_7
            const double R5 = ro(c->R[4]), R7 = ro(c->R[6]), R8 = ro(c->R[7]), R9 = ro(c->R[8]);
            sg[0][tid] += a8cb * R8 / (R5 * R5);
            sg[3][tid] -= a8cb / R5;
            sg[2][tid] += a9cb * R9 / (R7 * R7);
            sg[4][tid] -= a9cb / R7;
        }

        // chemistry: Cochran step and C_i
        if (ro(c->chem)) {
            const double p = m.rho * m.T;
            const double pm = ro(c->m_is_one) ? p : pow(p, ro(c->pm));
            const double pn = ro(c->n_is_one) ? p : pow(p, ro(c->pn));
            const double ar = ro(c->w1) * pm, br = ro(c->w2) * pn, cc = ar + br;
            if (m.T > ro(c->Tig) && lm < 1.0 && cc > 0.0) {
                const double y0 = 1.0 - lm;
                const double E = exp(cc * dt);
                const double den = br * y0 + (cc - br * y0) * E;
                const double y1 = cc * y0 / den;
                const double dl = y0 - y1;
                const double F = dl / dt;
                const double kk = 1.0 / (I * DI * m.T * m.T);
                const double K = ro(c->Q) * F * kk;
                // f^eq = M^-1 f_hat^eq (f_hat^eq evaluated again here)
                double Kb = 0.0, brs = 0.0, bxs = 0.0, bys = 0.0;
                double* feqb = sbar;          // src_bar is not needed after this loop
                {
                    Blocks e, se;
                    equilibrium(m.rho, m.ux, m.uy, m.T, I, e);
                    inverse(c->mat, e, se);
                    double feq[NV];
                    from_combos(se, feq);
#pragma unroll
                    for (int g = 0; g < 3; ++g)
#pragma unroll
                        for (int d = 0; d < 8; ++d) {
                            const int i = 8 * g + d;
                            const double cx = ro(c->vg[g]) * DUX[d] - m.ux, cy = ro(c->vg[g]) * DUY[d] - m.uy;
                            const double bri = -(1.0 + D) * I * m.T + I * (cx * cx + cy * cy) + ro(c->eta2[g]);
                            const double sb_i = sbar[i];
                            feqb[i] = sb_i * bri * K;
                            const double brb = sb_i * feq[i] * K;
                            Kb = fma(sb_i, feq[i] * bri, Kb);
                            brs += brb;
                            bxs += brb * cx;
                            bys += brb * cy;
                        }
                }
                Tb += -(1.0 + D) * I * brs;
                xb += -2.0 * I * bxs;
                yb += -2.0 * I * bys;
                sg[20][tid] = Kb * F * kk;                             // d/dQ
                const double Fb = Kb * ro(c->Q) * kk;
                Tb += Kb * (-2.0 * K / m.T);
                {
                    Blocks eb2;
                    inverse_t(c->mat, feqb, eb2);
                    equilibrium_t(m.rho, m.ux, m.uy, m.T, I, eb2, rb, xb, yb, Tb);
                }
                dlamb += Fb / dt;
                // dl = y0 - y1(y0, cc, b)
                const double q = cc * y0 / (den * den);
                const double dy1_dy0 = cc / den - q * br * (1.0 - E);
                const double dy1_dcc = y0 / den - q * (E + (cc - br * y0) * E * dt);
                const double dy1_db = -q * y0 * (1.0 - E);
                const double y0b = dlamb * (1.0 - dy1_dy0);
                const double ccb = -dlamb * dy1_dcc;
                const double bbar = -dlamb * dy1_db + ccb;
                const double abar = ccb;
                sg[21][tid] = abar * pm;                               // d/domega_1
                sg[22][tid] = bbar * pn;                               // d/domega_2
                const double dpm = ro(c->m_is_one) ? 1.0 : ro(c->pm) * pow(p, ro(c->pm) - 1.0);
                const double dpn = ro(c->n_is_one) ? 1.0 : ro(c->pn) * pow(p, ro(c->pn) - 1.0);
                const double pb = abar * ro(c->w1) * dpm + bbar * ro(c->w2) * dpn;
                rb += pb * m.T;
                Tb += pb * m.rho;
                lamb -= y0b;
            }
        }

        {
            // adjoints of h_1..h_4 from those of rho, u_x, u_y, T (macro_t on zeros)
            Blocks hh, hc;
            zero(hc);
            hh.ee[1] = h4;
            macro_t(hh, m, DI, rb, xb, yb, Tb, hc);
            Wout[3 * plane + at] = hc.ee[0];
            Wout[4 * plane + at] = hc.oe[0];
            Wout[5 * plane + at] = hc.eo[0];
            Wout[6 * plane + at] = hc.ee[1];
        }
        al0[at] = lamb;
        Wout[at] = GX;
        Wout[plane + at] = GY;
        Wout[2 * plane + at] = S_b;
    }
    __syncthreads();
    // fixed-order reduction of the per-thread gradients: parameter k by thread k
    // (R_1..R_4 never receive a contribution: their moments carry g = 0)
    if (tid < kNumGrad) {
        double t = 0.0;
        const int k = tid - 4;
        if (k >= 0)
            for (int j = 0; j < kAdjThreads; ++j) t += sg[k][j];
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        const int64_t nb = (int64_t)gridDim.x * gridDim.y;
        part[tid * nb + b] = t;
    }
}

__global__ __launch_bounds__(kAdjThreads, 2) void k_adj_stream(const Consts* __restrict__ c,
                                                            const double* __restrict__ f,
                                                            const double* __restrict__ lam,
                                                            const double* __restrict__ af1,
                                                            const double* __restrict__ al1,
                                                            const double* __restrict__ U,
                                                            const double* __restrict__ W,
                                                            double* __restrict__ af0, double* __restrict__ al0) {
    const int nx = c->nx, ny = c->ny;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const int64_t plane = (int64_t)nx * ny, at = (int64_t)y * nx + x, row = (int64_t)y * nx;
    const double dt = c->dt;
    const AxisAdj AX = axis_adj(x, nx, c->bc_x);
    const AxisAdj AY = axis_adj(y, ny, c->bc_y);
    int64_t ox[5], oy[5];
    uint32_t bx[5], by[5];                 // the same as byte offsets within a plane
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        ox[t] = row + AX.pos[t];
        oy[t] = (int64_t)AY.pos[t] * nx + x;
        bx[t] = (uint32_t)ox[t] * 8u;
        by[t] = (uint32_t)oy[t] * 8u;
    }
    const uint32_t bc = (uint32_t)at * 8u;
    // planes through buffer resources: the plane offset is a scalar operand
    const Soa Fb = soa(f, plane), Ab = soa(af1, plane), Ob = soa(af0, plane);
    const uint32_t pb = opaque(Fb.plane_bytes);

    // neighbours' A_hat terms: adjoint of this cell's velocity
    double uxn = 0.0, uyn = 0.0;
    {
        const double* Wx = W;               // adjoint of d u_x/dx at the owning cell
        const double* Wy = W + plane;       // adjoint of d u_y/dy
        const double* Ws = W + 2 * plane;   // adjoint of (d u_y/dx + d u_x/dy)
        const double hx = c->half_inv_dx, hy = c->half_inv_dy;
        // cells whose +1 neighbour along an axis is this one, and whose -1 neighbour is
        auto pre = [](int x, int n, int bc, int& j1, double& w1, int& j2, double& w2, int side) {
            if (bc == 0) {
                j1 = wrap(x - side, n, 0);
                w1 = 1.0;
                j2 = x;
                w2 = 0.0;
            } else {
                j1 = x - side;
                w1 = (j1 >= 0 && j1 < n) ? 1.0 : 0.0;
                j1 = j1 < 0 ? 0 : (j1 >= n ? n - 1 : j1);
                j2 = x;
                w2 = (side > 0 ? x == n - 1 : x == 0) ? 1.0 : 0.0;
            }
        };
        int j1, j2;
        double w1, w2;
        pre(x, nx, c->bc_x, j1, w1, j2, w2, +1);
        uxn += hx * (w1 * Wx[row + j1] + w2 * Wx[row + j2]);
        uyn += hx * (w1 * Ws[row + j1] + w2 * Ws[row + j2]);
        pre(x, nx, c->bc_x, j1, w1, j2, w2, -1);
        uxn -= hx * (w1 * Wx[row + j1] + w2 * Wx[row + j2]);
        uyn -= hx * (w1 * Ws[row + j1] + w2 * Ws[row + j2]);
        pre(y, ny, c->bc_y, j1, w1, j2, w2, +1);
        uxn += hy * (w1 * Ws[(int64_t)j1 * nx + x] + w2 * Ws[(int64_t)j2 * nx + x]);
        uyn += hy * (w1 * Wy[(int64_t)j1 * nx + x] + w2 * Wy[(int64_t)j2 * nx + x]);
        pre(y, ny, c->bc_y, j1, w1, j2, w2, -1);
        uxn -= hy * (w1 * Ws[(int64_t)j1 * nx + x] + w2 * Ws[(int64_t)j2 * nx + x]);
        uyn -= hy * (w1 * Wy[(int64_t)j1 * nx + x] + w2 * Wy[(int64_t)j2 * nx + x]);
    }
    const double rho = U[at], ux = U[plane + at], uy = U[2 * plane + at];
    const double cx_n = uxn / rho, cy_n = uyn / rho;
    // adjoints of the conserved moments h_1..h_4 of this cell (from k_adj_local)
    const double hb1 = W[3 * plane + at], hb2 = W[4 * plane + at], hb3 = W[5 * plane + at],
                 hb4 = W[6 * plane + at];

    // transposed streaming of f: adv_i = v_ix D_x f_i + v_iy D_y f_i, adjoint -dt a_i.  The
    // loads of plane i+1's stencils are issued before plane i is differenced (the scheduling
    // barrier keeps them there), so each plane's memory latency hides behind the previous
    // plane's arithmetic; all 24 updates are formed before any store into af0, which would
    // otherwise hold the following loads behind it.
    // Where the wave's 64 cells and two more on each side lie inside the row, the x-stencils
    // of f and a^{n+1} are the centre values of the neighbouring lanes plus one halo load
    // each (the two cells beyond each end of the wave), instead of five gathers each.
    struct PlaneLoads {
        double fx[5], ax[5], fy[5], ay[5];   // f and a^{n+1} at offsets -2..2 along x and y
        double hf, ha;                       // the halo values of f and a^{n+1} (lane moves)
    };
    const int lane = (int)(threadIdx.x & 63u);
    const int x0 = x - lane;
    const bool by_lanes = x0 >= 2 && x0 + 66 <= nx;      // uniform per wave
    const uint32_t bh = (uint32_t)(row + (lane < 32 ? (lane == 0 ? x0 - 2 : x0 - 1) : (lane == 63 ? x0 + 65 : x0 + 64))) * 8u;
    __shared__ double upd_s[NV][kAdjThreads];   // this thread's 24 updates (own slots only)
    auto run = [&](auto from_lanes) {
        constexpr bool XL = decltype(from_lanes)::value;
        auto load_plane = [&](int i, PlaneLoads& p) {
            const uint32_t so = (uint32_t)i * pb;
            const int d = i & 7;
            if (DUX[d] != 0) {
                if (XL) {
                    p.fx[2] = ld(Fb, so, bc);
                    p.ax[2] = ld(Ab, so, bc);
                    p.hf = ld(Fb, so, bh);
                    p.ha = ld(Ab, so, bh);
                } else {
#pragma unroll
                    for (int t = 0; t < 5; ++t) {
                        p.fx[t] = ld(Fb, so, bx[t]);
                        p.ax[t] = ld(Ab, so, bx[t]);
                    }
                }
            }
            if (DUY[d] != 0) {
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    p.fy[t] = ld(Fb, so, by[t]);
                    p.ay[t] = ld(Ab, so, by[t]);
                }
            }
        };
        PlaneLoads cur, nxt;
        load_plane(0, cur);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i + 1 < NV) load_plane(i + 1, nxt);
            __builtin_amdgcn_sched_barrier(0);
            const int g = i / 8, d = i % 8;
            const double vg = ro(c->vg[g]);
            double acc = 0.0, a_c = 0.0;          // a_c: a^{n+1} of this cell (offset 0 of a stencil)
            if (DUX[d] != 0) {
                if (XL) {
                    const XNeighbours nf = x_neighbours(cur.fx[2], cur.hf);
                    const XNeighbours na = x_neighbours(cur.ax[2], cur.ha);
                    cur.fx[0] = nf.m2;
                    cur.fx[1] = nf.m1;
                    cur.fx[3] = nf.p1;
                    cur.fx[4] = nf.p2;
                    cur.ax[0] = na.m2;
                    cur.ax[1] = na.m1;
                    cur.ax[3] = na.p1;
                    cur.ax[4] = na.p2;
                }
                double av[5];
#pragma unroll
                for (int t = 0; t < 5; ++t) av[t] = AX.val[t] * cur.ax[t];
                acc += vg * DUX[d] * ro(c->inv_dx) * nnd_t(AX, cur.fx, av, DUX[d]);
                a_c = cur.ax[2];
            }
            if (DUY[d] != 0) {
                double av[5];
#pragma unroll
                for (int t = 0; t < 5; ++t) av[t] = AY.val[t] * cur.ay[t];
                acc += vg * DUY[d] * ro(c->inv_dy) * nnd_t(AY, cur.fy, av, DUY[d]);
                a_c = cur.ay[2];
            }
            const double vx = vg * DUX[d], vy = vg * DUY[d];
            const double mt = hb1 + vx * hb2 + vy * hb3 + (vx * vx + vy * vy + ro(c->eta2[g])) * hb4;
            upd_s[i][threadIdx.x] = a_c - dt * acc + (vx - ux) * cx_n + (vy - uy) * cy_n + mt;
            cur = nxt;
        }
    };
    if (by_lanes)
        run(std::true_type{});
    else
        run(std::false_type{});

    // transposed advection of lambda: D lambda at cell j is upwinded by the sign of u(j)
    auto lam_t = [&](const AxisAdj& A, const int64_t o[5], const double* __restrict__ Ua, double inv) {
        double lv[5], ap[5], an[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            lv[t] = lam[o[t]];
            const double u = Ua[o[t]];
            const double adj = A.val[t] * (-dt * al1[o[t]] * u);
            ap[t] = u > 0.0 ? adj : 0.0;
            an[t] = u > 0.0 ? 0.0 : adj;
        }
        return inv * (nnd_t(A, lv, ap, +1) + nnd_t(A, lv, an, -1));
    };
    const double lb = lam_t(AX, ox, U + plane, c->inv_dx) + lam_t(AY, oy, U + 2 * plane, c->inv_dy);
    // add the collision part that k_adj_local wrote: 24 loads in one burst, then the stores
    double o[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) o[i] = ld(Ob, (uint32_t)i * pb, bc);
#pragma unroll
    for (int i = 0; i < NV; ++i) st(Ob, (uint32_t)i * pb, bc, o[i] + upd_s[i][threadIdx.x]);
    al0[at] += lb;
}

__global__ __launch_bounds__(kAdjThreads) void k_grad_final(const double* __restrict__ part, int64_t nb,
                                                            double* __restrict__ grad) {
    // one work-group per parameter, fixed summation order
    __shared__ double sh[4];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) s += part[k * nb + b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
        grad[k] += t;
    }
}

// dL/df for L = sum_cells sum_{k=5..24} Delta_k^2, and per-work-group partial sums of L
__global__ __launch_bounds__(kAdjThreads) void k_tne_loss(const Consts* __restrict__ c,
                                                          const double* __restrict__ f,
                                                          double* __restrict__ gf, double* __restrict__ part) {
    __shared__ double sh[4 * kNumGrad];
    const int nx = c->nx, ny = c->ny;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    const int64_t plane = (int64_t)nx * ny;
    double acc[kNumGrad];
#pragma unroll
    for (int k = 0; k < kNumGrad; ++k) acc[k] = 0.0;
    if (x < nx) {
        const int64_t at = (int64_t)y * nx + x;
        double v[NV];
        load_dense(f, plane, at, v);
        Blocks s, h, e, hb, eb;
        to_combos(v, s);
        forward(c->mat, s, h);
        const Macro m = macro_of(h, c->DI);
        equilibrium(m.rho, m.ux, m.uy, m.T, c->I, e);
        zero(hb);
        zero(eb);
        double L = 0.0;
#pragma unroll
        for (int r = 2; r < NEE; ++r) {
            const double d = h.ee[r] - e.ee[r];
            L = fma(d, d, L);
            hb.ee[r] = 2.0 * d;
            eb.ee[r] = -2.0 * d;
        }
#pragma unroll
        for (int r = 1; r < NOE; ++r) {
            const double d = h.oe[r] - e.oe[r];
            L = fma(d, d, L);
            hb.oe[r] = 2.0 * d;
            eb.oe[r] = -2.0 * d;
        }
#pragma unroll
        for (int r = 1; r < NEO; ++r) {
            const double d = h.eo[r] - e.eo[r];
            L = fma(d, d, L);
            hb.eo[r] = 2.0 * d;
            eb.eo[r] = -2.0 * d;
        }
#pragma unroll
        for (int r = 0; r < NOO; ++r) {
            const double d = h.oo[r] - e.oo[r];
            L = fma(d, d, L);
            hb.oo[r] = 2.0 * d;
            eb.oo[r] = -2.0 * d;
        }
        acc[0] = L;
        if (gf) {
            double rb = 0.0, xb = 0.0, yb = 0.0, Tb = 0.0;
            equilibrium_t(m.rho, m.ux, m.uy, m.T, c->I, eb, rb, xb, yb, Tb);
            macro_t(h, m, c->DI, rb, xb, yb, Tb, hb);
            double fb[NV];
            forward_t(c->mat, hb, fb);
#pragma unroll
            for (int i = 0; i < NV; ++i) gf[i * plane + at] = fb[i];
        }
    }
    block_reduce_grad(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(kAdjThreads) void k_sum_final(const double* __restrict__ part, int64_t nb,
                                                           double* __restrict__ out) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
        *out = t;
    }
}

// adjoint of f = M^-1 f_hat^eq(rho, u, T): dL/d(rho, u_x, u_y, T) from dL/df
__global__ __launch_bounds__(kAdjThreads) void k_adj_init(const Consts* __restrict__ c,
                                                          const double* __restrict__ rho,
                                                          const double* __restrict__ ux,
                                                          const double* __restrict__ uy,
                                                          const double* __restrict__ T,
                                                          const double* __restrict__ af, double* __restrict__ arho,
                                                          double* __restrict__ aux, double* __restrict__ auy,
                                                          double* __restrict__ aT) {
    const int nx = c->nx, ny = c->ny;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const int64_t plane = (int64_t)nx * ny, at = (int64_t)y * nx + x;
    double a[NV];
    load_dense(af, plane, at, a);
    Blocks eb;
    inverse_t(c->mat, a, eb);
    double rb = 0.0, xb = 0.0, yb = 0.0, Tb = 0.0;
    equilibrium_t(rho[at], ux[at], uy[at], T[at], c->I, eb, rb, xb, yb, Tb);
    arho[at] = rb;
    aux[at] = xb;
    auy[at] = yb;
    aT[at] = Tb;
}

dim3 adj_grid(int nx, int ny) { return dim3((nx + kAdjThreads - 1) / kAdjThreads, ny); }

// scratch: U (3 planes), W (7 planes), partials (27 per work-group)
lbkm_status ensure_adjoint_scratch(lbkm_ctx* ctx) {
    const int64_t cells = (int64_t)ctx->grid.nx * ctx->grid.ny;
    const dim3 g = adj_grid(ctx->grid.nx, ctx->grid.ny);
    const int64_t nb = (int64_t)g.x * g.y;
    const int64_t need = 10 * cells + kNumGrad * nb;
    if (ctx->adj_scratch && ctx->adj_scratch_n >= need) return LBKM_OK;
    if (ctx->adj_scratch) (void)hipFree(ctx->adj_scratch);
    ctx->adj_scratch = nullptr;
    ctx->adj_scratch_n = 0;
    hipError_t e = hipMalloc((void**)&ctx->adj_scratch, sizeof(double) * need);
    if (e != hipSuccess) return hip_fail(ctx, e, "adjoint scratch allocation");
    ctx->adj_scratch_n = need;
    return LBKM_OK;
}

// the checks of every adjoint entry point (no allocation)
lbkm_status adj_check(lbkm_ctx* ctx) {
    if (!ctx) return LBKM_EINVAL;
    if ((int64_t)NV * ctx->grid.nx * ctx->grid.ny * 8 > 0xFFFFFFFFll)
        return fail(ctx, LBKM_EINVAL, "the adjoint needs a dense state below 4 GiB");
    if (ctx->batched) return fail(ctx, LBKM_ESTATE, "not available on a batched context");
    if (!ctx->bound) return fail(ctx, LBKM_ESTATE, "buffers not bound");
    if (!ctx->params) return fail(ctx, LBKM_ESTATE, "parameters not set");
    return LBKM_OK;
}

lbkm_status adj_ready(lbkm_ctx* ctx) {
    const lbkm_status st = adj_check(ctx);
    return st != LBKM_OK ? st : ensure_adjoint_scratch(ctx);
}

// Scratch of the allocation-free loss (lbkm_tne_loss_noalloc): the per-work-group partial
// sums live in this file-scope device array, one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it only stands
// for the symbol): it looks up each device's address once, with that device current, and
// passes that address.
constexpr int64_t kNoAllocPartials = 65536;          // 512 KiB
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocPartials];
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];

// address of `scratch` on the current device (looked up on the first call per device)
hipError_t scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (g_scratch_err[dev] == hipSuccess) g_scratch_ptr[dev] = static_cast<double*>(p);
    });
    if (g_scratch_err[dev] != hipSuccess) return g_scratch_err[dev];
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

// Looks up the allocation-free loss's scratch address on the current device (called when a
// context's device tables are set up, so that the lookup happens outside any stream capture).
hipError_t setup_noalloc_scratch() {
    double* p = nullptr;
    return scratch_address(&p);
}

}  // namespace lbkm

using namespace lbkm;

extern "C" {

lbkm_status lbkm_adjoint_step(lbkm_ctx* ctx, const double* f_n, const double* lam_n, const double* af_np1,
                              const double* alam_np1, double* af_n, double* alam_n, double* grad_params) {
    lbkm_status st = adj_ready(ctx);
    if (st != LBKM_OK) return st;
    if (ctx->h.srt) return fail(ctx, LBKM_ESTATE, "the adjoint step covers the MRT form only");
    if (ctx->rk != 1) return fail(ctx, LBKM_ESTATE, "the adjoint step covers forward Euler only");
    for (int k = 0; k < 4; ++k)
        if (ctx->h.wall[k] != kWallNone)
            return fail(ctx, LBKM_ESTATE, "the adjoint step covers periodic and outflow boundaries only");
    if (!f_n || !lam_n || !af_np1 || !alam_np1 || !af_n || !alam_n || !grad_params)
        return fail(ctx, LBKM_EINVAL, "NULL argument");
    if (af_n == af_np1 || alam_n == alam_np1)
        return fail(ctx, LBKM_EINVAL, "the level-n adjoint must not alias the level-(n+1) adjoint");
    const int nx = ctx->grid.nx, ny = ctx->grid.ny;
    const int64_t cells = (int64_t)nx * ny;
    const dim3 g = adj_grid(nx, ny);
    const int64_t nb = (int64_t)g.x * g.y;
    double* U = ctx->adj_scratch;
    double* W = U + 3 * cells;
    double* part = W + 7 * cells;
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_adj_macro, g, dim3(kAdjThreads), 0, s, ctx->d, f_n, U);
    hipLaunchKernelGGL(k_adj_local, g, dim3(kAdjThreads), 0, s, ctx->d, f_n, lam_n, af_np1, alam_np1, U, af_n,
                       alam_n, W, part);
    hipLaunchKernelGGL(k_adj_stream, g, dim3(kAdjThreads), 0, s, ctx->d, f_n, lam_n, af_np1, alam_np1, U, W, af_n,
                       alam_n);
    hipLaunchKernelGGL(k_grad_final, dim3(kNumGrad), dim3(kAdjThreads), 0, s, part, nb, grad_params);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "adjoint step kernels");
}

lbkm_status lbkm_adjoint_init(lbkm_ctx* ctx, const double* rho, const double* ux, const double* uy, const double* T,
                              const double* af, double* arho, double* aux, double* auy, double* aT) {
    lbkm_status st = adj_ready(ctx);
    if (st != LBKM_OK) return st;
    if (!rho || !ux || !uy || !T || !af || !arho || !aux || !auy || !aT) return fail(ctx, LBKM_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_adj_init, adj_grid(ctx->grid.nx, ctx->grid.ny), dim3(kAdjThreads), 0, ctx->stream, ctx->d,
                       rho, ux, uy, T, af, arho, aux, auy, aT);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "adjoint init kernel");
}

lbkm_status lbkm_tne_loss(lbkm_ctx* ctx, const double* f, double* loss_dev, double* grad_f) {
    lbkm_status st = adj_ready(ctx);
    if (st != LBKM_OK) return st;
    if (!f || !loss_dev) return fail(ctx, LBKM_EINVAL, "NULL argument");
    const int nx = ctx->grid.nx, ny = ctx->grid.ny;
    const int64_t cells = (int64_t)nx * ny;
    const dim3 g = adj_grid(nx, ny);
    double* part = ctx->adj_scratch + 10 * cells;
    hipLaunchKernelGGL(k_tne_loss, g, dim3(kAdjThreads), 0, ctx->stream, ctx->d, f, grad_f, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kAdjThreads), 0, ctx->stream, part, (int64_t)g.x * g.y, loss_dev);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "loss kernels");
}

lbkm_status lbkm_tne_loss_noalloc(lbkm_ctx* ctx, const double* f, double* loss_dev, double* grad_f) {
    lbkm_status st = adj_check(ctx);
    if (st != LBKM_OK) return st;
    if (!f || !loss_dev) return fail(ctx, LBKM_EINVAL, "NULL argument");
    const int nx = ctx->grid.nx, ny = ctx->grid.ny;
    const dim3 g = adj_grid(nx, ny);
    const int64_t nb = (int64_t)g.x * g.y;
    if (nb > kNoAllocPartials)
        return fail(ctx, LBKM_EINVAL,
                    "grid too large for the allocation-free loss: it needs ceil(nx/256) * ny partial sums, "
                    "at most 65536");
    double* part = nullptr;
    hipError_t e = scratch_address(&part);
    if (e != hipSuccess) return hip_fail(ctx, e, "scratch address of the allocation-free loss");
    hipLaunchKernelGGL(k_tne_loss, g, dim3(kAdjThreads), 0, ctx->stream, ctx->d, f, grad_f, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kAdjThreads), 0, ctx->stream, part, nb, loss_dev);
    e = hipGetLastError();
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "loss kernels");
}

}  // extern "C"
