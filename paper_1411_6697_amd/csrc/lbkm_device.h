// Device-side building blocks of the MRT-LBKM step (gfx950, float64).
//
// The per-cell arithmetic is expressed in the mirror-symmetry basis of the velocity set
// (see lbkm_internal.h): f_hat = M f costs 36 additions plus 162 multiply-adds instead of
// 576, and M^-1 g the same.
#pragma once

#include <hip/hip_runtime.h>

#include "lbkm_internal.h"

namespace lbkm {

// A read of constant data (the constants block, per-instance rates) through the constant
// address space.  Kernels never write these, and such loads stay scalar loads even after
// stores or fences that the compiler cannot separate from them (LDS stores through a
// generic pointer, the batch kernel's device-scope fences); through a plain pointer they
// would turn into vector loads, each a wait that drains all loads in flight.
template <typename T>
__device__ __forceinline__ T ro(const T& v) {
    return *(const __attribute__((address_space(4))) T*)(const void*)&v;
}

// direction table inside a group
__device__ constexpr int DUX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int DUY[8] = {0, 1, 0, -1, 1, 1, -1, -1};

struct Blocks {
    double ee[NEE], oe[NOE], eo[NEO], oo[NOO];
};

// Symmetric combinations s = P f of the 24 values of one cell.
__device__ __forceinline__ void to_combos(const double f[NV], Blocks& s) {
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const double a0 = f[8 * g + 0], a1 = f[8 * g + 1], a2 = f[8 * g + 2], a3 = f[8 * g + 3];
        const double d0 = f[8 * g + 4], d1 = f[8 * g + 5], d2 = f[8 * g + 6], d3 = f[8 * g + 7];
        const double t1 = d0 + d2, t2 = d1 + d3, t3 = d0 - d2, t4 = d1 - d3;
        s.ee[3 * g + 0] = a0 + a2;
        s.ee[3 * g + 1] = a1 + a3;
        s.ee[3 * g + 2] = t1 + t2;
        s.oe[2 * g + 0] = a0 - a2;
        s.oe[2 * g + 1] = t3 - t4;
        s.eo[2 * g + 0] = a1 - a3;
        s.eo[2 * g + 1] = t3 + t4;
        s.oo[g] = t1 - t2;
    }
}

// f from combination-space values (the 1/2, 1/4 factors are already in the C blocks).
__device__ __forceinline__ void from_combos(const Blocks& s, double f[NV]) {
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const double e1 = s.ee[3 * g + 0], e2 = s.ee[3 * g + 1], e3 = s.ee[3 * g + 2];
        const double o1 = s.oe[2 * g + 0], o2 = s.oe[2 * g + 1];
        const double q1 = s.eo[2 * g + 0], q2 = s.eo[2 * g + 1];
        const double r1 = s.oo[g];
        f[8 * g + 0] = e1 + o1;
        f[8 * g + 2] = e1 - o1;
        f[8 * g + 1] = e2 + q1;
        f[8 * g + 3] = e2 - q1;
        const double u1 = e3 + r1, u2 = e3 - r1, w1 = o2 + q2, w2 = q2 - o2;
        f[8 * g + 4] = u1 + w1;
        f[8 * g + 5] = u2 + w2;
        f[8 * g + 6] = u1 - w1;
        f[8 * g + 7] = u2 - w2;
    }
}

// Make the (scalar) pointer p depend on the N values y: loads through p cannot be issued
// before y is computed.
template <int N>
__device__ __forceinline__ void tie_after(const double*& p, const double* y) {
    if constexpr (N == 9)
        asm volatile("" : "+s"(p) : "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]), "v"(y[4]), "v"(y[5]),
                     "v"(y[6]), "v"(y[7]), "v"(y[8]));
    else if constexpr (N == 6)
        asm volatile("" : "+s"(p) : "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]), "v"(y[4]), "v"(y[5]));
    else
        asm volatile("" : "+s"(p) : "v"(y[0]), "v"(y[1]), "v"(y[2]));
}

// y = A x with A stored column-major (At[k][r] = A[r][k]).  The loop runs over columns:
// the N accumulators are independent multiply-add chains, and each column's N constants
// (one scalar load) are consumed right after they arrive, so few of the 324 matrix entries
// are held in scalar registers at a time.  Each y[r] still sums over k in increasing order.
template <int N>
__device__ __forceinline__ void matvec(const double (*At)[N], const double* x, double* y) {
    // A fresh (opaque) copy of the matrix address per product: the inverse blocks are used
    // twice per cell, and letting the compiler share their loads keeps 162 doubles in
    // scalar registers between the two uses (and spills them).
    // The copy is read through the constant address space, which the kernel never writes,
    // so the loads stay scalar.
    // Tying the copy to the input vector also keeps these loads from being hoisted ahead of
    // the code that produces x, and each column's address is tied to all results of the
    // previous column, so one column (<= 18 scalar registers) is in flight at a time.
    asm volatile("" : "+s"(At) : "v"(x[N - 1]));
    typedef const __attribute__((address_space(4))) double cdouble;
    cdouble* A = (cdouble*)(const void*)At;
#pragma unroll
    for (int r = 0; r < N; ++r) y[r] = A[r] * x[0];
#pragma unroll
    for (int k = 1; k < N; ++k) {
        const double* col = At[k];
        tie_after<N>(col, y);
        cdouble* Ak = (cdouble*)(const void*)col;
#pragma unroll
        for (int r = 0; r < N; ++r) y[r] = fma(Ak[r], x[k], y[r]);
    }
}

// f_hat = M f in block order (M from global constants or from an LDS copy)
__device__ __forceinline__ void forward(const Mats& M, const Blocks& s, Blocks& h) {
    matvec<NEE>(M.BEE, s.ee, h.ee);
    matvec<NOE>(M.BOE, s.oe, h.oe);
    matvec<NEO>(M.BEO, s.eo, h.eo);
    matvec<NOO>(M.BOO, s.oo, h.oo);
}
__device__ __forceinline__ void forward(const Consts* __restrict__ c, const Blocks& s, Blocks& h) {
    forward(c->mat, s, h);
}

// combination values of M^-1 g
__device__ __forceinline__ void inverse(const Mats& M, const Blocks& g, Blocks& s) {
    matvec<NEE>(M.CEE, g.ee, s.ee);
    matvec<NOE>(M.COE, g.oe, s.oe);
    matvec<NEO>(M.CEO, g.eo, s.eo);
    matvec<NOO>(M.COO, g.oo, s.oo);
}
__device__ __forceinline__ void inverse(const Consts* __restrict__ c, const Blocks& g, Blocks& s) {
    inverse(c->mat, g, s);
}

// Equilibrium moments f_hat^eq (Sec. II closed forms, factor T in entries 14 and 16 as
// Eq. moment7 requires), D = 2, in block order.
__device__ __forceinline__ void equilibrium(double rho, double ux, double uy, double T, double I,
                                            Blocks& e) {
    const double D = 2.0;
    const double u2 = ux * ux + uy * uy;
    const double a2 = (D + I + 2.0) * T + u2;
    const double a4 = (D + I + 4.0) * T + u2;
    const double c10 = u2 * u2 + (D + 2.0) * (D + I + 4.0) * T * T + (2.0 * D + I + 8.0) * u2 * T;
    const double c11 = u2 + (D + 3.0 * I + 2.0) * T;
    const double rT = rho * T, rIT = rho * I * T;
    // EE: m1 m4 m5 m7 m14 m16 m17 m19 m20
    e.ee[0] = rho;
    e.ee[1] = rho * ((D + I) * T + u2);
    e.ee[2] = rho * (T + ux * ux);
    e.ee[3] = rho * (T + uy * uy);
    e.ee[4] = rho * a2 * T + rho * ux * ux * a4;
    e.ee[5] = rho * a2 * T + rho * uy * uy * a4;
    e.ee[6] = rIT * T + rIT * ux * ux;
    e.ee[7] = rIT * T + rIT * uy * uy;
    e.ee[8] = rIT * (u2 + (D + 3.0 * I) * T);
    // OE: m2 m8 m10 m12 m21 m23
    e.oe[0] = rho * ux;
    e.oe[1] = rho * ux * a2;
    e.oe[2] = 3.0 * rT * ux + rho * ux * ux * ux;
    e.oe[3] = rT * ux + rho * ux * uy * uy;
    e.oe[4] = rho * ux * c10;
    e.oe[5] = rIT * ux * c11;
    // EO: m3 m9 m11 m13 m22 m24
    e.eo[0] = rho * uy;
    e.eo[1] = rho * uy * a2;
    e.eo[2] = rT * uy + rho * ux * ux * uy;
    e.eo[3] = 3.0 * rT * uy + rho * uy * uy * uy;
    e.eo[4] = rho * uy * c10;
    e.eo[5] = rIT * uy * c11;
    // OO: m6 m15 m18
    e.oo[0] = rho * ux * uy;
    e.oo[1] = rho * ux * uy * a4;
    e.oo[2] = rIT * ux * uy;
}

// R_k of each block slot (0-based moment indices, see lbkm_internal.h)
__device__ constexpr int EE_M[NEE] = {0, 3, 4, 6, 13, 15, 16, 18, 19};
__device__ constexpr int OE_M[NOE] = {1, 7, 9, 11, 20, 22};
__device__ constexpr int EO_M[NEO] = {2, 8, 10, 12, 21, 23};
__device__ constexpr int OO_M[NOO] = {5, 14, 17};

// macroscopic variables from the conserved moments (Eqs. moment1-moment3)
struct Macro {
    double rho, ux, uy, T;
};

__device__ __forceinline__ Macro macro_of(const Blocks& h, double DI) {
    Macro m;
    m.rho = h.ee[0];
    m.ux = h.oe[0] / m.rho;
    m.uy = h.eo[0] / m.rho;
    m.T = (h.ee[1] / m.rho - m.ux * m.ux - m.uy * m.uy) / DI;
    return m;
}

// Velocity of a cell from its 24 values, summed plane by plane in plane order (rho, j_x,
// j_y of Eqs. moment1-moment2).  The inputs of A_hat are the neighbours' velocities; every
// kernel forms them with this same sequence of operations, either from stored values
// (k_velocity) or while it writes a new state, so they agree bitwise.
struct VelAcc {
    double r = 0.0, jx = 0.0, jy = 0.0;
};
__device__ __forceinline__ void vel_add(VelAcc& a, double vg, int d, double v) {
    a.r += v;
    if (DUX[d] != 0) a.jx = fma(DUX[d] > 0 ? vg : -vg, v, a.jx);
    if (DUY[d] != 0) a.jy = fma(DUY[d] > 0 ? vg : -vg, v, a.jy);
}
__device__ __forceinline__ void vel_add(VelAcc& a, const Consts* __restrict__ c, int g, int d, double v) {
    vel_add(a, ro(c->vg[g]), d, v);
}

// NND differences h_{j+1/2} - h_{j-1/2} (to be divided by the spacing), Zhang 1988,
// flux-split minmod form.  Positive speed uses j-2..j+1, negative speed j-1..j+2.
// With h_{j+1/2} = f_j + mm(f_j - f_{j-1}, f_{j+1} - f_j)/2 and its neighbour, the
// difference is the centred jump plus half the change of the limited slopes.
// minmod(d, s), the argument of smaller magnitude if both have the same strict sign and
// else 0, is the median of (d, s, 0), i.e. s clamped to the interval between 0 and d.
// Both limited slopes of one difference take the jump d as an argument, so the bounds
// min(d, 0) and max(d, 0) are formed once: six FP64 min/max operations for the two slopes
// instead of eight, branch-free, and the result is one of the arguments exactly.
__device__ __forceinline__ double clamp_between(double s, double lo, double hi) {
    return fmin(fmax(s, lo), hi);
}
__device__ __forceinline__ double nnd_pos(double fm2, double fm1, double f0, double fp1) {
    const double d = f0 - fm1, lo = fmin(d, 0.0), hi = fmax(d, 0.0);
    return fma(0.5, clamp_between(fp1 - f0, lo, hi) - clamp_between(fm1 - fm2, lo, hi), d);
}
__device__ __forceinline__ double nnd_neg(double fm1, double f0, double fp1, double fp2) {
    const double d = fp1 - f0, lo = fmin(d, 0.0), hi = fmax(d, 0.0);
    return fma(-0.5, clamp_between(fp2 - fp1, lo, hi) - clamp_between(f0 - fm1, lo, hi), d);
}

// The NND difference upwinded by the sign of a velocity that varies from cell to cell
// (u > 0: the positive-speed form, else the negative one), from the five stencil values.
// Both forms are evaluated and one is selected, so the caller loads the whole stencil
// unconditionally: a wave whose lanes differ in that sign then waits for one set of loads,
// not for one set per side.
__device__ __forceinline__ double nnd_upwind(bool pos, double fm2, double fm1, double f0, double fp1,
                                             double fp2) {
    const double a = nnd_pos(fm2, fm1, f0, fp1);
    const double b = nnd_neg(fm1, f0, fp1, fp2);
    return pos ? a : b;
}

// Lane moves of a double across the wave (DPP): lane i receives lane i-1's value
// (from_left) or lane i+1's (from_right).  The end lane, which has no source lane, is not
// written and keeps `edge`.
__device__ __forceinline__ double from_left(double v, double edge) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);   // 0x138: wave_shr:1
}
__device__ __forceinline__ double from_right(double v, double edge) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);   // 0x130: wave_shl:1
}

// The x-neighbours at offsets -2, -1, +1, +2 of a row of 64 cells held one per lane
// (centre value f0), with h the lane's halo value: x0-2 on lane 0, x0-1 on lanes 1..31,
// x0+64 on lanes 32..62, x0+65 on lane 63 (x0 the row's first cell, positions under the
// boundary rule).  Each neighbour is one lane move whose end lane keeps the halo value it
// needs: -1 on lane 0 is x0-1 (lane 1's halo), -2 on lane 1 is lane 0's -1, -2 on lane 0
// is its own halo, and the same mirrored at lane 63.
struct XNeighbours {
    double m2, m1, p1, p2;
};
__device__ __forceinline__ XNeighbours x_neighbours(double f0, double h) {
    // every lane takes part in the halo load (left to itself the compiler would load it on
    // the end lanes only, behind a branch and a wait per plane)
    asm("" : "+v"(h));
    XNeighbours n;
    n.m1 = from_left(f0, from_right(h, 0.0));
    n.p1 = from_right(f0, from_left(h, 0.0));
    n.m2 = from_left(n.m1, h);
    n.p2 = from_right(n.p1, h);
    return n;
}

// Cochran increment of lambda over one step, p frozen (exact solution of the Bernoulli
// equation d(1-lambda)/dt = -(1-lambda)(a + b lambda)); zero unless T > T_ig,
// lambda < 1 and a + b > 0.  CHEM = false compiles the reaction out (omega1 = omega2 = 0);
// GEXP = false assumes m = n = 1 (the paper's choice), so p^m = p without a pow call.
template <bool CHEM = true, bool GEXP = true>
__device__ __forceinline__ double cochran(const Consts* __restrict__ c, double lam, double p, double T) {
    if (!CHEM || !ro(c->chem)) return 0.0;
    double a, b;
    if (GEXP) {
        a = ro(c->w1) * (ro(c->m_is_one) ? p : pow(p, ro(c->pm)));
        b = ro(c->w2) * (ro(c->n_is_one) ? p : pow(p, ro(c->pn)));
    } else {
        a = ro(c->w1) * p;
        b = ro(c->w2) * p;
    }
    const double cc = a + b;
    if (!(T > ro(c->Tig) && lam < 1.0 && cc > 0.0)) return 0.0;
    const double y0 = 1.0 - lam;
    const double E = exp(cc * ro(c->dt));
    const double y1 = cc * y0 / (b * y0 + (cc - b * y0) * E);
    return y0 - y1;
}

// C_i = f^eq_i Q [-(1+D) I T + I |v_i - u|^2 + eta_i^2] F / (I (D+I) T^2) with F = dlam/dt
// (Eq. C_i, discrete f^eq), added to src.
__device__ __forceinline__ void add_chemical(const Consts* __restrict__ c, const Macro& m, double dlam,
                                             const double feq[NV], double src[NV]) {
    const double F = dlam / ro(c->dt);
    const double common = ro(c->Q) * F / (ro(c->I) * ro(c->DI) * m.T * m.T);
    // The bracket -(1+D) I T + I |v_i - u|^2 + eta_i^2, already times `common`, split into a
    // part fixed by the group and |v_i| and a part linear in v_i:
    //   common [I (u^2 - (1+D) T) + eta_g^2 + I |v_i|^2] - 2 I common (v_i . u).
    const double I = ro(c->I);
    const double k0 = common * (I * (m.ux * m.ux + m.uy * m.uy) - (1.0 + 2.0) * I * m.T);
    const double px = -2.0 * I * common * m.ux, py = -2.0 * I * common * m.uy;
#pragma unroll
    for (int g2 = 0; g2 < 3; ++g2) {
        const double v = ro(c->vg[g2]);
        const double ka = fma(common, ro(c->eta2[g2]) + I * (v * v), k0);          // |v_i|^2 = v^2
        const double kd = fma(common, ro(c->eta2[g2]) + I * (2.0 * v * v), k0);    // |v_i|^2 = 2 v^2
        const double qx = v * px, qy = v * py, sp = qx + qy, sm = qx - qy;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            double br;
            if (DUY[d] == 0) br = DUX[d] > 0 ? ka + qx : ka - qx;
            else if (DUX[d] == 0) br = DUY[d] > 0 ? ka + qy : ka - qy;
            else if (DUX[d] == DUY[d]) br = DUX[d] > 0 ? kd + sp : kd - sp;
            else br = DUX[d] > 0 ? kd + sm : kd - sm;
            src[8 * g2 + d] = fma(feq[8 * g2 + d], br, src[8 * g2 + d]);
        }
    }
}

// Collision and chemistry of one cell.
// Input: the macroscopic state m, the moments h = M f of the cell, lam, A8/A9 (modification
// terms, 0 if inactive).  Output: src[i] = -Omega_i + C_i (the non-streaming right-hand
// side) and dlam.  Ordered to keep few 24-vectors live: g = R (h - f_hat^eq) - A_hat
// (h and f_hat^eq die), src = -M^-1 g (g dies), then f_hat^eq is evaluated again for
// C_i = f^eq_i w_i with f^eq = M^-1 f_hat^eq.
template <bool CHEM = true, bool GEXP = true>
__device__ __forceinline__ void local_source(const Consts* __restrict__ c, const Mats& M, double lam,
                                             double A8, double A9, const Macro& m, const Blocks& h,
                                             double src[NV], double& dlam,
                                             const double* __restrict__ Rk = nullptr) {
    const double* __restrict__ R = Rk ? Rk : c->R;     // R_1..R_24 (per instance when batched)
    {
        Blocks e;
        equilibrium(m.rho, m.ux, m.uy, m.T, ro(c->I), e);
        // g = R (f_hat - f_hat^eq) - A_hat, Delta_1..4 = 0
        Blocks g;
#pragma unroll
        for (int r = 0; r < NEE; ++r) g.ee[r] = ro(R[EE_M[r]]) * (h.ee[r] - e.ee[r]);
#pragma unroll
        for (int r = 0; r < NOE; ++r) g.oe[r] = ro(R[OE_M[r]]) * (h.oe[r] - e.oe[r]);
#pragma unroll
        for (int r = 0; r < NEO; ++r) g.eo[r] = ro(R[EO_M[r]]) * (h.eo[r] - e.eo[r]);
#pragma unroll
        for (int r = 0; r < NOO; ++r) g.oo[r] = ro(R[OO_M[r]]) * (h.oo[r] - e.oo[r]);
        g.ee[0] = 0.0;   // m1
        g.ee[1] = 0.0;   // m4
        g.oe[0] = 0.0;   // m2
        g.eo[0] = 0.0;   // m3
        g.oe[1] -= A8;   // m8
        g.eo[1] -= A9;   // m9
        Blocks s;
        inverse(M, g, s);
        double om[NV];
        from_combos(s, om);
#pragma unroll
        for (int i = 0; i < NV; ++i) src[i] = -om[i];
    }
    dlam = cochran<CHEM, GEXP>(c, lam, m.rho * m.T, m.T);
    if (CHEM && dlam != 0.0) {
        // f_hat^eq is evaluated again (from an opaque copy of T, so the compiler does not
        // reuse the first evaluation) rather than kept live through the collision.
        __builtin_amdgcn_sched_barrier(0);
        double T2 = m.T;
        asm volatile("" : "+v"(T2));
        Blocks e2;
        equilibrium(m.rho, m.ux, m.uy, T2, ro(c->I), e2);
        Blocks se;
        inverse(M, e2, se);
        double feq[NV];
        from_combos(se, feq);
        add_chemical(c, m, dlam, feq, src);
    }
}

// rho, u and T from the conserved sums of Eqs. moment1-moment3 taken straight over the 24
// values (rho = sum f, j = sum f v, sum f (v^2 + eta^2) = rho ((D+I) T + u^2)).
__device__ __forceinline__ Macro macro_sums(const Consts* __restrict__ c, const double f[NV]) {
    double r = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const double v = ro(c->vg[g]);
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const double x = f[8 * g + d];
            r += x;
            if (DUX[d] != 0) jx = fma(DUX[d] > 0 ? v : -v, x, jx);
            if (DUY[d] != 0) jy = fma(DUY[d] > 0 ? v : -v, x, jy);
            e = fma((double)(DUX[d] * DUX[d] + DUY[d] * DUY[d]) * (v * v) + ro(c->eta2[g]), x, e);
        }
    }
    Macro m;
    m.rho = r;
    m.ux = jx / r;
    m.uy = jy / r;
    m.T = (e / r - m.ux * m.ux - m.uy * m.uy) / ro(c->DI);
    return m;
}

// Single-relaxation-time source (Eq. SRT): src_i = -(f_i - f^eq_i) / tau + C_i with the
// discrete equilibrium f^eq = M^-1 f_hat^eq, which also serves C_i.  No A_hat.
template <bool CHEM = true, bool GEXP = true>
__device__ __forceinline__ void srt_source(const Consts* __restrict__ c, const Mats& M, double lam,
                                           const Macro& m, const double f[NV], double src[NV],
                                           double& dlam) {
    Blocks e, se;
    equilibrium(m.rho, m.ux, m.uy, m.T, ro(c->I), e);
    inverse(M, e, se);
    double feq[NV];
    from_combos(se, feq);
#pragma unroll
    for (int i = 0; i < NV; ++i) src[i] = (feq[i] - f[i]) * ro(c->inv_tau);
    dlam = cochran<CHEM, GEXP>(c, lam, m.rho * m.T, m.T);
    if (CHEM && dlam != 0.0) add_chemical(c, m, dlam, feq, src);
}

// A_hat_8, A_hat_9 (Eqs. ArtificialA8/ArtificialA9) from central differences of u
__device__ __forceinline__ void modification(double a8c, double a9c, double DI, const Macro& m,
                                             double dux_dx, double dux_dy, double duy_dx,
                                             double duy_dy, double& A8, double& A9) {
    const double rT = m.rho * m.T;
    const double iDI = 1.0 / DI;
    A8 = rT * a8c * (4.0 * m.ux * (dux_dx - dux_dx * iDI - duy_dy * iDI) +
                     2.0 * m.uy * (duy_dx + dux_dy));
    A9 = rT * a9c * (4.0 * m.uy * (duy_dy - dux_dx * iDI - duy_dy * iDI) +
                     2.0 * m.ux * (duy_dx + dux_dy));
}
__device__ __forceinline__ void modification(const Consts* __restrict__ c, const Macro& m,
                                             double dux_dx, double dux_dy, double duy_dx,
                                             double duy_dy, double& A8, double& A9) {
    modification(ro(c->a8c), ro(c->a9c), ro(c->DI), m, dux_dx, dux_dy, duy_dx, duy_dy, A8, A9);
}

// A structure-of-arrays buffer seen through one buffer resource: plane i of a cell is at
// byte offset i * plane_bytes (scalar offset operand) + the cell's byte offset (vector
// operand).  The whole buffer must lie within 4 GiB of its base.
struct Soa {
    __amdgpu_buffer_rsrc_t r;
    uint32_t plane_bytes;
};

__device__ __forceinline__ Soa soa(const double* base, int64_t plane) {
    Soa s;
    s.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, -1, 0x00020000);
    s.plane_bytes = (uint32_t)(plane * 8);
    return s;
}

// load/store at scalar byte offset `soff` (e.g. a plane) plus vector byte offset `voff`
__device__ __forceinline__ double ld(const Soa& b, uint32_t soff, uint32_t voff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void st(const Soa& b, uint32_t soff, uint32_t voff, double v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b.r, (int)voff, (int)soff, 0);
}
// The same with the non-temporal cache policy: the new state is not read again within the
// step, so its lines should not displace the stencil data that the caches are reusing.
__device__ __forceinline__ void st_stream(const Soa& b, uint32_t soff, uint32_t voff, double v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b.r, (int)voff, (int)soff, 2);
}

// An opaque copy of a wave-uniform value.  Offsets derived from different copies are not
// merged by the compiler, so the 24 plane offsets of one phase are not kept alive (and
// spilled) through the other phase.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
    asm volatile("" : "+s"(x));
    return x;
}

// the 24 values of one cell; the plane step is added to the vector offset
__device__ __forceinline__ void load_cell(const Soa& f, uint32_t off, double v[NV]) {
    const uint32_t pb = opaque(f.plane_bytes);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        v[i] = ld(f, 0u, off);
        off += pb;
    }
}

// load_cell issued at raised wave priority: the other waves of the SIMD, usually deep in
// their collision arithmetic, do not hold up the start of this memory phase.  Used for the
// centre values of the single-grid step (it made the 256-thread tiles at three waves per
// SIMD the fastest launch); the persistent batch kernel runs slightly slower with it.
// With l given, the cell's lambda is loaded in the same window (its latency would otherwise
// surface just before the reaction step).
__device__ __forceinline__ void load_cell_first(const Soa& f, uint32_t off, double v[NV],
                                                const Soa* l = nullptr, double* lam = nullptr) {
    __builtin_amdgcn_s_setprio(1);
    __builtin_amdgcn_sched_barrier(0);
    load_cell(f, off, v);
    if (l) *lam = ld(*l, 0u, off);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(0);
}

// neighbour index along one axis with the boundary rule (periodic wrap or clamp)
__device__ __forceinline__ int wrap(int j, int n, int bc) {
    if (bc == 0) {   // periodic
        j %= n;
        return j < 0 ? j + n : j;
    }
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

}  // namespace lbkm
