// The fused MRT-LBKM time step (gfx950, float64).
//
// One thread advances one cell through the whole step of Sec. II: macroscopic moments,
// f_hat = M f, equilibrium, A_hat (when active), collision, chemistry and C_i, M^-1,
// NND streaming of all 24 planes, forward Euler, and the lambda update.  All inputs are
// read at level n from `fin`/`lin`; results go to the other buffer pair.
//
// Compile-time specialisations (the host picks one per launch): A_hat possible, general
// rate exponents; the single-relaxation-time collision of Eq. SRT; a
// Runge-Kutta stage (the Euler update blended with f^n at the cell); wall sides (stencil
// points beyond a wall read the ghost layers that k_ghost filled).
//
// Instruction economy (the kernel is issue-bound unless this is watched):
//  - the 324 moment-matrix entries are read column by column with scalar loads and
//    consumed at once (column-major matrix-vector products);
//  - the state is read through buffer resources: plane i of a cell is the scalar offset
//    i * plane_bytes plus the cell's 32-bit byte offset, which is the same for all 24
//    planes, so loads need no per-load address arithmetic;
//  - minmod is branch-free (four min/max).
//
// Work-groups cover TX x TY tiles.  The hardware hands consecutive work-group ids to the
// eight XCDs in turn; `tile_of` renumbers tiles so that XCD k walks the k-th contiguous
// band of tiles (a band of tile columns when their number divides by eight, else a band of
// tile rows), keeping halo re-reads inside one XCD's L2.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbkm_device.h"
#include "lbkm_kernels.h"

namespace lbkm {

namespace {

constexpr int kXcds = 8;

// byte offsets (within one plane) of a cell and its stencil neighbours
struct Off {
    uint32_t c, xm2, xm1, xp1, xp2, ym2, ym1, yp1, yp2;
};

__device__ __forceinline__ Off stencil_offsets(const Consts* __restrict__ c, int x, int y) {
    const int nx = ro(c->nx), ny = ro(c->ny);
    const uint32_t p = (uint32_t)ro(c->pitch);
    const uint32_t row = (uint32_t)y * p;
    Off s;
    s.c = (row + x) * 8u;
    s.xm2 = (row + wrap(x - 2, nx, ro(c->bc_x))) * 8u;
    s.xm1 = (row + wrap(x - 1, nx, ro(c->bc_x))) * 8u;
    s.xp1 = (row + wrap(x + 1, nx, ro(c->bc_x))) * 8u;
    s.xp2 = (row + wrap(x + 2, nx, ro(c->bc_x))) * 8u;
    s.ym2 = ((uint32_t)wrap(y - 2, ny, ro(c->bc_y)) * p + x) * 8u;
    s.ym1 = ((uint32_t)wrap(y - 1, ny, ro(c->bc_y)) * p + x) * 8u;
    s.yp1 = ((uint32_t)wrap(y + 1, ny, ro(c->bc_y)) * p + x) * 8u;
    s.yp2 = ((uint32_t)wrap(y + 2, ny, ro(c->bc_y)) * p + x) * 8u;
    return s;
}

// Stencil points that fall on a wall side's ghost layers (sides with kWall* != none):
// bit k of `is` set for point k (0 x-2, 1 x-1, 2 x+1, 3 x+2, 4 y-2, 5 y-1, 6 y+1, 7 y+2),
// off[k] its byte offset within a ghost-buffer plane (0 where not a ghost, a valid address).
struct Ghosts {
    uint32_t off[8];
    uint32_t is;
};

__device__ __forceinline__ Ghosts ghosts_of(const Consts* __restrict__ c, int x, int y) {
    Ghosts g;
    g.is = 0;
    const uint32_t L = (uint32_t)ro(c->gL);
    auto set = [&](int k, int side, int layer, int along) {
        g.is |= 1u << k;
        g.off[k] = ((uint32_t)(side * 2 + layer) * L + (uint32_t)along) * 8u;
    };
#pragma unroll
    for (int k = 0; k < 8; ++k) g.off[k] = 0u;
    const int nx = ro(c->nx), ny = ro(c->ny);
    if (ro(c->wall[0]) != kWallNone) {
        if (x < 2) set(0, 0, 1 - x, y);
        if (x < 1) set(1, 0, 0, y);
    }
    if (ro(c->wall[1]) != kWallNone) {
        if (x + 1 >= nx) set(2, 1, x + 1 - nx, y);
        if (x + 2 >= nx) set(3, 1, x + 2 - nx, y);
    }
    if (ro(c->wall[2]) != kWallNone) {
        if (y < 2) set(4, 2, 1 - y, x);
        if (y < 1) set(5, 2, 0, x);
    }
    if (ro(c->wall[3]) != kWallNone) {
        if (y + 1 >= ny) set(6, 3, y + 1 - ny, x);
        if (y + 2 >= ny) set(7, 3, y + 2 - ny, x);
    }
    return g;
}

// value of stencil point k of one plane: the state, or the ghost buffer on a wall side
template <bool GHOST>
__device__ __forceinline__ double sld(const Soa& F, uint32_t so, uint32_t off, const Soa& Gb, uint32_t sg,
                                      const Ghosts& gh, int k) {
    const double v = ld(F, so, off);
    if (!GHOST) return v;
    const double w = ld(Gb, sg, gh.off[k]);
    return ((gh.is >> k) & 1u) ? w : v;
}

// Phase 1 of one cell: src = -Omega + C (the right-hand side without streaming), the
// reaction increment dlam, lambda and the macroscopic state, from the cell's 24 values at
// level n (and, when A_hat is active, the four neighbours' velocities, written by the
// previous step or by k_velocity).  SRT: the single-relaxation-time form of Eq. SRT.
template <bool AMOD, bool CHEM, bool GEXP, bool SRT, bool GHOST = false>
__device__ __forceinline__ void cell_source(const Consts* __restrict__ c, const Mats& M, const Soa& F,
                                            const Soa& L, const Soa& Ui, const Off& s, double src[NV],
                                            double& dlam, double& lam, Macro& m, const Soa* Gb = nullptr,
                                            const Ghosts* gh = nullptr) {
    double f[NV];
    if (SRT) {
        load_cell_first(F, s.c, f, &L, &lam);
        m = macro_sums(c, f);
        srt_source<CHEM, GEXP>(c, M, lam, m, f, src, dlam);
        return;
    }
    // velocity gradients for A_hat first, so only four numbers are carried on
    double gxx = 0.0, gxy = 0.0, gyx = 0.0, gyy = 0.0;
    if (AMOD && GHOST) {
        // velocities of the ghost points come from the ghost buffer's velocity planes
        const uint32_t up = opaque(Ui.plane_bytes), gp = opaque(Gb->plane_bytes);
        const uint32_t gx0 = (NV + 1) * gp, gy0 = (NV + 2) * gp;
        gxx = (sld<true>(Ui, 0u, s.xp1, *Gb, gx0, *gh, 2) - sld<true>(Ui, 0u, s.xm1, *Gb, gx0, *gh, 1)) * ro(c->half_inv_dx);
        gyx = (sld<true>(Ui, up, s.xp1, *Gb, gy0, *gh, 2) - sld<true>(Ui, up, s.xm1, *Gb, gy0, *gh, 1)) * ro(c->half_inv_dx);
        gxy = (sld<true>(Ui, 0u, s.yp1, *Gb, gx0, *gh, 6) - sld<true>(Ui, 0u, s.ym1, *Gb, gx0, *gh, 5)) * ro(c->half_inv_dy);
        gyy = (sld<true>(Ui, up, s.yp1, *Gb, gy0, *gh, 6) - sld<true>(Ui, up, s.ym1, *Gb, gy0, *gh, 5)) * ro(c->half_inv_dy);
    } else if (AMOD) {
        // the four neighbours' velocities join the raised-priority window of the centre loads
        const uint32_t up = opaque(Ui.plane_bytes);
        __builtin_amdgcn_s_setprio(1);
        __builtin_amdgcn_sched_barrier(0);
        const double a0 = ld(Ui, 0u, s.xp1), a1 = ld(Ui, 0u, s.xm1), a2 = ld(Ui, up, s.xp1), a3 = ld(Ui, up, s.xm1);
        const double b0 = ld(Ui, 0u, s.yp1), b1 = ld(Ui, 0u, s.ym1), b2 = ld(Ui, up, s.yp1), b3 = ld(Ui, up, s.ym1);
        load_cell(F, s.c, f);
        lam = ld(L, 0u, s.c);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
        gxx = (a0 - a1) * ro(c->half_inv_dx);   // d u_x / dx
        gyx = (a2 - a3) * ro(c->half_inv_dx);   // d u_y / dx
        gxy = (b0 - b1) * ro(c->half_inv_dy);   // d u_x / dy
        gyy = (b2 - b3) * ro(c->half_inv_dy);   // d u_y / dy
    }
    if constexpr (!AMOD || GHOST) load_cell_first(F, s.c, f, &L, &lam);
    Blocks sb, h;
    to_combos(f, sb);
    forward(M, sb, h);
    m = macro_of(h, ro(c->DI));
    double A8 = 0.0, A9 = 0.0;
    if (AMOD) modification(c, m, gxx, gxy, gyx, gyy, A8, A9);
    local_source<CHEM, GEXP>(c, M, lam, A8, A9, m, h, src, dlam);
}

// The same from the cell's 24 values and lambda already in registers (read while
// streaming, or in the centre burst); when A_hat is active, the four neighbours'
// velocities are loaded here.
template <bool AMOD, bool CHEM, bool GEXP, bool SRT, bool GHOST = false>
__device__ __forceinline__ void cell_source_held(const Consts* __restrict__ c, const Mats& M, const double f[NV],
                                                 double lam, const Soa& Ui, const Off& s, double src[NV],
                                                 double& dlam, Macro& m, const Soa* Gb = nullptr,
                                                 const Ghosts* gh = nullptr) {
    if (SRT) {
        m = macro_sums(c, f);
        srt_source<CHEM, GEXP>(c, M, lam, m, f, src, dlam);
        return;
    }
    double gxx = 0.0, gxy = 0.0, gyx = 0.0, gyy = 0.0;
    if (AMOD && GHOST) {
        // velocities of the ghost points come from the ghost buffer's velocity planes
        const uint32_t up = opaque(Ui.plane_bytes), gp = opaque(Gb->plane_bytes);
        const uint32_t gx0 = (NV + 1) * gp, gy0 = (NV + 2) * gp;
        gxx = (sld<true>(Ui, 0u, s.xp1, *Gb, gx0, *gh, 2) - sld<true>(Ui, 0u, s.xm1, *Gb, gx0, *gh, 1)) * ro(c->half_inv_dx);
        gyx = (sld<true>(Ui, up, s.xp1, *Gb, gy0, *gh, 2) - sld<true>(Ui, up, s.xm1, *Gb, gy0, *gh, 1)) * ro(c->half_inv_dx);
        gxy = (sld<true>(Ui, 0u, s.yp1, *Gb, gx0, *gh, 6) - sld<true>(Ui, 0u, s.ym1, *Gb, gx0, *gh, 5)) * ro(c->half_inv_dy);
        gyy = (sld<true>(Ui, up, s.yp1, *Gb, gy0, *gh, 6) - sld<true>(Ui, up, s.ym1, *Gb, gy0, *gh, 5)) * ro(c->half_inv_dy);
    } else if (AMOD) {
        const uint32_t up = opaque(Ui.plane_bytes);
        const double a0 = ld(Ui, 0u, s.xp1), a1 = ld(Ui, 0u, s.xm1), a2 = ld(Ui, up, s.xp1), a3 = ld(Ui, up, s.xm1);
        const double b0 = ld(Ui, 0u, s.yp1), b1 = ld(Ui, 0u, s.ym1), b2 = ld(Ui, up, s.yp1), b3 = ld(Ui, up, s.ym1);
        gxx = (a0 - a1) * ro(c->half_inv_dx);   // d u_x / dx
        gyx = (a2 - a3) * ro(c->half_inv_dx);   // d u_y / dx
        gxy = (b0 - b1) * ro(c->half_inv_dy);   // d u_x / dy
        gyy = (b2 - b3) * ro(c->half_inv_dy);   // d u_y / dy
    }
    Blocks sb, h;
    to_combos(f, sb);
    forward(M, sb, h);
    m = macro_of(h, ro(c->DI));
    double A8 = 0.0, A9 = 0.0;
    if (AMOD) modification(c, m, gxx, gxy, gyx, gyy, A8, A9);
    local_source<CHEM, GEXP>(c, M, lam, A8, A9, m, h, src, dlam);
}

// one full time step of one cell (all inputs at level n); M holds the matrix blocks.
// AMOD: A_hat can be non-zero; CHEM: the reaction can run; GEXP: exponents m, n not both 1;
// SRT: single relaxation time (then AMOD is false); BLEND: a Runge-Kutta stage, the result
// is bl.a * (f^n, lambda^n) + bl.b * (the forward-Euler update).
template <bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND, bool GHOST>
__device__ __forceinline__ void step_cell(const Consts* __restrict__ c, const Mats& M, int x, int y,
                                          const double* __restrict__ fin, double* __restrict__ fout,
                                          const double* __restrict__ lin, double* __restrict__ lout,
                                          const double* __restrict__ uin, double* __restrict__ uout,
                                          const Blend& bl, const double* __restrict__ gb) {
    const Soa F = soa(fin, ro(c->plane)), G = soa(fout, ro(c->plane));
    const Soa L = soa(lin, 0), Lo = soa(lout, 0);
    const Soa Ui = soa(uin, ro(c->plane)), Uo = soa(uout, ro(c->plane));
    // f^n, lambda^n of a Runge-Kutta stage; null: the output buffers themselves (in place)
    const Soa Fn = soa(BLEND ? (bl.fn ? bl.fn : fout) : fin, ro(c->plane));
    const Soa Ln = soa(BLEND ? (bl.ln ? bl.ln : lout) : lin, 0);
    const Off s = stencil_offsets(c, x, y);
    // wall sides: the ghost buffer and which stencil points read it
    const Soa Gb = soa(GHOST ? gb : fin, 8 * (int64_t)ro(c->gL));
    Ghosts gh;
    if (GHOST) gh = ghosts_of(c, x, y);

    // Phase 1: collision and chemistry from the 24 centre values -> src = -Omega + C.
    double src[NV], dlam, lam;
    Macro m;
    cell_source<AMOD, CHEM, GEXP, SRT, GHOST>(c, M, F, L, Ui, s, src, dlam, lam, m, &Gb, &gh);
    __builtin_amdgcn_sched_barrier(0);

    // Phase 2: NND streaming plane by plane; the centre value is read again (a cache hit)
    // so that only src[] stays live across the planes.  GH: stencil points may lie on wall
    // ghost layers (instantiated only in the wall specialisation).
    const double dt = ro(c->dt), idx_ = ro(c->inv_dx), idy = ro(c->inv_dy);
    const uint32_t pb = opaque(F.plane_bytes);
    auto phase2 = [&](auto gh_on) {
        constexpr bool GH = decltype(gh_on)::value;
        VelAcc va;                                  // velocity of the new state (for A_hat)
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const double wx = ro(c->cx[g]), wy = ro(c->cy[g]);   // Courant numbers of the group
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const uint32_t so = (uint32_t)(8 * g + d) * pb;
                const uint32_t sg = GH ? (uint32_t)(8 * g + d) * Gb.plane_bytes : 0u;
                auto at = [&](uint32_t off, int k) { return sld<GH>(F, so, off, Gb, sg, gh, k); };
                const double f0 = ld(F, so, s.c);
                double a = f0;
                if (DUX[d] > 0) a = fma(-wx, nnd_pos(at(s.xm2, 0), at(s.xm1, 1), f0, at(s.xp1, 2)), a);
                if (DUX[d] < 0) a = fma(wx, nnd_neg(at(s.xm1, 1), f0, at(s.xp1, 2), at(s.xp2, 3)), a);
                if (DUY[d] > 0) a = fma(-wy, nnd_pos(at(s.ym2, 4), at(s.ym1, 5), f0, at(s.yp1, 6)), a);
                if (DUY[d] < 0) a = fma(wy, nnd_neg(at(s.ym1, 5), f0, at(s.yp1, 6), at(s.yp2, 7)), a);
                double out = fma(dt, src[8 * g + d], a);
                if (BLEND) out = fma(bl.a, ld(Fn, so, s.c), bl.b * out);   // one rounding order in every variant
                if (AMOD) vel_add(va, c, g, d, out);
                st_stream(G, so, s.c, out);
            }
        }
        if (AMOD) {
            st_stream(Uo, 0u, s.c, va.jx / va.r);
            st_stream(Uo, opaque(Uo.plane_bytes), s.c, va.jy / va.r);
        }
        const uint32_t sl = GH ? NV * Gb.plane_bytes : 0u;
        auto lat = [&](uint32_t off, int k) { return sld<GH>(L, 0u, off, Gb, sl, gh, k); };
        const double dlx = nnd_upwind(m.ux > 0.0, lat(s.xm2, 0), lat(s.xm1, 1), lam, lat(s.xp1, 2), lat(s.xp2, 3));
        const double dly = nnd_upwind(m.uy > 0.0, lat(s.ym2, 4), lat(s.ym1, 5), lam, lat(s.yp1, 6), lat(s.yp2, 7));
        double lnew = lam + dlam - dt * (m.ux * (dlx * idx_) + m.uy * (dly * idy));
        if (BLEND) lnew = fma(bl.a, ld(Ln, 0u, s.c), bl.b * lnew);
        st_stream(Lo, 0u, s.c, lnew);
    };
    if constexpr (GHOST) {
        // only waves with a stencil point on a ghost layer take the selecting path
        if (__ballot(gh.is != 0u) != 0ull)
            phase2(std::true_type{});
        else
            phase2(std::false_type{});
    } else {
        phase2(std::false_type{});
    }
}

// ---------------------------------------------------------------------------------------
// LDS-staged variant.  Phase 1 is the same per-cell collision; in phase 2 the work-group
// stages each velocity plane's tile plus a two-cell halo, (TX+4) x (TY+4) values, in LDS
// with coalesced loads (one per value instead of the seven stencil loads per cell), and
// every thread reads its NND stencil from there.  Plane i+1 is fetched into registers
// while plane i is being differenced (double-buffered patch, one barrier per plane).
template <int TX, int TY>
struct Patch {
    static constexpr int PW = TX + 4, PH = TY + 4, N = PW * PH;
    static constexpr int NT = TX * TY;
    static constexpr int NS = (N + NT - 1) / NT;     // patch values loaded per thread
};

template <int TX, int TY, bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND>
__device__ __forceinline__ void step_tile_lds(const Consts* __restrict__ c, const Mats& M, int x0, int y0,
                                              const double* __restrict__ fin, double* fout,
                                              const double* __restrict__ lin, double* lout,
                                              const double* __restrict__ uin, double* __restrict__ uout,
                                              const Blend& bl, double* __restrict__ patch /* [2][PW*PH] */) {
    using P = Patch<TX, TY>;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < ro(c->nx) && y < ro(c->ny);
    const Soa F = soa(fin, ro(c->plane)), G = soa(fout, ro(c->plane));
    const Soa L = soa(lin, 0), Lo = soa(lout, 0);
    const Soa Ui = soa(uin, ro(c->plane)), Uo = soa(uout, ro(c->plane));
    const Soa Fn = soa(BLEND ? (bl.fn ? bl.fn : fout) : fin, ro(c->plane));
    const Soa Ln = soa(BLEND ? (bl.ln ? bl.ln : lout) : lin, 0);

    // the patch values this thread loads: LDS index and within-plane byte offset
    uint32_t goff[P::NS];
#pragma unroll
    for (int j = 0; j < P::NS; ++j) {
        const int k = tid + j * P::NT;
        const int px = k % P::PW, py = k / P::PW;
        const int gx = wrap(x0 - 2 + px, ro(c->nx), ro(c->bc_x));
        const int gy = wrap(y0 - 2 + py, ro(c->ny), ro(c->bc_y));
        goff[j] = ((uint32_t)gy * (uint32_t)ro(c->pitch) + (uint32_t)gx) * 8u;
    }

    // Phase 1: collision and chemistry of this thread's cell
    double src[NV], dlam = 0.0, lam = 0.0;
    Macro m{1.0, 0.0, 0.0, 1.0};
    if (inside) {
        const Off s = stencil_offsets(c, x, y);
        cell_source<AMOD, CHEM, GEXP, SRT>(c, M, F, L, Ui, s, src, dlam, lam, m);
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) src[i] = 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);

    // Phase 2: planes 0..23 of f, then lambda (plane 24), through the LDS patch
    const double dt = ro(c->dt), idx_ = ro(c->inv_dx), idy = ro(c->inv_dy);
    const uint32_t pb = opaque(F.plane_bytes);
    const uint32_t out_off = ((uint32_t)y * (uint32_t)ro(c->pitch) + (uint32_t)x) * 8u;
    const int cidx = (ly + 2) * P::PW + (lx + 2);
    double pre[P::NS];
    VelAcc va;                                  // velocity of the new state (for A_hat)
    auto fetch = [&](int plane) {
#pragma unroll
        for (int j = 0; j < P::NS; ++j) {
            if (P::N % P::NT == 0 || tid + j * P::NT < P::N)
                pre[j] = (plane < NV) ? ld(F, (uint32_t)plane * pb, goff[j]) : ld(L, 0u, goff[j]);
        }
    };
    fetch(0);
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
        double* buf = patch + (i & 1) * P::N;
#pragma unroll
        for (int j = 0; j < P::NS; ++j)
            if (P::N % P::NT == 0 || tid + j * P::NT < P::N) buf[tid + j * P::NT] = pre[j];
        __syncthreads();
        if (i < NV) fetch(i + 1);
        const double* q = buf + cidx;
        const double f0 = q[0];
        if (i < NV) {
            const int g = i / 8, d = i % 8;
            const double wx = ro(c->cx[g]), wy = ro(c->cy[g]);
            double a = f0;
            if (DUX[d] > 0) a = fma(-wx, nnd_pos(q[-2], q[-1], f0, q[1]), a);
            if (DUX[d] < 0) a = fma(wx, nnd_neg(q[-1], f0, q[1], q[2]), a);
            if (DUY[d] > 0) a = fma(-wy, nnd_pos(q[-2 * P::PW], q[-P::PW], f0, q[P::PW]), a);
            if (DUY[d] < 0) a = fma(wy, nnd_neg(q[-P::PW], f0, q[P::PW], q[2 * P::PW]), a);
            double out = fma(dt, src[i], a);
            if (BLEND && inside) out = fma(bl.a, ld(Fn, (uint32_t)i * pb, out_off), bl.b * out);
            if (AMOD) vel_add(va, c, g, d, out);
            if (inside) st_stream(G, (uint32_t)i * pb, out_off, out);
        } else if (inside) {
            if (AMOD) {
                st_stream(Uo, 0u, out_off, va.jx / va.r);
                st_stream(Uo, opaque(Uo.plane_bytes), out_off, va.jy / va.r);
            }
            const double dlx = nnd_upwind(m.ux > 0.0, q[-2], q[-1], f0, q[1], q[2]);
            const double dly = nnd_upwind(m.uy > 0.0, q[-2 * P::PW], q[-P::PW], f0, q[P::PW], q[2 * P::PW]);
            double lnew = f0 + dlam - dt * (m.ux * (dlx * idx_) + m.uy * (dly * idy));
            if (BLEND) lnew = fma(bl.a, ld(Ln, 0u, out_off), bl.b * lnew);
            st_stream(Lo, 0u, out_off, lnew);
        }
    }
}

// tile t of the XCD-aware order for work-group b; returns false past the last tile
__device__ __forceinline__ bool tile_of(int b, int gx, int ntiles, int vertical, int& tx, int& ty) {
    if (vertical && gx % kXcds == 0) {
        // vertical bands: XCD k owns tile columns [k gx/8, (k+1) gx/8) and walks them row
        // by row, so the rows above and below a tile (its y halo) were fetched into the
        // same L2 moments earlier; only the two-cell x halo at band edges crosses XCDs
        const int cols = gx / kXcds, k = b % kXcds, i = b / kXcds;
        tx = k * cols + i % cols;
        ty = i / cols;
        return ty * gx < ntiles;
    }
    // horizontal bands of tiles in row-major order
    const int per = (ntiles + kXcds - 1) / kXcds;
    const int t = (b % kXcds) * per + b / kXcds;
    if (t >= ntiles) return false;
    tx = t % gx;
    ty = t / gx;
    return true;
}

// Stream-first step: every value of the input state is read from HBM once.  Phase A walks
// the 24 planes, reading each plane's centre value with its NND stencil, and keeps the
// streamed value f_i - dt v_i . grad_NND f_i in this thread's slots of LDS and the 24
// centre values in registers; phase B collides from those registers and writes
// f^{n+1} = streamed + dt src.  (The two-phase kernel above collides first and re-reads
// each centre value with its stencil; at three waves per SIMD the centre values of all
// resident tiles do not fit the L2 between the two reads, so they come from HBM twice.)
// Each thread touches only its own LDS slots: no barrier.
template <int TX, int TY, bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND>
__global__ __launch_bounds__(TX * TY, GEXP ? 2 : 3) void k_step_sf(const Consts* __restrict__ c,
                                                               const double* __restrict__ fin,
                                                               double* __restrict__ fout,
                                                               const double* __restrict__ lin,
                                                               double* __restrict__ lout,
                                                               const double* __restrict__ uin,
                                                               double* __restrict__ uout, int gx, int ntiles,
                                                               int vertical, Blend bl) {
    constexpr int NT = TX * TY;
    __shared__ double streamed[NV * NT];
    int tx, ty;
    if (!tile_of(blockIdx.x, gx, ntiles, vertical, tx, ty)) return;
    const int tid = (int)threadIdx.x;
    const int x = tx * TX + tid % TX;
    const int y = ty * TY + tid / TX;
    if (x >= ro(c->nx) || y >= ro(c->ny)) return;
    const Soa F = soa(fin, ro(c->plane)), G = soa(fout, ro(c->plane));
    const Soa L = soa(lin, 0), Lo = soa(lout, 0);
    const Soa Ui = soa(uin, ro(c->plane)), Uo = soa(uout, ro(c->plane));
    const Soa Fn = soa(BLEND ? (bl.fn ? bl.fn : fout) : fin, ro(c->plane));
    const Soa Ln = soa(BLEND ? (bl.ln ? bl.ln : lout) : lin, 0);
    const Off s = stencil_offsets(c, x, y);
    const double dt = ro(c->dt), idx_ = ro(c->inv_dx), idy = ro(c->inv_dy);

    // Phase A: the 24 centre values in one burst at raised wave priority (all of them miss
    // in the caches: many loads in flight per wave), then the NND streaming of every plane,
    // whose stencil neighbours are mostly the lines those bursts have just brought in.
    double f[NV];
    load_cell_first(F, s.c, f);
    // The x-neighbours of a cell are the centre values of the neighbouring lanes when the
    // wave holds 64 consecutive cells of a row (tiles 64 or more wide, away from a ragged
    // right edge): lane moves then replace two of the three x-stencil loads of a plane, and
    // one halo load per plane serves the lanes at both ends.  L1 bandwidth, not HBM, bounds
    // this phase (about 140 eight-byte gathers per cell), so the loads saved are what counts.
    const int lane = tid & 63;
    const bool lanes_form_row = TX % 64 == 0 && (x - lane) + 64 <= ro(c->nx);   // uniform per wave
    uint32_t halo = 0u;
    if (TX % 64 == 0) {
        const int x0 = x - lane, nx = ro(c->nx), bcx = ro(c->bc_x);
        const int hx = lane < 32 ? (lane == 0 ? x0 - 2 : x0 - 1) : (lane == 63 ? x0 + 65 : x0 + 64);
        halo = ((uint32_t)y * (uint32_t)ro(c->pitch) + (uint32_t)wrap(hx, nx, bcx)) * 8u;
    }
    auto phase_a = [&](auto by_lanes) {
        constexpr bool XL = decltype(by_lanes)::value;
        const uint32_t pb = opaque(F.plane_bytes);
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const double wx = ro(c->cx[g]), wy = ro(c->cy[g]);   // Courant numbers of the group
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const uint32_t so = (uint32_t)(8 * g + d) * pb;
                const double f0 = f[8 * g + d];
                double a = f0;
                if (XL && DUX[d] != 0) {
                    const XNeighbours n = x_neighbours(f0, ld(F, so, halo));
                    if (DUX[d] > 0) a = fma(-wx, nnd_pos(n.m2, n.m1, f0, n.p1), a);
                    if (DUX[d] < 0) a = fma(wx, nnd_neg(n.m1, f0, n.p1, n.p2), a);
                } else {
                    if (DUX[d] > 0) a = fma(-wx, nnd_pos(ld(F, so, s.xm2), ld(F, so, s.xm1), f0, ld(F, so, s.xp1)), a);
                    if (DUX[d] < 0) a = fma(wx, nnd_neg(ld(F, so, s.xm1), f0, ld(F, so, s.xp1), ld(F, so, s.xp2)), a);
                }
                if (DUY[d] > 0) a = fma(-wy, nnd_pos(ld(F, so, s.ym2), ld(F, so, s.ym1), f0, ld(F, so, s.yp1)), a);
                if (DUY[d] < 0) a = fma(wy, nnd_neg(ld(F, so, s.ym1), f0, ld(F, so, s.yp1), ld(F, so, s.yp2)), a);
                streamed[(8 * g + d) * NT + tid] = a;
            }
        }
    };
    if constexpr (TX % 64 == 0) {
        if (lanes_form_row)
            phase_a(std::true_type{});
        else
            phase_a(std::false_type{});
    } else {
        phase_a(std::false_type{});
    }
    __builtin_amdgcn_sched_barrier(0);

    // Phase B: collision and chemistry, then the update of each plane
    double src[NV], dlam;
    Macro m;
    const double lam = ld(L, 0u, s.c);
    cell_source_held<AMOD, CHEM, GEXP, SRT>(c, c->mat, f, lam, Ui, s, src, dlam, m);
    __builtin_amdgcn_sched_barrier(0);
    {
        const uint32_t pb = opaque(G.plane_bytes);
        VelAcc va;                                  // velocity of the new state (for A_hat)
#pragma unroll
        for (int g = 0; g < 3; ++g) {
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const uint32_t so = (uint32_t)(8 * g + d) * pb;
                double out = fma(dt, src[8 * g + d], streamed[(8 * g + d) * NT + tid]);
                if (BLEND) out = fma(bl.a, ld(Fn, so, s.c), bl.b * out);   // one rounding order in every variant
                if (AMOD) vel_add(va, c, g, d, out);
                st_stream(G, so, s.c, out);
            }
        }
        if (AMOD) {
            st_stream(Uo, 0u, s.c, va.jx / va.r);
            st_stream(Uo, opaque(Uo.plane_bytes), s.c, va.jy / va.r);
        }
    }
    const double dlx = nnd_upwind(m.ux > 0.0, ld(L, 0u, s.xm2), ld(L, 0u, s.xm1), lam, ld(L, 0u, s.xp1),
                                  ld(L, 0u, s.xp2));
    const double dly = nnd_upwind(m.uy > 0.0, ld(L, 0u, s.ym2), ld(L, 0u, s.ym1), lam, ld(L, 0u, s.yp1),
                                  ld(L, 0u, s.yp2));
    double lnew = lam + dlam - dt * (m.ux * (dlx * idx_) + m.uy * (dly * idy));
    if (BLEND) lnew = fma(bl.a, ld(Ln, 0u, s.c), bl.b * lnew);
    st_stream(Lo, 0u, s.c, lnew);
}

// Collide first with the tile's centre values shared in LDS.  Each wave loads its cells'
// 24 centre values in one burst and writes them to LDS; after the collision and one
// barrier, the streaming phase takes the cell's own value and its y-neighbours inside the
// tile from LDS, its x-neighbours from the neighbouring lanes (a wave is 64 cells of one
// row), and loads only the halo: the rows beyond the tile and the two cells beyond each
// end of the row.  The choice between LDS and memory is fixed at compile time per row of
// the tile, so the loads of consecutive planes stay free to overlap; rows within two cells
// of a y edge (where the boundary rule may map a neighbour anywhere) and waves that are not
// whole rows load every neighbour.
template <int RW>
struct RowOf {
    static constexpr int value = RW;
};

template <bool IN, bool GH = false>
__device__ __forceinline__ double centre_or_load(const double* slot, int delta, const Soa& F, uint32_t so,
                                                 uint32_t off, const Soa* Gb = nullptr, uint32_t sg = 0u,
                                                 const Ghosts* gh = nullptr, int k = 0) {
    if constexpr (IN)
        return slot[delta];
    else if constexpr (GH)
        return sld<true>(F, so, off, *Gb, sg, *gh, k);
    else
        return ld(F, so, off);
}

template <int TX, int TY, bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND, bool GHOST>
__global__ __launch_bounds__(TX * TY, (GEXP || (GHOST && AMOD && CHEM)) ? 2 : 3) void k_step_sh(
        const Consts* __restrict__ c, const double* __restrict__ fin, double* __restrict__ fout,
        const double* __restrict__ lin, double* __restrict__ lout, const double* __restrict__ uin,
        double* __restrict__ uout, int gx, int ntiles, int vertical, Blend bl, const double* __restrict__ gb) {
    static_assert(TX % 64 == 0, "a wave must hold cells of one row");
    constexpr int NT = TX * TY;
    __shared__ double cen[(NV + 1) * NT];     // the 24 planes and lambda
    int tx, ty;
    if (!tile_of(blockIdx.x, gx, ntiles, vertical, tx, ty)) return;   // uniform over the work-group
    const int tid = (int)threadIdx.x;
    const int x = tx * TX + tid % TX;
    const int y = ty * TY + tid / TX;
    const int nx = ro(c->nx), ny = ro(c->ny);
    const bool inside = x < nx && y < ny;     // every thread stays for the barrier
    const Soa F = soa(fin, ro(c->plane)), G = soa(fout, ro(c->plane));
    const Soa L = soa(lin, 0), Lo = soa(lout, 0);
    const Soa Ui = soa(uin, ro(c->plane)), Uo = soa(uout, ro(c->plane));
    const Soa Fn = soa(BLEND ? (bl.fn ? bl.fn : fout) : fin, ro(c->plane));
    const Soa Ln = soa(BLEND ? (bl.ln ? bl.ln : lout) : lin, 0);
    const Off s = stencil_offsets(c, inside ? x : 0, inside ? y : 0);
    const double dt = ro(c->dt), idx_ = ro(c->inv_dx), idy = ro(c->inv_dy);
    // wall sides: the ghost buffer and which stencil points read it
    const Soa Gb = soa(GHOST ? gb : fin, 8 * (int64_t)ro(c->gL));
    Ghosts gh;
    gh.is = 0u;
    if (GHOST && inside) gh = ghosts_of(c, x, y);

    // Phase 1: centre burst, the values to LDS, collision and chemistry
    double src[NV], dlam = 0.0, lam = 0.0;
    Macro m{1.0, 0.0, 0.0, 1.0};
    if (inside) {
        double f[NV];
        load_cell_first(F, s.c, f, &L, &lam);
#pragma unroll
        for (int i = 0; i < NV; ++i) cen[i * NT + tid] = f[i];
        cen[NV * NT + tid] = lam;
        cell_source_held<AMOD, CHEM, GEXP, SRT, GHOST>(c, c->mat, f, lam, Ui, s, src, dlam, m, &Gb, &gh);
    }
    __syncthreads();
    if (!inside) return;

    // Phase 2: NND streaming from LDS and the halo, forward Euler, store
    const int lane = tid & 63;
    const bool lanes_form_row = (x - lane) + 64 <= nx;                  // uniform per wave
    uint32_t halo;
    {
        const int x0 = x - lane;
        const int hx = lane < 32 ? (lane == 0 ? x0 - 2 : x0 - 1) : (lane == 63 ? x0 + 65 : x0 + 64);
        halo = ((uint32_t)y * (uint32_t)ro(c->pitch) + (uint32_t)wrap(hx, nx, ro(c->bc_x))) * 8u;
    }
    auto phase2 = [&](auto by_lanes, auto row, auto ghost_on) {
        constexpr bool XL = decltype(by_lanes)::value;
        constexpr int RW = decltype(row)::value;   // row of the tile, -1: load every y-neighbour
        constexpr bool GH = decltype(ghost_on)::value;   // stencil points may lie on wall ghost layers
        constexpr bool IM2 = RW >= 2, IM1 = RW >= 1, IP1 = RW >= 0 && RW + 1 < TY, IP2 = RW >= 0 && RW + 2 < TY;
        const uint32_t pb = opaque(F.plane_bytes);
        VelAcc va;                                  // velocity of the new state (for A_hat)
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const double wx = ro(c->cx[g]), wy = ro(c->cy[g]);   // Courant numbers of the group
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int i = 8 * g + d;
                const uint32_t so = (uint32_t)i * pb;
                const double* slot = cen + i * NT + tid;
                const double f0 = slot[0];
                const uint32_t sg = GH ? (uint32_t)i * Gb.plane_bytes : 0u;
                auto at = [&](uint32_t off, int k) { return sld<GH>(F, so, off, Gb, sg, gh, k); };
                double a = f0;
                if (XL && DUX[d] != 0) {
                    const XNeighbours n = x_neighbours(f0, ld(F, so, halo));
                    if (DUX[d] > 0) a = fma(-wx, nnd_pos(n.m2, n.m1, f0, n.p1), a);
                    if (DUX[d] < 0) a = fma(wx, nnd_neg(n.m1, f0, n.p1, n.p2), a);
                } else {
                    if (DUX[d] > 0) a = fma(-wx, nnd_pos(at(s.xm2, 0), at(s.xm1, 1), f0, at(s.xp1, 2)), a);
                    if (DUX[d] < 0) a = fma(wx, nnd_neg(at(s.xm1, 1), f0, at(s.xp1, 2), at(s.xp2, 3)), a);
                }
                if (DUY[d] > 0)
                    a = fma(-wy, nnd_pos(centre_or_load<IM2, GH>(slot, -2 * TX, F, so, s.ym2, &Gb, sg, &gh, 4),
                                         centre_or_load<IM1, GH>(slot, -TX, F, so, s.ym1, &Gb, sg, &gh, 5), f0,
                                         centre_or_load<IP1, GH>(slot, TX, F, so, s.yp1, &Gb, sg, &gh, 6)), a);
                if (DUY[d] < 0)
                    a = fma(wy, nnd_neg(centre_or_load<IM1, GH>(slot, -TX, F, so, s.ym1, &Gb, sg, &gh, 5), f0,
                                        centre_or_load<IP1, GH>(slot, TX, F, so, s.yp1, &Gb, sg, &gh, 6),
                                        centre_or_load<IP2, GH>(slot, 2 * TX, F, so, s.yp2, &Gb, sg, &gh, 7)), a);
                double out = fma(dt, src[i], a);
                if (BLEND) out = fma(bl.a, ld(Fn, so, s.c), bl.b * out);   // one rounding order in every variant
                if (AMOD) vel_add(va, c, g, d, out);
                st_stream(G, so, s.c, out);
            }
        }
        if (AMOD) {
            st_stream(Uo, 0u, s.c, va.jx / va.r);
            st_stream(Uo, opaque(Uo.plane_bytes), s.c, va.jy / va.r);
        }
        // lambda, upwind by the sign of u, from the same sources
        const double* lslot = cen + NV * NT + tid;
        const uint32_t sl = GH ? NV * Gb.plane_bytes : 0u;
        auto lat = [&](uint32_t off, int k) { return sld<GH>(L, 0u, off, Gb, sl, gh, k); };
        double dlx;
        if (XL) {
            const XNeighbours n = x_neighbours(lam, ld(L, 0u, halo));
            dlx = nnd_upwind(m.ux > 0.0, n.m2, n.m1, lam, n.p1, n.p2);
        } else {
            dlx = nnd_upwind(m.ux > 0.0, lat(s.xm2, 0), lat(s.xm1, 1), lam, lat(s.xp1, 2), lat(s.xp2, 3));
        }
        const double dly = nnd_upwind(m.uy > 0.0, centre_or_load<IM2, GH>(lslot, -2 * TX, L, 0u, s.ym2, &Gb, sl, &gh, 4),
                                      centre_or_load<IM1, GH>(lslot, -TX, L, 0u, s.ym1, &Gb, sl, &gh, 5), lam,
                                      centre_or_load<IP1, GH>(lslot, TX, L, 0u, s.yp1, &Gb, sl, &gh, 6),
                                      centre_or_load<IP2, GH>(lslot, 2 * TX, L, 0u, s.yp2, &Gb, sl, &gh, 7));
        double lnew = lam + dlam - dt * (m.ux * (dlx * idx_) + m.uy * (dly * idy));
        if (BLEND) lnew = fma(bl.a, ld(Ln, 0u, s.c), bl.b * lnew);
        st_stream(Lo, 0u, s.c, lnew);
    };
    const int rw = __builtin_amdgcn_readfirstlane(tid / TX);
    const std::false_type no_ghost{};
    // only waves with a stencil point on a wall's ghost layer take the selecting path (those
    // lie within two cells of a wall side, so every other wave takes the paths below)
    if (GHOST && __ballot(gh.is != 0u) != 0ull) {
        phase2(std::false_type{}, RowOf<-1>{}, std::bool_constant<GHOST>{});
    } else if (lanes_form_row && y >= 2 && y + 2 < ny) {
        static_assert(TY <= 6, "rows of the tile are specialised up to six");
        if (rw == 0) phase2(std::true_type{}, RowOf<0>{}, no_ghost);
        else if (TY > 1 && rw == 1) phase2(std::true_type{}, RowOf<(TY > 1 ? 1 : 0)>{}, no_ghost);
        else if (TY > 2 && rw == 2) phase2(std::true_type{}, RowOf<(TY > 2 ? 2 : 0)>{}, no_ghost);
        else if (TY > 3 && rw == 3) phase2(std::true_type{}, RowOf<(TY > 3 ? 3 : 0)>{}, no_ghost);
        else if (TY > 4 && rw == 4) phase2(std::true_type{}, RowOf<(TY > 4 ? 4 : 0)>{}, no_ghost);
        else if (TY > 5) phase2(std::true_type{}, RowOf<(TY > 5 ? 5 : 0)>{}, no_ghost);
    } else if (lanes_form_row) {
        phase2(std::true_type{}, RowOf<-1>{}, no_ghost);
    } else {
        phase2(std::false_type{}, RowOf<-1>{}, no_ghost);
    }
}

// At least three waves per SIMD (a budget of 168 registers) unless the rate exponents are
// general, or walls meet A_hat and the reaction: the other specialisations then fit without
// spilling, the compiler stops parking scalar registers in vector lanes, and the wall
// specialisation's interior waves run as fast as the plain kernel; those two would spill.
template <int TX, int TY, bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND, bool GHOST>
__global__ __launch_bounds__(TX * TY, (GEXP || (GHOST && AMOD && CHEM)) ? 2 : 3) void k_step(const Consts* __restrict__ c, const double* __restrict__ fin,
                                                  double* __restrict__ fout, const double* __restrict__ lin,
                                                  double* __restrict__ lout, const double* __restrict__ uin,
                                                  double* __restrict__ uout, int gx, int ntiles, int vertical,
                                                  Blend bl, const double* __restrict__ gb) {
    int tx, ty;
    if (!tile_of(blockIdx.x, gx, ntiles, vertical, tx, ty)) return;
    const int x = tx * TX + (int)(threadIdx.x % TX);
    const int y = ty * TY + (int)(threadIdx.x / TX);
    if (x >= ro(c->nx) || y >= ro(c->ny)) return;
    step_cell<AMOD, CHEM, GEXP, SRT, BLEND, GHOST>(c, c->mat, x, y, fin, fout, lin, lout, uin, uout, bl, gb);
}

template <int TX, int TY, bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND>
__global__ __launch_bounds__(TX * TY) void k_step_lds(const Consts* __restrict__ c,
                                                      const double* __restrict__ fin, double* fout,
                                                      const double* __restrict__ lin, double* lout,
                                                      const double* __restrict__ uin, double* __restrict__ uout,
                                                      int gx, int ntiles, int vertical, Blend bl) {
    __shared__ double patch[2 * Patch<TX, TY>::N];
    int tx, ty;
    if (!tile_of(blockIdx.x, gx, ntiles, vertical, tx, ty)) return;
    step_tile_lds<TX, TY, AMOD, CHEM, GEXP, SRT, BLEND>(c, c->mat, tx * TX, ty * TY, fin, fout, lin, lout, uin, uout,
                                                        bl, patch);
}

template <int TX, int TY, int MODE, bool AMOD, bool CHEM, bool GEXP, bool SRT, bool BLEND, bool GHOST>
hipError_t launch_tiles(const Consts* dc, int nx, int ny, const double* fin, double* fout, const double* lin,
                        double* lout, const double* uin, double* uout, int vertical, hipStream_t st,
                        const Blend& bl, const double* gb) {
    const int gx = (nx + TX - 1) / TX, gy = (ny + TY - 1) / TY;
    const int ntiles = gx * gy;
    const int per = (ntiles + kXcds - 1) / kXcds;
    if constexpr (MODE == 1)
        hipLaunchKernelGGL((k_step_lds<TX, TY, AMOD, CHEM, GEXP, SRT, BLEND>), dim3(per * kXcds), dim3(TX * TY), 0,
                           st, dc, fin, fout, lin, lout, uin, uout, gx, ntiles, vertical, bl);
    else if constexpr (MODE == 2)
        hipLaunchKernelGGL((k_step_sf<TX, TY, AMOD, CHEM, GEXP, SRT, BLEND>), dim3(per * kXcds), dim3(TX * TY), 0,
                           st, dc, fin, fout, lin, lout, uin, uout, gx, ntiles, vertical, bl);
    else if constexpr (MODE == 3)
        hipLaunchKernelGGL((k_step_sh<TX, TY, AMOD, CHEM, GEXP, SRT, BLEND, GHOST>), dim3(per * kXcds),
                           dim3(TX * TY), 0, st, dc, fin, fout, lin, lout, uin, uout, gx, ntiles, vertical, bl, gb);
    else
        hipLaunchKernelGGL((k_step<TX, TY, AMOD, CHEM, GEXP, SRT, BLEND, GHOST>), dim3(per * kXcds), dim3(TX * TY), 0,
                           st, dc, fin, fout, lin, lout, uin, uout, gx, ntiles, vertical, bl, gb);
    return hipGetLastError();
}

template <int TX, int TY, int MODE, bool BLEND, bool GHOST = false>
hipError_t launch_flags(const Consts* dc, int flags, int nx, int ny, const double* fin, double* fout,
                        const double* lin, double* lout, const double* uin, double* uout, int vertical,
                        hipStream_t st, const Blend& bl, const double* gb = nullptr) {
#define LBKM_TILES(A, C, G, S) \
    launch_tiles<TX, TY, MODE, A, C, G, S, BLEND, GHOST>(dc, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, \
                                                        bl, gb)
    switch (flags) {
        case 2: return LBKM_TILES(false, true, false, false);
        case 3: return LBKM_TILES(true, true, false, false);
        case 6: return LBKM_TILES(false, true, true, false);
        case 7: return LBKM_TILES(true, true, true, false);
        case 10: return LBKM_TILES(false, true, false, true);
        case 14: return LBKM_TILES(false, true, true, true);
        default: return hipErrorInvalidValue;
    }
#undef LBKM_TILES
}

template <int TX, int TY, int MODE>
hipError_t launch_shape(const Consts* dc, int flags, int nx, int ny, const double* fin, double* fout,
                        const double* lin, double* lout, const double* uin, double* uout, int vertical,
                        hipStream_t st, const Blend* bl) {
    if (bl) return launch_flags<TX, TY, MODE, true>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, *bl);
    const Blend none{nullptr, nullptr, 0.0, 1.0};
    return launch_flags<TX, TY, MODE, false>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, none);
}

}  // namespace

// Launch variants compiled in: {tile_x, tile_y, mode}.  mode 0 collides first and reads the
// stencil straight from the caches; mode 1 collides first and stages each stencil plane in
// LDS; mode 2 streams first (k_step_sf, each input value read from HBM once); mode 3
// collides first with the tile's centre values shared in LDS (k_step_sh).
const int kStepVariants[][3] = {{64, 4, 1}, {32, 8, 1}, {128, 2, 1}, {256, 2, 0}, {256, 1, 0}, {64, 4, 0},
                                {64, 4, 2}, {32, 8, 2}, {128, 2, 2}, {256, 1, 2}, {64, 4, 3}, {128, 2, 3}};
const int kNumStepVariants = sizeof(kStepVariants) / sizeof(kStepVariants[0]);
const int kWallTile[3] = {64, 4, 3};   // the one shape compiled with the wall (ghost-layer) stencil

// The reaction is always compiled in (flag 2): without a reaction the wave-uniform test on
// the Cochran increment skips it at run time, and that kernel runs an inert step faster
// (0.454 against 0.496 ms at 2048^2) than one compiled without the reaction, which the
// compiler schedules for four waves per SIMD instead of three.
int step_flags(const Consts& c) {
    const bool chem = c.chem != 0;
    const int rest = 2 | ((chem && !(c.m_is_one && c.n_is_one)) ? 4 : 0);
    if (c.srt) return 8 | rest;                   // no A_hat in the single-relaxation-time form
    return (c.amod ? 1 : 0) | rest;
}

hipError_t launch_step(const Consts* dc, int variant, int flags, int nx, int ny, const double* fin,
                       double* fout, const double* lin, double* lout, const double* uin, double* uout,
                       int vertical, hipStream_t st, const Blend* bl, const double* gb) {
    if (gb) {
        // wall sides: the 64 x 4 shared-centre shape (kWallTile), whatever the tuned one
        if (bl) return launch_flags<64, 4, 3, true, true>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout,
                                                               vertical, st, *bl, gb);
        const Blend none{nullptr, nullptr, 0.0, 1.0};
        return launch_flags<64, 4, 3, false, true>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical,
                                                        st, none, gb);
    }
    switch (variant) {
        case 1: return launch_shape<32, 8, 1>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 2: return launch_shape<128, 2, 1>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 3: return launch_shape<256, 2, 0>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 4: return launch_shape<256, 1, 0>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 5: return launch_shape<64, 4, 0>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 6: return launch_shape<64, 4, 2>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 7: return launch_shape<32, 8, 2>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 8: return launch_shape<128, 2, 2>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 9: return launch_shape<256, 1, 2>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 10: return launch_shape<64, 4, 3>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        case 11: return launch_shape<128, 2, 3>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
        default: return launch_shape<64, 4, 1>(dc, flags, nx, ny, fin, fout, lin, lout, uin, uout, vertical, st, bl);
    }
}

}  // namespace lbkm
