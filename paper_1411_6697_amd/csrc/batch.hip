// Batched 1D instances: many independent detonation tubes of uneven length advanced by
// one persistent kernel launch (replayed from a captured HIP graph).
//
// Layout: the instances' cells are packed back to back (global cell index j), state f[24][P]
// and lambda[P] with P = total cells rounded up to 64; each buffer exists twice (ping-pong).
// Every instance is nx x 1, y-periodic, with zero-gradient outflow at both x ends, so the
// y-differences of the NND scheme and of A_hat vanish identically and are not evaluated.
//
// Work decomposition: the packed cells are cut into `nwg` contiguous ranges of nearly
// equal size, one per work-group, with all work-groups resident at once (their number is
// bounded by the occupancy the device reports).  A range is split into segments at
// instance boundaries, so each segment's rates are wave-uniform (scalar loads).  For each
// step a work-group updates its range from buffer `cur` into the other buffer; it may start
// step s+1 once both neighbouring ranges have completed step s (then their step-s values,
// its halo, are final, and they no longer read the buffer it is about to overwrite).  After
// a work-group barrier, thread 0 publishes the counter with one device-scope release store;
// a reader polls with relaxed loads and then issues one device-scope acquire fence.
// Waiting is bounded: past the spin
// limit the kernel records an error and every work-group returns, so the launch always
// drains.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lbkm_abi_internal.h"
#include "lbkm_device.h"
#include "lbkm_kernels.h"

namespace lbkm {

struct BatchInst {
    double R[NV];
    double a8c, a9c;
    int32_t amod;
    int32_t lo, hi;      // first and last packed cell of the instance
    int32_t pad;
};

struct BatchSeg {
    int32_t inst;        // instance index
    int32_t begin, end;  // global cells [begin, end) updated by this segment
    int32_t lo, hi;      // first and last global cell of the instance (outflow clamp)
};

constexpr int kBatchThreads = 256;
constexpr int kStepChunk = 64;        // launches per captured graph in the one-launch-per-step mode (even)
constexpr int kSpinLimit = 1 << 20;   // neighbour waits are bounded (error, never a hang)

struct BatchState {
    int32_t n_inst = 0;
    std::vector<int32_t> nx;
    std::vector<int32_t> off;
    int64_t total = 0, plane = 0;
    double* f[2] = {nullptr, nullptr};
    double* lam[2] = {nullptr, nullptr};
    double* u[2] = {nullptr, nullptr};     // velocity planes [2][plane] (inputs of A_hat)
    bool u_valid = false;
    int cur = 0;
    std::vector<BatchInst> h_inst;
    BatchInst* d_inst = nullptr;
    bool any_amod = false;
    // launch decomposition (wgs_per_cu = 0: one launch per step instead of the persistent kernel)
    int wgs_per_cu = 2, nwg = 0, cus = 0;
    int32_t* d_wave_inst = nullptr;    // per 64-cell wave: first and last instance it overlaps
    int nwaves = 0;
    BatchSeg* d_seg = nullptr;
    int32_t* d_wg_seg = nullptr;
    int seg_cap = 0;
    uint32_t* d_flags = nullptr;
    int32_t* d_err = nullptr;
    // captured graphs: [parity]
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int64_t exec_steps[2] = {-1, -1};
    int exec_nwg[2] = {-1, -1};
    // one launch per step: [parity][a chunk of kStepChunk steps, the remainder]
    hipGraphExec_t sexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int64_t sexec_steps[2][2] = {{-1, -1}, {-1, -1}};
    hipStream_t cap = nullptr;
};

namespace {

// Poll a neighbour's completed-step counter with relaxed loads (the caller issues one
// acquire fence once both neighbours are ready, so the caches are invalidated once per
// step rather than once per poll).
__device__ __forceinline__ bool wait_counter(const uint32_t* flags, int nb, int nwg, uint32_t want,
                                             const int32_t* err) {
    if (nb < 0 || nb >= nwg) return true;
    for (int k = 0; k < kSpinLimit; ++k) {
        if (__hip_atomic_load(flags + nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) return true;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

// one step of one cell of a 1D instance (x-derivatives only; y-differences are zero).
// [lo, hi] is the instance, cells below `end` are updated in this pass of the work-group,
// stash holds this thread's 24 LDS slots ([plane][kBatchThreads]).
template <bool AMOD, bool CHEM, bool GEXP>
__device__ __forceinline__ void cell_1d(const Consts* __restrict__ c,
                                        const BatchInst* __restrict__ I, int lo, int hi, int end, int j,
                                        const Soa& F, const Soa& G, const Soa& L, const Soa& Lo, const Soa& Ui,
                                        const Soa& Uo, double* stash) {
    const uint32_t oc = (uint32_t)j * 8u;
    // A wave updates 64 consecutive cells; when they and their two neighbours on each side
    // lie inside the instance, the x-stencil of a plane is the centre values of the
    // neighbouring lanes plus one halo load (the two cells beyond each end), and each lane
    // keeps its centre values in its own LDS slots between the collision and the streaming.
    const int lane = (int)(threadIdx.x & 63u);
    const int j0 = j - lane;
    const bool by_lanes = j0 - 2 >= lo && j0 + 65 <= hi && j0 + 64 <= end;     // uniform per wave
    const uint32_t om2 = (uint32_t)max(j - 2, lo) * 8u, om1 = (uint32_t)max(j - 1, lo) * 8u;
    const uint32_t op1 = (uint32_t)min(j + 1, hi) * 8u, op2 = (uint32_t)min(j + 2, hi) * 8u;

    double src[NV], dlam, lam;
    Macro m;
    {
        double gxx = 0.0, gyx = 0.0;
        if (AMOD && ro(I->amod)) {
            // the neighbours' velocities, written by the previous step (or k_velocity)
            const uint32_t up = opaque(Ui.plane_bytes);
            gxx = (ld(Ui, 0u, op1) - ld(Ui, 0u, om1)) * ro(c->half_inv_dx);
            gyx = (ld(Ui, up, op1) - ld(Ui, up, om1)) * ro(c->half_inv_dx);
        }
        double f[NV];
        load_cell(F, oc, f);
        if (by_lanes) {
#pragma unroll
            for (int i = 0; i < NV; ++i) stash[i * kBatchThreads] = f[i];
        }
        Blocks sb, h;
        to_combos(f, sb);
        forward(c->mat, sb, h);
        m = macro_of(h, ro(c->DI));
        double A8 = 0.0, A9 = 0.0;
        if (AMOD && ro(I->amod)) modification(ro(I->a8c), ro(I->a9c), ro(c->DI), m, gxx, 0.0, gyx, 0.0, A8, A9);
        lam = ld(L, 0u, oc);
        local_source<CHEM, GEXP>(c, c->mat, lam, A8, A9, m, h, src, dlam, I->R);
    }
    __builtin_amdgcn_sched_barrier(0);
    const double dt = ro(c->dt), idx_ = ro(c->inv_dx);
    const uint32_t pb = opaque(F.plane_bytes);
    // The input and output buffers trade places from step to step, so the compiler cannot
    // tell that a store of plane i leaves plane i+1's stencil unchanged, and would issue
    // those loads only after the store: one memory round trip per plane.  Plane i+1's loads
    // (and, with the last plane, lambda's stencil) are therefore issued before plane i is
    // differenced and stored, and the scheduling barrier keeps them there.
    struct PlaneLoads {
        double v[5];                            // offsets -2..2 (those the upwind side uses)
    };
    auto load_plane = [&](int i, PlaneLoads& p) {
        const uint32_t so = (uint32_t)i * pb;
        const int d = i & 7;
        p.v[2] = ld(F, so, oc);
        if (DUX[d] > 0) {
            p.v[0] = ld(F, so, om2);
            p.v[1] = ld(F, so, om1);
            p.v[3] = ld(F, so, op1);
        }
        if (DUX[d] < 0) {
            p.v[1] = ld(F, so, om1);
            p.v[3] = ld(F, so, op1);
            p.v[4] = ld(F, so, op2);
        }
    };
    auto by_loads = [&]() {
        VelAcc va;                              // velocity of the new state (for A_hat)
        PlaneLoads cur, nxt;
        double lm2 = 0.0, lm1 = 0.0, lp1 = 0.0, lp2 = 0.0;
        load_plane(0, cur);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i + 1 < NV) {
                load_plane(i + 1, nxt);
            } else {
                lm2 = ld(L, 0u, om2);
                lm1 = ld(L, 0u, om1);
                lp1 = ld(L, 0u, op1);
                lp2 = ld(L, 0u, op2);
            }
            __builtin_amdgcn_sched_barrier(0);
            const int g = i / 8, d = i % 8;
            const double wx = ro(c->cx[g]);           // Courant number of the group
            const double f0 = cur.v[2];
            double a = f0;
            if (DUX[d] > 0) a = fma(-wx, nnd_pos(cur.v[0], cur.v[1], f0, cur.v[3]), a);
            if (DUX[d] < 0) a = fma(wx, nnd_neg(cur.v[1], f0, cur.v[3], cur.v[4]), a);
            double out = fma(dt, src[i], a);
            if (AMOD) vel_add(va, c, g, d, out);
            st(G, (uint32_t)i * pb, oc, out);
            cur = nxt;
        }
        if (AMOD) {
            st(Uo, 0u, oc, va.jx / va.r);
            st(Uo, opaque(Uo.plane_bytes), oc, va.jy / va.r);
        }
        const double dlx = nnd_upwind(m.ux > 0.0, lm2, lm1, lam, lp1, lp2);
        st(Lo, 0u, oc, lam + dlam - dt * (m.ux * (dlx * idx_)));
    };
    auto from_lanes = [&]() {
        const uint32_t halo = (uint32_t)(lane < 32 ? (lane == 0 ? j0 - 2 : j0 - 1) : (lane == 63 ? j0 + 65 : j0 + 64)) * 8u;
        VelAcc va;
        double hcur = ld(F, 0u, halo), hnxt = 0.0, hlam = 0.0;    // plane 0 moves along x
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i + 1 < NV) {
                if (DUX[(i + 1) & 7] != 0) hnxt = ld(F, (uint32_t)(i + 1) * pb, halo);
            } else {
                hlam = ld(L, 0u, halo);
            }
            __builtin_amdgcn_sched_barrier(0);
            const int g = i / 8, d = i % 8;
            const double wx = ro(c->cx[g]);
            const double f0 = stash[i * kBatchThreads];
            double a = f0;
            if (DUX[d] != 0) {
                const XNeighbours n = x_neighbours(f0, hcur);
                if (DUX[d] > 0) a = fma(-wx, nnd_pos(n.m2, n.m1, f0, n.p1), a);
                if (DUX[d] < 0) a = fma(wx, nnd_neg(n.m1, f0, n.p1, n.p2), a);
            }
            double out = fma(dt, src[i], a);
            if (AMOD) vel_add(va, c, g, d, out);
            st(G, (uint32_t)i * pb, oc, out);
            hcur = hnxt;
        }
        if (AMOD) {
            st(Uo, 0u, oc, va.jx / va.r);
            st(Uo, opaque(Uo.plane_bytes), oc, va.jy / va.r);
        }
        const XNeighbours n = x_neighbours(lam, hlam);
        const double dlx = nnd_upwind(m.ux > 0.0, n.m2, n.m1, lam, n.p1, n.p2);
        st(Lo, 0u, oc, lam + dlam - dt * (m.ux * (dlx * idx_)));
    };
    if (by_lanes)
        from_lanes();
    else
        by_loads();
}

template <bool AMOD, bool CHEM, bool GEXP>
__global__ __launch_bounds__(kBatchThreads) void k_batch(const Consts* __restrict__ c,
                                                         const BatchInst* __restrict__ inst,
                                                         const BatchSeg* __restrict__ segs,
                                                         const int32_t* __restrict__ wg_seg, int nwg,
                                                         double* f0, double* f1, double* l0, double* l1,
                                                         double* u0, double* u1, int64_t steps, int parity,
                                                         uint32_t* flags, int32_t* err) {
    // Ranges are dealt to the XCDs in contiguous bands (the hardware hands consecutive
    // work-group ids to the eight XCDs in turn), so neighbouring ranges, which exchange
    // halos every step, mostly share an L2.  nwg is a multiple of 8 or below 8.
    const int b8 = (int)blockIdx.x;
    const int w = nwg >= 8 ? (b8 % 8) * (nwg / 8) + b8 / 8 : b8;
    const int sbeg = wg_seg[w], send = wg_seg[w + 1];
    __shared__ int32_t stop;
    __shared__ double stash[NV * kBatchThreads];       // each thread's centre values (own slots)
    // the descriptors are swapped after every step (selecting them by step parity inside
    // the loop would turn them into per-lane values)
    Soa F = soa(parity ? f1 : f0, c->plane), G = soa(parity ? f0 : f1, c->plane);
    Soa L = soa(parity ? l1 : l0, 0), Lo = soa(parity ? l0 : l1, 0);
    Soa Ui = soa(parity ? u1 : u0, c->plane), Uo = soa(parity ? u0 : u1, c->plane);
    for (int64_t s = 0; s < steps; ++s) {
        if (s > 0) {
            if (threadIdx.x == 0) {
                const uint32_t want = (uint32_t)s;
                const bool ok = wait_counter(flags, w - 1, nwg, want, err) &&
                                wait_counter(flags, w + 1, nwg, want, err);
                if (!ok) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                stop = ok ? 0 : 1;
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(stop)) return;   // uniform over the work-group
        }
        for (int q = sbeg; q < send; ++q) {
            const BatchSeg S = segs[q];
            const BatchInst* I = inst + S.inst;
            // uniform trip count; the tail is masked
            for (int base = S.begin; base < S.end; base += kBatchThreads) {
                const int j = base + (int)threadIdx.x;
                if (j < S.end)
                    cell_1d<AMOD, CHEM, GEXP>(c, I, S.lo, S.hi, S.end, j, F, G, L, Lo, Ui, Uo,
                                              stash + threadIdx.x);
            }
        }
        // The barrier orders every thread's stores before thread 0's release (cumulative),
        // so one device-scope release per work-group publishes the whole range.
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(flags + w, (uint32_t)(s + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        Soa t = F;
        F = G;
        G = t;
        t = L;
        L = Lo;
        Lo = t;
        t = Ui;
        Ui = Uo;
        Uo = t;
    }
}

// clears the step counters before each persistent launch (a kernel, so that the clear can
// sit in a captured graph)
__global__ void k_zero_u32(uint32_t* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// One step of every instance, one packed cell per thread: the launch-per-step form of
// k_batch (its launches replayed from a captured graph, the kernel boundary orders the
// steps).  Wave w holds cells [64 w, 64 w + 64) and takes the instances that overlap it,
// wave_inst[2 w] .. wave_inst[2 w + 1], one at a time, so that an instance's rates are
// uniform over the wave; the cells are updated by the same code as in k_batch.
template <bool AMOD, bool CHEM, bool GEXP>
__global__ __launch_bounds__(kBatchThreads, 3) void k_batch_step(const Consts* __restrict__ c,
                                                                 const BatchInst* __restrict__ inst,
                                                                 const int32_t* __restrict__ wave_inst, int nwaves,
                                                                 const double* f_in, double* f_out,
                                                                 const double* l_in, double* l_out,
                                                                 const double* u_in, double* u_out) {
    __shared__ double stash[NV * kBatchThreads];       // each thread's centre values (own slots)
    const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kBatchThreads / 64) + (threadIdx.x >> 6)));
    if (w >= nwaves) return;                           // whole waves
    const int j = (int)(blockIdx.x * kBatchThreads + threadIdx.x);
    const int64_t plane = ro(c->plane);
    const Soa F = soa(f_in, plane), G = soa(f_out, plane);
    const Soa L = soa(l_in, 0), Lo = soa(l_out, 0);
    const Soa Ui = soa(u_in, plane), Uo = soa(u_out, plane);
    const int k0 = ro(wave_inst[2 * w]), k1 = ro(wave_inst[2 * w + 1]);
    for (int k = k0; k <= k1; ++k) {
        const BatchInst* I = inst + k;
        const int lo = ro(I->lo), hi = ro(I->hi);
        if (j >= lo && j <= hi)
            cell_1d<AMOD, CHEM, GEXP>(c, I, lo, hi, hi + 1, j, F, G, L, Lo, Ui, Uo, stash + threadIdx.x);
    }
}

template <bool AMOD, bool CHEM, bool GEXP>
void launch_batch_step_kernel(const Consts* dc, BatchState* b, int parity, hipStream_t st) {
    const int q = parity & 1;
    hipLaunchKernelGGL((k_batch_step<AMOD, CHEM, GEXP>), dim3((b->nwaves + kBatchThreads / 64 - 1) / (kBatchThreads / 64)),
                       dim3(kBatchThreads), 0, st, dc, b->d_inst, b->d_wave_inst, b->nwaves, b->f[q], b->f[1 - q],
                       b->lam[q], b->lam[1 - q], b->u[q], b->u[1 - q]);
}

// one step launch per step, `steps` of them, starting from buffer parity `parity`
hipError_t launch_batch_steps(const Consts* dc, int flags, BatchState* b, int64_t steps, int parity, hipStream_t st) {
    for (int64_t s = 0; s < steps; ++s) {
        const int q = (int)((parity + s) & 1);
        switch (flags) {
            case 0: launch_batch_step_kernel<false, false, false>(dc, b, q, st); break;
            case 1: launch_batch_step_kernel<true, false, false>(dc, b, q, st); break;
            case 2: launch_batch_step_kernel<false, true, false>(dc, b, q, st); break;
            case 3: launch_batch_step_kernel<true, true, false>(dc, b, q, st); break;
            case 6: launch_batch_step_kernel<false, true, true>(dc, b, q, st); break;
            default: launch_batch_step_kernel<true, true, true>(dc, b, q, st); break;
        }
    }
    return hipGetLastError();
}

template <bool AMOD, bool CHEM, bool GEXP>
void launch_batch_kernel(const Consts* dc, BatchState* b, int64_t steps, int parity, hipStream_t st) {
    hipLaunchKernelGGL((k_batch<AMOD, CHEM, GEXP>), dim3(b->nwg), dim3(kBatchThreads), 0, st, dc, b->d_inst,
                       b->d_seg, b->d_wg_seg, b->nwg, b->f[0], b->f[1], b->lam[0], b->lam[1], b->u[0], b->u[1],
                       steps, parity, b->d_flags, b->d_err);
}

const void* batch_kernel_ptr(int flags) {
    switch (flags) {
        case 0: return (const void*)k_batch<false, false, false>;
        case 1: return (const void*)k_batch<true, false, false>;
        case 2: return (const void*)k_batch<false, true, false>;
        case 3: return (const void*)k_batch<true, true, false>;
        case 6: return (const void*)k_batch<false, true, true>;
        default: return (const void*)k_batch<true, true, true>;
    }
}

hipError_t launch_batch(const Consts* dc, int flags, BatchState* b, int64_t steps, int parity, hipStream_t st) {
    const int nflags = b->nwg + 2;
    hipLaunchKernelGGL(k_zero_u32, dim3((nflags + 255) / 256), dim3(256), 0, st, b->d_flags, nflags);
    switch (flags) {
        case 0: launch_batch_kernel<false, false, false>(dc, b, steps, parity, st); break;
        case 1: launch_batch_kernel<true, false, false>(dc, b, steps, parity, st); break;
        case 2: launch_batch_kernel<false, true, false>(dc, b, steps, parity, st); break;
        case 3: launch_batch_kernel<true, true, false>(dc, b, steps, parity, st); break;
        case 6: launch_batch_kernel<false, true, true>(dc, b, steps, parity, st); break;
        default: launch_batch_kernel<true, true, true>(dc, b, steps, parity, st); break;
    }
    return hipGetLastError();
}

int batch_flags(const Consts& c, const BatchState* b) {
    const bool chem = c.chem != 0;
    return (b->any_amod ? 1 : 0) | (chem ? 2 : 0) | ((chem && !(c.m_is_one && c.n_is_one)) ? 4 : 0);
}

void drop_graphs(BatchState* b) {
    for (int p = 0; p < 2; ++p) {
        if (b->exec[p]) (void)hipGraphExecDestroy(b->exec[p]);
        b->exec[p] = nullptr;
        b->exec_steps[p] = -1;
        b->exec_nwg[p] = -1;
        for (int r = 0; r < 2; ++r) {
            if (b->sexec[p][r]) (void)hipGraphExecDestroy(b->sexec[p][r]);
            b->sexec[p][r] = nullptr;
            b->sexec_steps[p][r] = -1;
        }
    }
}

// Cut the packed cells into nwg ranges and the ranges into per-instance segments.
lbkm_status build_decomposition(lbkm_ctx* ctx, int wgs_per_cu) {
    BatchState* b = ctx->batch;
    if (wgs_per_cu == 0) {                              // one launch per step: no ranges
        b->nwg = (b->nwaves + kBatchThreads / 64 - 1) / (kBatchThreads / 64);
        b->wgs_per_cu = 0;
        drop_graphs(b);
        return LBKM_OK;
    }
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_kernel_ptr(batch_flags(ctx->h, b)),
                                                                 kBatchThreads, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "occupancy query");
    if (occ < 1) return fail(ctx, LBKM_EDEVICE, "batch kernel cannot be resident");
    const int per_cu = std::min(wgs_per_cu, occ);
    int nwg = std::max(1, b->cus * per_cu);
    nwg = (int)std::min<int64_t>(nwg, std::max<int64_t>(1, b->total / 64));
    if (nwg >= 8) nwg -= nwg % 8;                       // whole XCD bands (see k_batch)
    std::vector<BatchSeg> segs;
    std::vector<int32_t> wg_seg(nwg + 1, 0);
    int k = 0;
    for (int w = 0; w < nwg; ++w) {
        const int64_t a = b->total * w / nwg, z = b->total * (w + 1) / nwg;
        wg_seg[w] = (int32_t)segs.size();
        int64_t j = a;
        while (j < z) {
            while (k + 1 < b->n_inst && j >= b->off[k + 1]) ++k;
            const int64_t lo = b->off[k], hi = b->off[k] + b->nx[k] - 1;
            const int64_t end = std::min<int64_t>(z, hi + 1);
            segs.push_back(BatchSeg{k, (int32_t)j, (int32_t)end, (int32_t)lo, (int32_t)hi});
            j = end;
        }
    }
    wg_seg[nwg] = (int32_t)segs.size();
    if ((int)segs.size() > b->seg_cap || nwg + 2 > b->seg_cap) {
        if (b->d_seg) (void)hipFree(b->d_seg);
        if (b->d_wg_seg) (void)hipFree(b->d_wg_seg);
        if (b->d_flags) (void)hipFree(b->d_flags);
        b->d_seg = nullptr;
        b->d_wg_seg = nullptr;
        b->d_flags = nullptr;
        b->seg_cap = std::max((int)segs.size(), nwg + 2) * 2;
        e = hipMalloc((void**)&b->d_seg, sizeof(BatchSeg) * b->seg_cap);
        if (e == hipSuccess) e = hipMalloc((void**)&b->d_wg_seg, sizeof(int32_t) * (b->seg_cap + 1));
        if (e == hipSuccess) e = hipMalloc((void**)&b->d_flags, sizeof(uint32_t) * (b->seg_cap + 2));
        if (e != hipSuccess) return hip_fail(ctx, e, "batch decomposition allocation");
    }
    e = hipMemcpy(b->d_seg, segs.data(), sizeof(BatchSeg) * segs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_wg_seg, wg_seg.data(), sizeof(int32_t) * (nwg + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch decomposition upload");
    b->nwg = nwg;
    b->wgs_per_cu = per_cu;
    drop_graphs(b);
    return LBKM_OK;
}

lbkm_status batch_ready(lbkm_ctx* ctx, bool need_fields) {
    if (!ctx) return LBKM_EINVAL;
    if (!ctx->batched || !ctx->batch) return fail(ctx, LBKM_ESTATE, "not a batched context");
    if (!ctx->params) return fail(ctx, LBKM_ESTATE, "parameters not set");
    if (need_fields && !ctx->fields) return fail(ctx, LBKM_ESTATE, "fields not initialised");
    return LBKM_OK;
}

// One launch per step: graphs of kStepChunk launches (an even count, so the buffer parity
// is the same after each replay) and one of the remainder, cached per parity and count.
lbkm_status batch_run_steps(lbkm_ctx* ctx, int64_t n, hipStream_t st) {
    BatchState* b = ctx->batch;
    const int p = b->cur;
    hipError_t e = hipSuccess;
    auto ready = [&](int r, int64_t count) -> hipError_t {
        if (b->sexec[p][r] && b->sexec_steps[p][r] == count) return hipSuccess;
        if (b->sexec[p][r]) (void)hipGraphExecDestroy(b->sexec[p][r]);
        b->sexec[p][r] = nullptr;
        b->sexec_steps[p][r] = -1;
        hipError_t ce = hipSuccess;
        if (!b->cap) ce = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        hipGraph_t g = nullptr;
        if (ce == hipSuccess) ce = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (ce == hipSuccess) {
            hipError_t le = launch_batch_steps(ctx->d, batch_flags(ctx->h, b), b, count, p, b->cap);
            ce = hipStreamEndCapture(b->cap, &g);
            if (le != hipSuccess) ce = le;
        }
        if (ce == hipSuccess) ce = hipGraphInstantiate(&b->sexec[p][r], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (ce == hipSuccess) b->sexec_steps[p][r] = count;
        return ce;
    };
    const int64_t full = n / kStepChunk, rem = n % kStepChunk;
    if (full > 0) {
        e = ready(0, kStepChunk);
        for (int64_t i = 0; i < full && e == hipSuccess; ++i) e = hipGraphLaunch(b->sexec[p][0], st);
    }
    if (rem > 0 && e == hipSuccess) {
        e = ready(1, rem);
        if (e == hipSuccess) e = hipGraphLaunch(b->sexec[p][1], st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "batch step graphs");
    return LBKM_OK;
}

// run `n` steps through the graph cache (one graph per buffer parity and step count)
lbkm_status batch_run(lbkm_ctx* ctx, int64_t n, hipStream_t st) {
    BatchState* b = ctx->batch;
    if (n == 0) return LBKM_OK;
    const int p = b->cur;
    hipError_t e = hipSuccess;
    if (b->any_amod && !b->u_valid) {
        e = launch_velocity(ctx->d, (int)b->total, 1, b->f[p], b->u[p], st);
        if (e != hipSuccess) return hip_fail(ctx, e, "velocity kernel");
    }
    if (b->wgs_per_cu == 0) {
        const lbkm_status rs = batch_run_steps(ctx, n, st);
        if (rs != LBKM_OK) return rs;
        b->cur = (int)((p + n) & 1);
        b->u_valid = b->any_amod;
        ctx->steps += n;
        return LBKM_OK;
    }
    if (!b->exec[p] || b->exec_steps[p] != n || b->exec_nwg[p] != b->nwg) {
        if (b->exec[p]) (void)hipGraphExecDestroy(b->exec[p]);
        b->exec[p] = nullptr;
        if (!b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        hipGraph_t g = nullptr;
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = launch_batch(ctx->d, batch_flags(ctx->h, b), b, n, p, b->cap);
            e = hipStreamEndCapture(b->cap, &g);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[p], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(ctx, e, "batch graph capture");
        b->exec_steps[p] = n;
        b->exec_nwg[p] = b->nwg;
    }
    e = hipGraphLaunch(b->exec[p], st);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch graph launch");
    b->cur = (int)((p + n) & 1);
    b->u_valid = b->any_amod;
    ctx->steps += n;
    return LBKM_OK;
}

}  // namespace

void destroy_extras(lbkm_ctx* ctx) {
    BatchState* b = ctx->batch;
    if (!b) return;
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int i = 0; i < 2; ++i) {
        if (b->f[i]) (void)hipFree(b->f[i]);
        if (b->lam[i]) (void)hipFree(b->lam[i]);
        if (b->u[i]) (void)hipFree(b->u[i]);
    }
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_seg) (void)hipFree(b->d_seg);
    if (b->d_wg_seg) (void)hipFree(b->d_wg_seg);
    if (b->d_flags) (void)hipFree(b->d_flags);
    if (b->d_err) (void)hipFree(b->d_err);
    if (b->d_wave_inst) (void)hipFree(b->d_wave_inst);
    delete b;
    ctx->batch = nullptr;
}

}  // namespace lbkm

using namespace lbkm;

extern "C" {

lbkm_status lbkm_batch_create(int32_t n_inst, const int32_t* nx, const lbkm_grid* common, void* hip_stream,
                              lbkm_ctx** out) {
    if (!out) return LBKM_EINVAL;
    *out = nullptr;
    if (n_inst < 1 || !nx || !common) return LBKM_EINVAL;
    lbkm_ctx* ctx = new (std::nothrow) lbkm_ctx();
    if (!ctx) return LBKM_ENOMEM;
    *out = ctx;
    ctx->batched = 1;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->grid = *common;
    BatchState* b = new (std::nothrow) BatchState();
    if (!b) return fail(ctx, LBKM_ENOMEM, "host allocation");
    ctx->batch = b;
    b->n_inst = n_inst;
    b->nx.assign(nx, nx + n_inst);
    b->off.resize(n_inst);
    int64_t total = 0;
    for (int k = 0; k < n_inst; ++k) {
        if (nx[k] < 1) return fail(ctx, LBKM_EINVAL, "every instance needs nx >= 1");
        b->off[k] = (int32_t)total;
        total += nx[k];
        if (total >= (int64_t)1 << 28) return fail(ctx, LBKM_EINVAL, "too many cells in the batch (>= 2^28)");
    }
    b->total = total;
    b->plane = (total + 63) / 64 * 64;
    lbkm_grid g = *common;
    g.nx = (int32_t)total;
    g.ny = 1;
    g.bc_x = LBKM_BC_OUTFLOW;
    g.bc_y = LBKM_BC_PERIODIC;
    ctx->grid = g;
    lbkm_status st = validate_grid_common(ctx, &g);
    if (st == LBKM_OK) st = build_tables(ctx, &g);
    if (st != LBKM_OK) return st;
    ctx->h.pitch = b->plane;
    ctx->h.plane = b->plane;
    st = ensure_device_tables(ctx);
    if (st != LBKM_OK) return st;
    if ((int64_t)NV * b->plane * 8 > 0xFFFFFFFFll) return fail(ctx, LBKM_EINVAL, "batch state exceeds 4 GiB");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMalloc((void**)&b->f[i], sizeof(double) * NV * b->plane);
        if (e == hipSuccess) e = hipMalloc((void**)&b->lam[i], sizeof(double) * b->plane);
        if (e == hipSuccess) e = hipMalloc((void**)&b->u[i], sizeof(double) * 2 * b->plane);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_inst, sizeof(BatchInst) * n_inst);
    if (e == hipSuccess) {
        // per 64-cell wave of the packed cells: the first and the last instance it overlaps
        b->nwaves = (int)((total + 63) / 64);
        std::vector<int32_t> wi(2 * (size_t)b->nwaves);
        int k = 0;
        for (int w = 0; w < b->nwaves; ++w) {
            const int64_t a = 64 * (int64_t)w, z = std::min<int64_t>(a + 63, total - 1);
            while (k + 1 < n_inst && a >= b->off[k + 1]) ++k;
            int k1 = k;
            while (k1 + 1 < n_inst && z >= b->off[k1 + 1]) ++k1;
            wi[2 * (size_t)w] = k;
            wi[2 * (size_t)w + 1] = k1;
        }
        e = hipMalloc((void**)&b->d_wave_inst, sizeof(int32_t) * wi.size());
        if (e == hipSuccess) e = hipMemcpy(b->d_wave_inst, wi.data(), sizeof(int32_t) * wi.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_err, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(b->d_err, 0, sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(ctx, e, "batch allocation");
    b->h_inst.resize(n_inst);
    return LBKM_OK;
}

lbkm_status lbkm_batch_set_params(lbkm_ctx* ctx, const double* S, const double* Pr, double gamma, double Q,
                                  const lbkm_rates* rates) {
    if (!ctx) return LBKM_EINVAL;
    if (!ctx->batched || !ctx->batch) return fail(ctx, LBKM_ESTATE, "not a batched context");
    if (!S) return fail(ctx, LBKM_EINVAL, "NULL rates");
    BatchState* b = ctx->batch;
    Consts trial = ctx->h;
    bool any_amod = false;
    for (int k = 0; k < b->n_inst; ++k) {
        Consts ck = ctx->h;
        lbkm_status st = fill_physics(ctx, &ck, S + 24 * k, gamma, Pr ? Pr[k] : 0.0, Q, rates, ctx->grid.dt);
        if (st != LBKM_OK) return fail(ctx, st, "instance " + std::to_string(k) + ": " + ctx->err);
        if (k == 0) trial = ck;
        BatchInst& I = b->h_inst[k];
        std::memcpy(I.R, ck.R, sizeof(I.R));
        I.a8c = ck.a8c;
        I.a9c = ck.a9c;
        I.amod = ck.amod;
        I.lo = b->off[k];
        I.hi = b->off[k] + b->nx[k] - 1;
        any_amod |= ck.amod != 0;
    }
    ctx->h = trial;
    b->any_amod = any_amod;
    hipError_t e = hipMemcpy(b->d_inst, b->h_inst.data(), sizeof(BatchInst) * b->n_inst, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch parameter upload");
    ctx->params = true;
    lbkm_status st = upload_consts(ctx);
    if (st != LBKM_OK) return st;
    return build_decomposition(ctx, b->wgs_per_cu);
}

lbkm_status lbkm_batch_init_fields(lbkm_ctx* ctx, const double* rho, const double* ux, const double* uy,
                                   const double* T, const double* lambda) {
    lbkm_status st = batch_ready(ctx, false);
    if (st != LBKM_OK) return st;
    if (!rho || !ux || !uy || !T || !lambda) return fail(ctx, LBKM_EINVAL, "NULL field");
    BatchState* b = ctx->batch;
    b->cur = 0;
    b->u_valid = false;
    hipError_t e = hipMemsetAsync(b->d_err, 0, sizeof(int32_t), ctx->stream);   // a new run clears the error
    if (e == hipSuccess) e = launch_init(ctx->d, (int)b->total, 1, rho, ux, uy, T, lambda, b->f[0], b->lam[0], ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch init kernel");
    ctx->fields = true;
    ctx->steps = 0;
    return LBKM_OK;
}

lbkm_status lbkm_batch_step(lbkm_ctx* ctx, int64_t n) {
    lbkm_status st = batch_ready(ctx, true);
    if (st != LBKM_OK) return st;
    if (n < 0 || n > 0x7FFFFFFF) return fail(ctx, LBKM_EINVAL, "n out of range");
    return batch_run(ctx, n, ctx->stream);
}

lbkm_status lbkm_batch_autotune(lbkm_ctx* ctx, int32_t* cells_per_wg) {
    lbkm_status st = batch_ready(ctx, true);
    if (st != LBKM_OK) return st;
    BatchState* b = ctx->batch;
    // save the state, time a few steps per candidate, restore
    double *sf = nullptr, *sl = nullptr;
    hipError_t e = hipMalloc((void**)&sf, sizeof(double) * NV * b->plane);
    if (e == hipSuccess) e = hipMalloc((void**)&sl, sizeof(double) * b->plane);
    const int cur = b->cur;
    const int64_t steps0 = ctx->steps;
    if (e == hipSuccess) e = hipMemcpyAsync(sf, b->f[cur], sizeof(double) * NV * b->plane, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sl, b->lam[cur], sizeof(double) * b->plane, hipMemcpyDeviceToDevice, ctx->stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    int best = b->wgs_per_cu;
    float best_ms = 1e30f;
    const int cands[] = {0, 1, 2, 3, 4, 6, 8};          // 0: one launch per step
    for (int cand : cands) {
        if (e != hipSuccess) break;
        st = build_decomposition(ctx, cand);
        if (st != LBKM_OK) break;
        if (b->wgs_per_cu != cand) continue;                 // occupancy does not allow it
        const int64_t trial = 16;
        e = hipMemsetAsync(b->d_err, 0, sizeof(int32_t), ctx->stream);
        if (e != hipSuccess) break;
        st = batch_run(ctx, 2, ctx->stream);                  // warm-up (also captures)
        if (st == LBKM_OK) st = batch_run(ctx, trial, ctx->stream);   // capture the timed graph
        if (st != LBKM_OK) break;
        e = hipEventRecord(t0, ctx->stream);
        if (e == hipSuccess) st = batch_run(ctx, trial, ctx->stream);
        if (e == hipSuccess && st == LBKM_OK) e = hipEventRecord(t1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        int32_t err = 0;
        if (e == hipSuccess) e = hipMemcpy(&err, b->d_err, sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess && err == 0 && ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    }
    if (e == hipSuccess && st == LBKM_OK) st = build_decomposition(ctx, best);
    b->cur = cur;
    b->u_valid = false;            // the trial steps overwrote the velocity planes
    ctx->steps = steps0;
    if (e == hipSuccess) e = hipMemcpyAsync(b->f[cur], sf, sizeof(double) * NV * b->plane, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->lam[cur], sl, sizeof(double) * b->plane, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_err, 0, sizeof(int32_t), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (sf) (void)hipFree(sf);
    if (sl) (void)hipFree(sl);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch autotune");
    if (st != LBKM_OK) return st;
    if (cells_per_wg) *cells_per_wg = (int32_t)((b->total + b->nwg - 1) / b->nwg);
    return LBKM_OK;
}

lbkm_status lbkm_batch_set_launch(lbkm_ctx* ctx, int32_t wgs_per_cu) {
    lbkm_status st = batch_ready(ctx, false);
    if (st != LBKM_OK) return st;
    if (wgs_per_cu < 0 || wgs_per_cu > 16) return fail(ctx, LBKM_EINVAL, "wgs_per_cu must be in 0..16");
    st = build_decomposition(ctx, wgs_per_cu);
    if (st != LBKM_OK) return st;
    if (ctx->batch->wgs_per_cu != wgs_per_cu)
        return fail(ctx, LBKM_EINVAL, "the kernel's occupancy allows only " +
                                          std::to_string(ctx->batch->wgs_per_cu) + " work-groups per CU");
    return LBKM_OK;
}

lbkm_status lbkm_batch_get_moments(lbkm_ctx* ctx, double* rho, double* ux, double* uy, double* T, double* p,
                                   double* lambda) {
    lbkm_status st = batch_ready(ctx, true);
    if (st != LBKM_OK) return st;
    BatchState* b = ctx->batch;
    hipError_t e = launch_moments(ctx->d, (int)b->total, 1, b->f[b->cur], b->lam[b->cur], rho, ux, uy, T, p,
                                  lambda, ctx->stream);
    return e == hipSuccess ? LBKM_OK : hip_fail(ctx, e, "batch moments kernel");
}

lbkm_status lbkm_batch_total_cells(lbkm_ctx* ctx, int64_t* out) {
    if (!ctx || !out) return LBKM_EINVAL;
    if (!ctx->batched || !ctx->batch) return fail(ctx, LBKM_ESTATE, "not a batched context");
    *out = ctx->batch->total;
    return LBKM_OK;
}

lbkm_status lbkm_batch_status(lbkm_ctx* ctx, int32_t* wgs, int32_t* wgs_per_cu) {
    if (!ctx) return LBKM_EINVAL;
    if (!ctx->batched || !ctx->batch) return fail(ctx, LBKM_ESTATE, "not a batched context");
    int32_t err = 0;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(&err, ctx->batch->d_err, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch status");
    if (wgs) *wgs = ctx->batch->nwg;
    if (wgs_per_cu) *wgs_per_cu = ctx->batch->wgs_per_cu;
    if (err) return fail(ctx, LBKM_EDEVICE, "a neighbour wait exceeded its bound (work-groups not co-resident)");
    return LBKM_OK;
}

}  // extern "C"
