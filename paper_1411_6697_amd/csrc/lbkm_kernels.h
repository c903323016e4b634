// Launchers of the HIP kernels (defined in kernels.hip), called by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include "lbkm_internal.h"

namespace lbkm {

extern const int kStepVariants[][3];   // {tile_x, tile_y, mode} per launch variant (step.hip)
extern const int kNumStepVariants;
extern const int kWallTile[3];          // {tile_x, tile_y, mode} of the wall specialisation
int step_flags(const Consts& c);        // compile-time specialisation of the step kernel
// vertical != 0: XCD-contiguous bands of tile columns (when the tile columns divide by
// eight), else bands of tile rows
// uin/uout: [2][plane] velocity planes of the input and output state (used and written only
// when A_hat is active)
// Stage of a Runge-Kutta step: the output is a * (f^n, lambda^n at the cell) + b * (the
// forward-Euler update of the input state).  fn, ln = nullptr: f^n and lambda^n are the
// output buffers themselves (the stage writes over them; each thread reads its own cell
// before writing it); otherwise they must not overlap the output.
struct Blend {
    const double* fn;
    const double* ln;
    double a, b;
};
// bl == nullptr: a plain forward-Euler step.  gb != nullptr: some side is a wall; gb holds
// the ghost layers of the input state (launch_ghost) and the kWallTile (64 x 4 shared-centre)
// shape is used.
hipError_t launch_step(const Consts* dc, int variant, int flags, int nx, int ny, const double* fin,
                       double* fout, const double* lin, double* lout, const double* uin, double* uout,
                       int vertical, hipStream_t st, const Blend* bl = nullptr, const double* gb = nullptr);
// ghost layers of the wall sides of state (f, lam) into gb [kGhostPlanes][4][2][gL]
hipError_t launch_ghost(const Consts* dc, int nx, int ny, const double* f, const double* lam, double* gb,
                        hipStream_t st);
// velocity planes u[2][plane] of a state (pitched layout of the constants)
hipError_t launch_velocity(const Consts* dc, int nx, int ny, const double* f, double* u, hipStream_t st);
hipError_t launch_init(const Consts* dc, int nx, int ny, const double* rho, const double* ux,
                       const double* uy, const double* T, const double* lam, double* f, double* lout,
                       hipStream_t st);
hipError_t launch_moments(const Consts* dc, int nx, int ny, const double* f, const double* lam,
                          double* rho, double* ux, double* uy, double* T, double* p, double* lout,
                          hipStream_t st);
hipError_t launch_tne(const Consts* dc, int nx, int ny, const double* f, double* delta, double* dist,
                      hipStream_t st);
hipError_t launch_reduce(const Consts* dc, const double* f, const double* lam, double* partials,
                         int nblocks, double* out, hipStream_t st);
hipError_t launch_check(const Consts* dc, int nx, int ny, const double* f, const double* lam, int* flag,
                        hipStream_t st);
// min over cells with lambda < 1 of |T - T_ig| into out[0] (partials: nblocks doubles)
hipError_t launch_margin(const Consts* dc, const double* f, const double* lam, double* partials,
                         int nblocks, double* out, hipStream_t st);
hipError_t launch_copy_state(const Consts* dc, int nx, int ny, const double* src, double* dst, int planes,
                             int to_dense, hipStream_t st);

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st);

}  // namespace lbkm
