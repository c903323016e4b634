// Internal definitions shared by the host code and the HIP kernels of liblbkm.
#pragma once

#include <cstdint>

namespace lbkm {

constexpr int NV = 24;     // D2V24: 3 groups x 8 directions (Sec. II)

// Unit directions inside a group: (1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
// The moment matrix is block diagonal in the basis of mirror-symmetric combinations of
// these directions (even/odd under x -> -x and y -> -y):
//   EE: a0+a2, a1+a3, d0+d1+d2+d3        OE: a0-a2, d0-d1-d2+d3
//   EO: a1-a3, d0+d1-d2-d3               OO: d0-d1+d2-d3
// with a = axis directions 0..3 and d = diagonal directions 4..7.  Moments m_k (Sec. II)
// fall into the same four classes by the parity of their polynomial in v_x and v_y.
// 0-based moment indices of each class, in the order used for the blocks:
//   EE: m1 m4 m5 m7 m14 m16 m17 m19 m20     OE: m2 m8 m10 m12 m21 m23
//   EO: m3 m9 m11 m13 m22 m24               OO: m6 m15 m18
constexpr int NEE = 9, NOE = 6, NEO = 6, NOO = 3;

// The moment-matrix blocks, each stored column-major (X[k][r] is row r, column k) so that
// a kernel reads one column with one scalar load.
struct Mats {
    // forward blocks: f_hat(class) = B(class) * s(class), s = symmetric combinations
    double BEE[NEE][NEE], BOE[NOE][NOE], BEO[NEO][NEO], BOO[NOO][NOO];
    // inverse blocks with the 1/2 (axis) and 1/4 (diagonal) recombination factors folded in
    double CEE[NEE][NEE], COE[NOE][NOE], CEO[NEO][NEO], COO[NOO][NOO];
};
constexpr int kMatsDoubles = sizeof(Mats) / sizeof(double);

struct Consts {
    Mats mat;
    double vg[3];                 // group speeds v_a, v_b, v_c
    double eta2[3];               // eta_g^2
    double R[NV];                 // R_1..R_24
    double I, DI;                 // I and D + I
    double Q, w1, w2, pm, pn, Tig;
    double dt, inv_dx, inv_dy, half_inv_dx, half_inv_dy;
    double cx[3], cy[3];          // Courant numbers (dt v_g) / dx and (dt v_g) / dy of the groups
    double a8c, a9c;              // (R_5 - R_8)/R_5 and (R_7 - R_9)/R_7
    double inv_tau;               // 1/tau of the single-relaxation-time form
    int32_t srt;                  // 1: single relaxation time (Eq. SRT) instead of MRT
    int32_t amod;                 // 1 if A_hat_8 or A_hat_9 can be non-zero
    int32_t chem;                 // 1 if the reaction can run (omega1 or omega2 > 0)
    int32_t m_is_one, n_is_one;   // exponents equal to 1 (p^1 = p exactly)
    int32_t nx, ny, bc_x, bc_y;   // grid (batched kernels: nx unused)
    int64_t pitch, plane;         // row pitch and plane stride (elements)
    // wall boundaries of single sides (x_lo, x_hi, y_lo, y_hi): kWall* type, and for
    // Dirichlet / non-equilibrium-extrapolation walls the state (rho, T, u_x, u_y, lambda)
    int32_t wall[4];
    int32_t gL;                   // ghost buffer row length max(nx, ny)
    double wall_state[4][5];
};

// wall types of lbkm_set_boundary (0: the axis rule of bc_x / bc_y)
constexpr int kWallNone = 0, kWallReflect = 1, kWallDirichlet = 2, kWallNee = 3;
// ghost buffer gb[kGhostPlanes][4 sides][2 layers][gL]: planes 0..23 f, 24 lambda, 25 u_x,
// 26 u_y; layer 0 is the ghost next to the edge cell
constexpr int kGhostPlanes = NV + 3;

// Host: fill the velocity model and the block matrices of `c` from the DVM parameters.
// Returns 0 on success, -2 if M is singular or cond_inf(M) > 1e12; *cond receives the
// estimate.
int build_moment_blocks(const double dvm[6], Consts* c, double* cond);

// Host: dense M and M^-1 (24x24 row-major) reassembled from the blocks (for tests).
void dense_from_blocks(const Consts* c, double* M, double* Minv);

}  // namespace lbkm
