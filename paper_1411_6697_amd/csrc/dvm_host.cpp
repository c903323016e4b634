// Host construction of the D2V24 moment matrix in symmetry-block form.
//
// The paper inverts M symbolically before the main loop and substitutes numbers
// (Sec. II end, Sec. V).  Here each mirror-symmetry block of M is built from the
// moment polynomials of Sec. II in long double and inverted by Gauss elimination with
// partial pivoting followed by two rounds of iterative refinement, also in long double,
// so the rounded float64 inverse is accurate to about one unit in the last place even
// for the ill-conditioned velocity sets the paper uses (cond(M) up to ~3e5).

#include <cmath>
#include <cstring>

#include "lbkm_internal.h"

namespace lbkm {

namespace {

constexpr int UX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
constexpr int UY[8] = {0, 1, 0, -1, 1, 1, -1, -1};

constexpr int EE_M[NEE] = {0, 3, 4, 6, 13, 15, 16, 18, 19};
constexpr int OE_M[NOE] = {1, 7, 9, 11, 20, 22};
constexpr int EO_M[NEO] = {2, 8, 10, 12, 21, 23};
constexpr int OO_M[NOO] = {5, 14, 17};
// representative direction of each combination slot within a group
constexpr int REP_EE[3] = {0, 1, 4};
constexpr int REP_OE[2] = {0, 4};
constexpr int REP_EO[2] = {1, 4};
constexpr int REP_OO[1] = {4};

typedef long double ld;

// m_1..m_24 of one velocity (Sec. II, the rows of M)
void moment_rows(ld vx, ld vy, ld eta, ld out[NV]) {
    const ld v2 = vx * vx + vy * vy, h = eta * eta, q = v2 + h;
    const ld r[NV] = {1.0L, vx, vy, q, vx * vx, vx * vy, vy * vy, q * vx, q * vy,
                      vx * vx * vx, vx * vx * vy, vx * vy * vy, vy * vy * vy,
                      q * vx * vx, q * vx * vy, q * vy * vy,
                      h * vx * vx, h * vx * vy, h * vy * vy, q * h,
                      q * v2 * vx, q * v2 * vy, q * h * vx, q * h * vy};
    for (int k = 0; k < NV; ++k) out[k] = r[k];
}

// Solve A X = I for an n x n long-double matrix (row-major), n <= 9.
bool invert(int n, const ld* A, ld* X) {
    ld LU[81];
    int piv[9];
    std::memcpy(LU, A, sizeof(ld) * n * n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(LU[r * n + c]) > fabsl(LU[p * n + c])) p = r;
        if (LU[p * n + c] == 0.0L) return false;
        piv[c] = p;
        if (p != c)
            for (int k = 0; k < n; ++k) { ld t = LU[c * n + k]; LU[c * n + k] = LU[p * n + k]; LU[p * n + k] = t; }
        for (int r = c + 1; r < n; ++r) {
            LU[r * n + c] /= LU[c * n + c];
            for (int k = c + 1; k < n; ++k) LU[r * n + k] -= LU[r * n + c] * LU[c * n + k];
        }
    }
    auto solve = [&](ld* b) {   // in place, b of length n
        for (int c = 0; c < n; ++c) { ld t = b[c]; b[c] = b[piv[c]]; b[piv[c]] = t; }
        for (int r = 0; r < n; ++r)
            for (int k = 0; k < r; ++k) b[r] -= LU[r * n + k] * b[k];
        for (int r = n - 1; r >= 0; --r) {
            for (int k = r + 1; k < n; ++k) b[r] -= LU[r * n + k] * b[k];
            b[r] /= LU[r * n + r];
        }
    };
    for (int j = 0; j < n; ++j) {
        ld x[9], res[9];
        for (int r = 0; r < n; ++r) x[r] = (r == j) ? 1.0L : 0.0L;
        solve(x);
        for (int it = 0; it < 2; ++it) {          // iterative refinement
            for (int r = 0; r < n; ++r) {
                ld s = (r == j) ? 1.0L : 0.0L;
                for (int k = 0; k < n; ++k) s -= A[r * n + k] * x[k];
                res[r] = s;
            }
            solve(res);
            for (int r = 0; r < n; ++r) x[r] += res[r];
        }
        for (int r = 0; r < n; ++r) X[r * n + j] = x[r];
    }
    return true;
}

}  // namespace

int build_moment_blocks(const double dvm[6], Consts* c, double* cond) {
    ld M[NV][NV];
    for (int g = 0; g < 3; ++g) {
        c->vg[g] = dvm[g];
        c->eta2[g] = dvm[3 + g] * dvm[3 + g];
        for (int d = 0; d < 8; ++d) {
            ld col[NV];
            moment_rows((ld)dvm[g] * UX[d], (ld)dvm[g] * UY[d], (ld)dvm[3 + g], col);
            for (int k = 0; k < NV; ++k) M[k][8 * g + d] = col[k];
        }
    }
    ld bee[NEE * NEE], boe[NOE * NOE], beo[NEO * NEO], boo[NOO * NOO];
    for (int g = 0; g < 3; ++g) {
        for (int r = 0; r < NEE; ++r)
            for (int s = 0; s < 3; ++s) bee[r * NEE + 3 * g + s] = M[EE_M[r]][8 * g + REP_EE[s]];
        for (int r = 0; r < NOE; ++r)
            for (int s = 0; s < 2; ++s) boe[r * NOE + 2 * g + s] = M[OE_M[r]][8 * g + REP_OE[s]];
        for (int r = 0; r < NEO; ++r)
            for (int s = 0; s < 2; ++s) beo[r * NEO + 2 * g + s] = M[EO_M[r]][8 * g + REP_EO[s]];
        for (int r = 0; r < NOO; ++r) boo[r * NOO + g] = M[OO_M[r]][8 * g + REP_OO[0]];
    }
    ld iee[NEE * NEE], ioe[NOE * NOE], ieo[NEO * NEO], ioo[NOO * NOO];
    if (!invert(NEE, bee, iee) || !invert(NOE, boe, ioe) || !invert(NEO, beo, ieo) ||
        !invert(NOO, boo, ioo)) {
        *cond = INFINITY;
        return -2;
    }
    // recombination factors: axis pairs 1/2, diagonal quadruples 1/4
    auto fac_ee = [](int row) { return (row % 3 == 2) ? 0.25L : 0.5L; };
    auto fac_2 = [](int row) { return (row % 2 == 1) ? 0.25L : 0.5L; };
    for (int r = 0; r < NEE; ++r)
        for (int k = 0; k < NEE; ++k) {
            c->mat.BEE[k][r] = (double)bee[r * NEE + k];
            c->mat.CEE[k][r] = (double)(fac_ee(r) * iee[r * NEE + k]);
        }
    for (int r = 0; r < NOE; ++r)
        for (int k = 0; k < NOE; ++k) {
            c->mat.BOE[k][r] = (double)boe[r * NOE + k];
            c->mat.COE[k][r] = (double)(fac_2(r) * ioe[r * NOE + k]);
            c->mat.BEO[k][r] = (double)beo[r * NEO + k];
            c->mat.CEO[k][r] = (double)(fac_2(r) * ieo[r * NEO + k]);
        }
    for (int r = 0; r < NOO; ++r)
        for (int k = 0; k < NOO; ++k) {
            c->mat.BOO[k][r] = (double)boo[r * NOO + k];
            c->mat.COO[k][r] = (double)(0.25L * ioo[r * NOO + k]);
        }
    // condition estimate of the dense M: ||M||_inf ||M^-1||_inf
    double Md[NV * NV], Mi[NV * NV];
    dense_from_blocks(c, Md, Mi);
    double nm = 0, ni = 0;
    for (int r = 0; r < NV; ++r) {
        double a = 0, b = 0;
        for (int k = 0; k < NV; ++k) { a += std::fabs(Md[r * NV + k]); b += std::fabs(Mi[r * NV + k]); }
        nm = a > nm ? a : nm;
        ni = b > ni ? b : ni;
    }
    *cond = nm * ni;
    if (!(*cond <= 1e12)) return -2;
    return 0;
}

void dense_from_blocks(const Consts* c, double* M, double* Minv) {
    // Forward: column i = 8g+d of M from the block entry of its class, with the sign of
    // the direction's parity (see the basis in lbkm_internal.h).
    std::memset(M, 0, sizeof(double) * NV * NV);
    std::memset(Minv, 0, sizeof(double) * NV * NV);
    // sign of direction d inside each combination slot
    const int sEE[3][8] = {{1, 0, 1, 0, 0, 0, 0, 0}, {0, 1, 0, 1, 0, 0, 0, 0}, {0, 0, 0, 0, 1, 1, 1, 1}};
    const int sOE[2][8] = {{1, 0, -1, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 1, -1, -1, 1}};
    const int sEO[2][8] = {{0, 1, 0, -1, 0, 0, 0, 0}, {0, 0, 0, 0, 1, 1, -1, -1}};
    const int sOO[1][8] = {{0, 0, 0, 0, 1, -1, 1, -1}};
    for (int g = 0; g < 3; ++g)
        for (int d = 0; d < 8; ++d) {
            const int i = 8 * g + d;
            for (int s = 0; s < 3; ++s)
                if (sEE[s][d])
                    for (int r = 0; r < NEE; ++r) {
                        M[EE_M[r] * NV + i] = sEE[s][d] * c->mat.BEE[3 * g + s][r];
                        Minv[i * NV + EE_M[r]] += sEE[s][d] * c->mat.CEE[r][3 * g + s];
                    }
            for (int s = 0; s < 2; ++s) {
                if (sOE[s][d])
                    for (int r = 0; r < NOE; ++r) {
                        M[OE_M[r] * NV + i] = sOE[s][d] * c->mat.BOE[2 * g + s][r];
                        Minv[i * NV + OE_M[r]] += sOE[s][d] * c->mat.COE[r][2 * g + s];
                    }
                if (sEO[s][d])
                    for (int r = 0; r < NEO; ++r) {
                        M[EO_M[r] * NV + i] = sEO[s][d] * c->mat.BEO[2 * g + s][r];
                        Minv[i * NV + EO_M[r]] += sEO[s][d] * c->mat.CEO[r][2 * g + s];
                    }
            }
            if (sOO[0][d])
                for (int r = 0; r < NOO; ++r) {
                    M[OO_M[r] * NV + i] = sOO[0][d] * c->mat.BOO[g][r];
                    Minv[i * NV + OO_M[r]] += sOO[0][d] * c->mat.COO[r][g];
                }
        }
}

}  // namespace lbkm
