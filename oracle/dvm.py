"""D2V24 discrete-velocity model and the moment matrix M (oracle; test
infrastructure only).

Sec. II of the paper fixes 24 discrete velocities in three groups of eight.
Each group is the unit set {cyc (+-1, 0)} (four axis directions) followed by
{cyc (+-1, +-1)} (four diagonals), scaled by the group speed v_a, v_b or v_c,
and every velocity of a group carries the same internal-degree parameter
eta_a, eta_b or eta_c.  The paper does not fix the order inside "cyc"; this
oracle uses (1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1), which only
changes summation order.  The index ranges 1..8, 9..16, 17..24 read the
paper's overlapping "8 <= i <= 16" as 9..16.

The moment matrix has rows m_1..m_24 as listed after the matrix form of the
moment relations (Sec. II, Eq. moment12).  The paper inverts M symbolically
before the main loop (Sec. II end, Sec. V); here M is built in exact rational
arithmetic from the float64 values of the velocity parameters and inverted
exactly with Gauss-Jordan elimination over the rationals, then every entry is
rounded once to float64.  The result is the correctly rounded inverse of the
exact matrix.

Pins: M^-1 M = I (tests), Gauss-Hermite Maxwellian moments reproduce the
closed-form equilibrium moments (tests, through model.equilibrium_moments),
conservation of the collision operator (tests).
"""

from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

# Unit vectors of one group, in the order used throughout this oracle.
UNIT = ((1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1))


@dataclass(frozen=True)
class DVM:
    """Velocity-model parameters (v_a, v_b, v_c, eta_a, eta_b, eta_c), Sec. II."""
    va: float
    vb: float
    vc: float
    eta_a: float
    eta_b: float
    eta_c: float

    def groups(self):
        return ((self.va, self.eta_a), (self.vb, self.eta_b), (self.vc, self.eta_c))


def velocity_set(dvm: DVM):
    """Return float64 arrays vx[24], vy[24], eta[24] of the D2V24 model (Sec. II)."""
    vx, vy, eta = [], [], []
    for speed, e in dvm.groups():
        for ux, uy in UNIT:
            vx.append(speed * ux)
            vy.append(speed * uy)
            eta.append(e)
    return np.array(vx, dtype=np.float64), np.array(vy, dtype=np.float64), \
        np.array(eta, dtype=np.float64)


def _moment_row_values(vx: Fraction, vy: Fraction, eta: Fraction):
    """The 24 polynomial moments m_1..m_24 of one velocity (Sec. II, after Eq. moment12)."""
    v2 = vx * vx + vy * vy          # v_i^2
    q = v2 + eta * eta              # v_i^2 + eta_i^2
    h = eta * eta                   # eta_i^2
    return [
        Fraction(1),                # m1  = 1
        vx,                         # m2  = v_x
        vy,                         # m3  = v_y
        q,                          # m4  = v^2 + eta^2
        vx * vx,                    # m5  = v_x^2
        vx * vy,                    # m6  = v_x v_y
        vy * vy,                    # m7  = v_y^2
        q * vx,                     # m8  = (v^2+eta^2) v_x
        q * vy,                     # m9  = (v^2+eta^2) v_y
        vx * vx * vx,               # m10 = v_x^3
        vx * vx * vy,               # m11 = v_x^2 v_y
        vx * vy * vy,               # m12 = v_x v_y^2
        vy * vy * vy,               # m13 = v_y^3
        q * vx * vx,                # m14 = (v^2+eta^2) v_x^2
        q * vx * vy,                # m15 = (v^2+eta^2) v_x v_y
        q * vy * vy,                # m16 = (v^2+eta^2) v_y^2
        h * vx * vx,                # m17 = eta^2 v_x^2
        h * vx * vy,                # m18 = eta^2 v_x v_y
        h * vy * vy,                # m19 = eta^2 v_y^2
        q * h,                      # m20 = (v^2+eta^2) eta^2
        q * v2 * vx,                # m21 = (v^2+eta^2) v^2 v_x
        q * v2 * vy,                # m22 = (v^2+eta^2) v^2 v_y
        q * h * vx,                 # m23 = (v^2+eta^2) eta^2 v_x
        q * h * vy,                 # m24 = (v^2+eta^2) eta^2 v_y
    ]


def moment_matrix_exact(dvm: DVM):
    """M as a 24x24 list of exact rationals; M[k][i] = m_{k+1}(velocity i+1)."""
    vx, vy, eta = velocity_set(dvm)
    cols = [_moment_row_values(Fraction(float(a)), Fraction(float(b)), Fraction(float(c)))
            for a, b, c in zip(vx, vy, eta)]
    return [[cols[i][k] for i in range(24)] for k in range(24)]


def _invert_exact(a):
    """Gauss-Jordan elimination over the rationals.  Raises ZeroDivisionError if singular."""
    n = len(a)
    w = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(a)]
    for c in range(n):
        piv = next((r for r in range(c, n) if w[r][c] != 0), None)
        if piv is None:
            raise ZeroDivisionError("moment matrix is singular for this velocity model")
        w[c], w[piv] = w[piv], w[c]
        pv = w[c][c]
        w[c] = [x / pv for x in w[c]]
        for r in range(n):
            if r != c and w[r][c] != 0:
                fac = w[r][c]
                w[r] = [x - fac * y for x, y in zip(w[r], w[c])]
    return [row[n:] for row in w]


def moment_matrix(dvm: DVM) -> np.ndarray:
    """M in float64, each entry the correctly rounded exact polynomial value."""
    return np.array([[float(x) for x in row] for row in moment_matrix_exact(dvm)],
                    dtype=np.float64)


def inverse_moment_matrix(dvm: DVM) -> np.ndarray:
    """M^-1 in float64, each entry the correctly rounded exact rational inverse."""
    inv = _invert_exact(moment_matrix_exact(dvm))
    return np.array([[float(x) for x in row] for row in inv], dtype=np.float64)
