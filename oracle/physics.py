"""Independent physics references used to pin the oracle (test infrastructure only).

None of this is the lattice Boltzmann method: these are the solutions the
paper compares its simulations with, computed from their own mathematics.

* exact_riemann  : exact solution of the Riemann problem of the 1D Euler
                   equations for an ideal gas (Sec. IV B compares the Sod, Lax
                   and Sjogreen problems with it).  Pressure-function Newton
                   iteration and self-similar sampling, as in standard
                   gas-dynamics texts (e.g. Toro, ch. 4).
* cj_state       : Chapman-Jouguet detonation state and speed for a quiescent
                   ideal gas with heat release Q (Sec. IV A).
* von_neumann_state : the state right behind the leading shock of a CJ
                   detonation (the ZND spike, Sec. IV A and Sec. VI).
* maxwellian_moments : moments of the continuous equilibrium distribution
                   Eq. feq_continuous by tensor Gauss-Hermite quadrature.
* maxwellian     : Eq. feq_continuous itself, evaluated pointwise.
"""

from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# Exact Riemann solver (ideal gas)
# --------------------------------------------------------------------------

def _pressure_fn(p, rho_k, p_k, c_k, g):
    """f_k(p) and f_k'(p): velocity jump across the left or right wave."""
    if p > p_k:                                   # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        return (p - p_k) * s, s * (1.0 - 0.5 * (p - p_k) / (p + B))
    r = p / p_k                                   # rarefaction
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * c_k / (g - 1.0) * (r ** e - 1.0), 1.0 / (rho_k * c_k) * r ** (-(g + 1.0) / (2.0 * g))


def riemann_star(left, right, g):
    """Star-region pressure and velocity (p*, u*) for left/right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    du = ur - ul
    if 2.0 * (cl + cr) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated")
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _pressure_fn(p, rl, pl, cl, g)
        fr, dfr = _pressure_fn(p, rr, pr, cr, g)
        dp = (fl + fr + du) / (dfl + dfr)
        p_new = max(1e-14, p - dp)
        if abs(p_new - p) <= 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _pressure_fn(p, rl, pl, cl, g)
    fr, _ = _pressure_fn(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def riemann_sample(left, right, g, xi):
    """Exact solution (rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = riemann_star(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for k, s in enumerate(xi.ravel()):
        if s <= us:                                      # left of the contact
            if ps > pl:                                  # left shock
                sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if s <= sl:
                    st = (rl, ul, pl)
                else:
                    st = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:                                        # left rarefaction
                cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                if s <= ul - cl:
                    st = (rl, ul, pl)
                elif s >= us - cs:
                    st = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    uu = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    rr_ = rl * (c / cl) ** (2.0 / (g - 1.0))
                    st = (rr_, uu, pl * (c / cl) ** (2.0 * g / (g - 1.0)))
        else:                                            # right of the contact
            if ps > pr:                                  # right shock
                sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if s >= sr:
                    st = (rr, ur, pr)
                else:
                    st = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:                                        # right rarefaction
                cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                if s >= ur + cr:
                    st = (rr, ur, pr)
                elif s <= us + cs:
                    st = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    uu = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    rr_ = rr * (c / cr) ** (2.0 / (g - 1.0))
                    st = (rr_, uu, pr * (c / cr) ** (2.0 * g / (g - 1.0)))
        rho.flat[k], u.flat[k], p.flat[k] = st
    return rho, u, p


# --------------------------------------------------------------------------
# Detonation states
# --------------------------------------------------------------------------

def oblique_shock(rho, p, speed, g, theta):
    """Weak oblique shock that turns a uniform supersonic stream (density rho, pressure p,
    speed `speed`) by the angle theta (radians, 0 < theta < the detachment angle).  Shock
    angle beta from the theta-beta-M relation tan(theta) = 2 cot(beta) (M^2 sin^2(beta) - 1) /
    (M^2 (g + cos 2 beta) + 2), weak root by bisection between the Mach angle and the
    angle of maximum deflection; downstream state from the normal-shock jumps of the normal
    Mach number M sin(beta).  Returns dict(beta, rho, p, speed) downstream."""
    c = math.sqrt(g * p / rho)
    M = speed / c
    f = lambda b: 2.0 / math.tan(b) * (M * M * math.sin(b) ** 2 - 1.0) / (M * M * (g + math.cos(2 * b)) + 2.0)
    lo = math.asin(1.0 / M)
    grid = [lo + (math.pi / 2 - lo) * k / 2000.0 for k in range(1, 2000)]
    hi = max(grid, key=f)                       # angle of maximum deflection
    if f(hi) < math.tan(theta):
        raise ValueError("deflection beyond the detachment angle")
    a, b = lo, hi
    for _ in range(200):
        m = 0.5 * (a + b)
        if f(m) < math.tan(theta):
            a = m
        else:
            b = m
    beta = 0.5 * (a + b)
    mn = M * math.sin(beta)
    rho2 = rho * (g + 1.0) * mn * mn / ((g - 1.0) * mn * mn + 2.0)
    p2 = p * (1.0 + 2.0 * g / (g + 1.0) * (mn * mn - 1.0))
    mn2 = math.sqrt((1.0 + 0.5 * (g - 1.0) * mn * mn) / (g * mn * mn - 0.5 * (g - 1.0)))
    M2 = mn2 / math.sin(beta - theta)
    return {"beta": beta, "rho": rho2, "p": p2, "speed": M2 * math.sqrt(g * p2 / rho2)}


def cj_state(rho0, p0, Q, g):
    """Chapman-Jouguet state behind a detonation moving into quiescent gas.

    Solving the Rankine-Hugoniot relations with heat release Q and the Rayleigh
    line tangent to the Hugoniot gives the CJ Mach number
    M = sqrt(1 + H) + sqrt(H), H = (g^2 - 1) Q / (2 c0^2).  Returns a dict with
    speed D, density, pressure, temperature T = p / rho and particle velocity u."""
    c0 = math.sqrt(g * p0 / rho0)
    H = (g * g - 1.0) * Q / (2.0 * c0 * c0)
    M = math.sqrt(1.0 + H) + math.sqrt(H)
    Dv = M * c0
    p1 = p0 * (1.0 + g * M * M) / (g + 1.0)
    rho1 = rho0 * (g + 1.0) * M * M / (1.0 + g * M * M)
    u1 = Dv * (1.0 - rho0 / rho1)
    return {"D": Dv, "rho": rho1, "p": p1, "T": p1 / rho1, "u": u1, "M": M}


def von_neumann_state(rho0, p0, Q, g):
    """State right behind the inert leading shock travelling at the CJ speed."""
    cj = cj_state(rho0, p0, Q, g)
    M = cj["M"]
    p1 = p0 * (1.0 + 2.0 * g / (g + 1.0) * (M * M - 1.0))
    rho1 = rho0 * (g + 1.0) * M * M / ((g - 1.0) * M * M + 2.0)
    u1 = cj["D"] * (1.0 - rho0 / rho1)
    return {"rho": rho1, "p": p1, "T": p1 / rho1, "u": u1}


# --------------------------------------------------------------------------
# Maxwellian moments by quadrature
# --------------------------------------------------------------------------

def maxwellian_moments(rho, ux, uy, T, I, polys, npts: int = 12):
    """Integrals of polys(vx, vy, eta) against the continuous equilibrium
    Eq. feq_continuous, rho (2 pi T)^-1 (2 pi I T)^-1/2 exp(-|v-u|^2/(2T) - eta^2/(2 I T)),
    computed with an npts-point Gauss-Hermite rule in each of vx, vy, eta (exact
    for polynomials of degree < 2 npts).  `polys` maps arrays (vx, vy, eta) to a
    list of arrays; returns a float64 array of the moments."""
    x, w = np.polynomial.hermite_e.hermegauss(npts)    # weight exp(-x^2/2)
    w = w / math.sqrt(2.0 * math.pi)                   # standard-normal weights
    sx, se = math.sqrt(T), math.sqrt(I * T)
    VX, VY, ET = np.meshgrid(ux + sx * x, uy + sx * x, se * x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return np.array([rho * np.sum(W * p) for p in polys(VX, VY, ET)])


def maxwellian(rho, ux, uy, T, I, vx, vy, eta, D: int = 2):
    """The continuous equilibrium distribution of Eq. feq_continuous evaluated at the
    velocity (vx, vy) and internal-degree variable eta:
    rho (2 pi T)^(-D/2) (2 pi I T)^(-1/2) exp(-|v - u|^2 / (2 T) - eta^2 / (2 I T))."""
    c2 = (vx - ux) ** 2 + (vy - uy) ** 2
    return rho * (2.0 * math.pi * T) ** (-0.5 * D) * (2.0 * math.pi * I * T) ** -0.5 * \
        np.exp(-c2 / (2.0 * T) - eta * eta / (2.0 * I * T))
