"""One time step of the MRT lattice Boltzmann kinetic model for combustion
(oracle; test infrastructure only).

Every function here follows a passage of the paper (Xu, Lin, Zhang, Li,
arXiv:1411.6697) and is written for a reader who checks it against the paper
by eye: field arithmetic is done on whole float64 CPU tensors of shape
[24, Ny, Nx] (distribution functions) or [Ny, Nx] (scalar fields), dense 24x24
matrix products stand for f_hat = M f and M^-1 g, and nothing is blocked,
fused or reordered beyond what the equations state.

Where the paper is silent or garbled this file takes these readings (the same
ones the GPU library takes):

* Sign of the modification term (Eq. Boltzmann_chemical vs Eq. CE_LB): the
  moment-space source is  -R (f_hat - f_hat^eq) + A_hat, so the collision
  term in velocity space is  -M^-1 [R (f_hat - f_hat^eq) - A_hat].  Only this
  sign gives the viscous-heating coefficient rho T / R_5 claimed after
  Eq. NSEnergy_new.
* f_hat^eq_14 and f_hat^eq_16 carry the factor T on their first term, as
  Eq. moment7 requires (the printed list drops it).
* Time integration of f: first-order forward Euler, all terms at level n.
* Space: the NND scheme of Zhang (1988) in its flux-split minmod form, two
  cells upwind and one downwind; the upwind side is the sign of v_i_alpha for
  f_i and the sign of the local u_alpha for lambda.
* Derivatives of u inside A_8, A_9: second-order central differences.
* Chemistry: the Cochran equation with pressure frozen over a step is solved
  exactly (a Bernoulli equation); the rate F(lambda) in C_i is the realised
  increment divided by dt, so the released energy equals rho Q dlambda.
  The reaction runs only where T > T_ig (strict), lambda < 1 and the rate
  constant omega_1 p^m + omega_2 p^n is positive.
* C_i uses the discrete equilibrium f^eq = M^-1 f_hat^eq.
* Boundaries: two ghost cells per side, either periodic or zero-gradient
  (each ghost copies the edge cell).
* Delta_1..Delta_4 are zero by definition (conserved moments, Sec. VI).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from .dvm import DVM, velocity_set, moment_matrix, inverse_moment_matrix

D = 2.0  # spatial dimension (Sec. II)

PERIODIC = "periodic"
OUTFLOW = "outflow"


@dataclass
class Params:
    """Physical and numerical parameters of one run (Sec. II, Sec. IV)."""
    dvm: DVM
    I: float                      # extra degrees of freedom; gamma = (D+I+2)/(D+I)
    R: Sequence[float]            # R_1..R_24, the diagonal of R_hat
    dx: float
    dy: float
    dt: float
    Q: float = 0.0                # heat release per unit mass (Eq. chemical_energy)
    omega1: float = 0.0           # Cochran rate constants (Eq. lambda_equation)
    omega2: float = 0.0
    m: float = 1.0
    n: float = 1.0
    T_ig: float = 1.1             # ignition temperature
    bc_x: str = OUTFLOW
    bc_y: str = PERIODIC
    tau: float = 0.0              # > 0: single-relaxation-time collision of Eq. SRT (Sec. V)
    rk: int = 1                   # time scheme: 1 forward Euler, 2 / 3 SSP Runge-Kutta
    # boundaries of single sides that override bc_x / bc_y: {"x_lo" | "x_hi" | "y_lo" |
    # "y_hi": spec}, spec = ("reflect",) | ("dirichlet", rho, T, u_x, u_y, lambda) |
    # ("nee", T, u_x, u_y)  (see wall_layers)
    walls: Optional[dict] = None


@dataclass
class Tables:
    """Float64 CPU tensors used by the step.  R, Q, omega1, omega2 are tensors so
    that a test may ask autograd for derivatives with respect to them."""
    vx: torch.Tensor
    vy: torch.Tensor
    eta: torch.Tensor
    M: torch.Tensor
    Minv: torch.Tensor
    R: torch.Tensor
    Q: torch.Tensor
    omega1: torch.Tensor
    omega2: torch.Tensor


def make_tables(P: Params) -> Tables:
    vx, vy, eta = velocity_set(P.dvm)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
    return Tables(vx=t(vx), vy=t(vy), eta=t(eta),
                  M=t(moment_matrix(P.dvm)), Minv=t(inverse_moment_matrix(P.dvm)),
                  R=t(list(P.R)), Q=t(P.Q), omega1=t(P.omega1), omega2=t(P.omega2))


def _b(v: torch.Tensor, like: torch.Tensor) -> torch.Tensor:
    """Broadcast a [24] vector over the trailing spatial dims of `like`."""
    return v.reshape((-1,) + (1,) * (like.dim() - 1))


# --------------------------------------------------------------------------
# Equilibrium moments and macroscopic quantities
# --------------------------------------------------------------------------

def equilibrium_moments(rho, ux, uy, T, I: float) -> torch.Tensor:
    """f_hat^eq_1..24 (Sec. II, closed forms after Eq. moment12, derived from
    Eqs. moment1-moment11), with the factor T restored in entries 14 and 16
    as Eq. moment7 requires.  Returns a tensor [24, *rho.shape]."""
    u2 = ux * ux + uy * uy
    a2 = (D + I + 2.0) * T + u2        # (D+I+2)T + u^2
    a4 = (D + I + 4.0) * T + u2        # (D+I+4)T + u^2
    c10 = u2 * u2 + (D + 2.0) * (D + I + 4.0) * T * T + (2.0 * D + I + 8.0) * u2 * T
    c11 = u2 + (D + 3.0 * I + 2.0) * T
    rows = [
        rho,                                        # 1
        rho * ux,                                   # 2
        rho * uy,                                   # 3
        rho * ((D + I) * T + u2),                   # 4
        rho * (T + ux * ux),                        # 5
        rho * ux * uy,                              # 6
        rho * (T + uy * uy),                        # 7
        rho * ux * a2,                              # 8
        rho * uy * a2,                              # 9
        3.0 * rho * ux * T + rho * ux ** 3,         # 10
        rho * uy * T + rho * ux * ux * uy,          # 11
        rho * ux * T + rho * ux * uy * uy,          # 12
        3.0 * rho * uy * T + rho * uy ** 3,         # 13
        rho * a2 * T + rho * ux * ux * a4,          # 14 (factor T restored, Eq. moment7)
        rho * ux * uy * a4,                         # 15
        rho * a2 * T + rho * uy * uy * a4,          # 16 (factor T restored, Eq. moment7)
        rho * I * T * T + rho * ux * ux * I * T,    # 17
        rho * ux * uy * I * T,                      # 18
        rho * I * T * T + rho * uy * uy * I * T,    # 19
        rho * I * T * (u2 + (D + 3.0 * I) * T),     # 20
        rho * ux * c10,                             # 21
        rho * uy * c10,                             # 22
        rho * ux * I * T * c11,                     # 23
        rho * uy * I * T * c11,                     # 24
    ]
    return torch.stack(rows, dim=0)


def moment_transform(f: torch.Tensor, T: Tables) -> torch.Tensor:
    """f_hat_k = M_ki f_i (Sec. II, below Eq. Boltzmann_chemical)."""
    return torch.einsum("ki,i...->k...", T.M, f)


def macroscopic(fhat: torch.Tensor, I: float):
    """rho, u_x, u_y, T from the conserved moments f_hat_1..4 (Eqs. moment1-moment3:
    rho = sum f, rho u = sum f v, rho[(D+I)T + u^2] = sum f (v^2 + eta^2))."""
    rho = fhat[0]
    ux = fhat[1] / rho
    uy = fhat[2] / rho
    T = (fhat[3] / rho - ux * ux - uy * uy) / (D + I)
    return rho, ux, uy, T


# --------------------------------------------------------------------------
# Boundaries and the NND scheme
# --------------------------------------------------------------------------

def ghost(a: torch.Tensor, dim: int, bc: str, w: int = 2) -> torch.Tensor:
    """Pad `a` along `dim` with w ghost cells per side: periodic wrap, or
    zero-gradient outflow (every ghost equals the edge cell)."""
    n = a.shape[dim]
    idx = torch.arange(-w, n + w)
    idx = idx % n if bc == PERIODIC else idx.clamp(0, n - 1)
    return a.index_select(dim, idx)


def mirror_permutation(tab: Tables, axis: str) -> torch.Tensor:
    """Index j(i) of the velocity v_j that is v_i mirrored across a wall normal to `axis`
    (v_x -> -v_x for "x", v_y -> -v_y for "y"; eta is the same within a group)."""
    vx, vy, eta = tab.vx.numpy(), tab.vy.numpy(), tab.eta.numpy()
    perm = []
    for i in range(len(vx)):
        tx, ty = (-vx[i], vy[i]) if axis == "x" else (vx[i], -vy[i])
        j = [k for k in range(len(vx)) if vx[k] == tx and vy[k] == ty and eta[k] == eta[i]]
        assert len(j) == 1
        perm.append(j[0])
    return torch.tensor(perm)


def _edge_layer(a: torch.Tensor, dim: int, side: str, k: int) -> torch.Tensor:
    """Layer k of `a` counted from the edge of `side` (k = 0: the edge cell), kept as a
    slice of width 1 along dim; layers beyond the grid repeat its far edge."""
    n = a.shape[dim]
    k = min(k, n - 1)
    return a.narrow(dim, k if side.endswith("lo") else n - 1 - k, 1)


def wall_layers(f: torch.Tensor, lam: torch.Tensor, P: Params, tab: Tables, side: str, spec):
    """The two ghost layers (nearest the edge first) of f [24, Ny, Nx] and lambda [Ny, Nx]
    beyond one side of the grid.  The wall sits on the face between the edge cell and
    the first ghost.  The paper names these boundaries (Sec. IV C, IV D) without
    formulas; the readings are:
      reflect:   specular wall; ghost layer k holds the distributions of interior layer k
                 with mirrored velocities (f_i <- f_{mirror(i)}), lambda mirrored alike;
      dirichlet: both layers hold the discrete equilibrium M^-1 f_hat^eq of the given
                 (rho, T, u_x, u_y), and the given lambda;
      nee:       non-equilibrium extrapolation: both layers hold the equilibrium at the
                 edge cell's density and the wall's (T, u_x, u_y) plus the edge cell's
                 non-equilibrium part f - f^eq; lambda copies the edge cell."""
    axis = side[0]
    fd, ld = (2, 1) if axis == "x" else (1, 0)
    kind = spec[0]
    if kind == "reflect":
        perm = mirror_permutation(tab, axis)
        fl = [_edge_layer(f, fd, side, k)[perm] for k in (0, 1)]
        ll = [_edge_layer(lam, ld, side, k) for k in (0, 1)]
    elif kind == "dirichlet":
        rho, T, ux, uy, lv = (float(v) for v in spec[1:])
        e = _edge_layer(f, fd, side, 0)
        one = torch.ones_like(e[0])
        feq = torch.einsum("ik,k...->i...", tab.Minv, equilibrium_moments(rho * one, ux * one, uy * one, T * one, P.I))
        fl = [feq, feq]
        ll = [torch.full_like(_edge_layer(lam, ld, side, 0), lv)] * 2
    elif kind == "nee":
        Tw, uxw, uyw = (float(v) for v in spec[1:])
        e = _edge_layer(f, fd, side, 0)
        rho0, ux0, uy0, T0 = macroscopic(moment_transform(e, tab), P.I)
        one = torch.ones_like(rho0)
        feq0 = torch.einsum("ik,k...->i...", tab.Minv, equilibrium_moments(rho0, ux0, uy0, T0, P.I))
        feqw = torch.einsum("ik,k...->i...", tab.Minv, equilibrium_moments(rho0, uxw * one, uyw * one, Tw * one, P.I))
        g = feqw + (e - feq0)
        fl = [g, g]
        ll = [_edge_layer(lam, ld, side, 0)] * 2
    else:
        raise ValueError(f"unknown wall type {kind!r}")
    return fl, ll


def padded(f: torch.Tensor, lam: torch.Tensor, P: Params, tab: Tables, axis: str):
    """f and lambda with two ghost layers per side along `axis` ("x" or "y"): the sides
    listed in P.walls take wall_layers, the others the axis rule of P.bc_x / P.bc_y
    (periodic wrap or zero-gradient outflow)."""
    fd, ld = (2, 1) if axis == "x" else (1, 0)
    bc = P.bc_x if axis == "x" else P.bc_y
    fp, lp = ghost(f, fd, bc), ghost(lam, ld, bc)
    walls = P.walls or {}
    n = f.shape[fd]
    # padded positions: 1 and 0 hold layers 0 and 1 of the low side, n+2 and n+3 those of
    # the high side
    fparts = [fp.narrow(fd, 0, 1), fp.narrow(fd, 1, 1), f, fp.narrow(fd, n + 2, 1), fp.narrow(fd, n + 3, 1)]
    lparts = [lp.narrow(ld, 0, 1), lp.narrow(ld, 1, 1), lam, lp.narrow(ld, n + 2, 1), lp.narrow(ld, n + 3, 1)]
    for side, where in ((axis + "_lo", (1, 0)), (axis + "_hi", (3, 4))):
        if side in walls:
            fl, ll = wall_layers(f, lam, P, tab, side, walls[side])
            for k in (0, 1):
                fparts[where[k]], lparts[where[k]] = fl[k], ll[k]
    return torch.cat(fparts, dim=fd), torch.cat(lparts, dim=ld)


def minmod(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """minmod(a, b): the argument of smaller magnitude when a and b have the same
    strict sign, else zero."""
    zero = torch.zeros_like(a)
    return torch.where((a > 0) & (b > 0), torch.minimum(a, b),
                       torch.where((a < 0) & (b < 0), torch.maximum(a, b), zero))


def nnd_derivative(a: torch.Tensor, dim: int, positive: bool, bc: str, h: float) -> torch.Tensor:
    """NND approximation of d a / d r along `dim` for an advection speed of the
    given sign (Sec. II, NND scheme of Zhang 1988, flux-split minmod form).

    Speed > 0: h_{j+1/2} = a_j + mm(a_j - a_{j-1}, a_{j+1} - a_j)/2
    Speed < 0: h_{j+1/2} = a_{j+1} - mm(a_{j+1} - a_j, a_{j+2} - a_{j+1})/2
    and the derivative is (h_{j+1/2} - h_{j-1/2}) / h.
    """
    return nnd_from_padded(ghost(a, dim, bc), dim, positive, h)


def nnd_from_padded(g: torch.Tensor, dim: int, positive: bool, h: float) -> torch.Tensor:
    """nnd_derivative of an array already padded with two ghost layers per side."""
    n = g.shape[dim] - 4
    s = lambda k: g.narrow(dim, 2 + k, n)       # a_{j+k}
    am2, am1, a0, ap1, ap2 = s(-2), s(-1), s(0), s(1), s(2)
    if positive:
        h_plus = a0 + 0.5 * minmod(a0 - am1, ap1 - a0)
        h_minus = am1 + 0.5 * minmod(am1 - am2, a0 - am1)
    else:
        h_plus = ap1 - 0.5 * minmod(ap1 - a0, ap2 - ap1)
        h_minus = a0 - 0.5 * minmod(a0 - am1, ap1 - a0)
    return (h_plus - h_minus) / h


def streaming(f: torch.Tensor, P: Params, T: Tables, fx=None, fy=None) -> torch.Tensor:
    """v_i_alpha d f_i / d r_alpha with the NND scheme; each f_i is upwinded by
    the sign of its own velocity component.  f has shape [24, Ny, Nx]; fx, fy are f
    padded along x and y (default: the axis rules of P.bc_x, P.bc_y)."""
    fx = ghost(f, 2, P.bc_x) if fx is None else fx
    fy = ghost(f, 1, P.bc_y) if fy is None else fy
    dxp = nnd_from_padded(fx, 2, True, P.dx)
    dxm = nnd_from_padded(fx, 2, False, P.dx)
    dyp = nnd_from_padded(fy, 1, True, P.dy)
    dym = nnd_from_padded(fy, 1, False, P.dy)
    vx, vy = _b(T.vx, f), _b(T.vy, f)
    dfx = torch.where(vx > 0, dxp, dxm)
    dfy = torch.where(vy > 0, dyp, dym)
    return vx * dfx + vy * dfy


# --------------------------------------------------------------------------
# Collision, modification and chemistry
# --------------------------------------------------------------------------

def modification_terms(rho, ux, uy, T, P: Params, tab: Tables, upad=None):
    """A_hat_8 and A_hat_9 (Eqs. ArtificialA8, ArtificialA9) with the velocity
    gradients taken as second-order central differences.  upad (optional): the velocity
    fields padded by one layer per side, {"x": (u_x, u_y) padded along x, "y": ...};
    default: the axis rules of P.bc_x, P.bc_y."""
    I = P.I
    nx, ny = rho.shape[1], rho.shape[0]
    if upad is None:
        upad = {"x": (ghost(ux, 1, P.bc_x, 1), ghost(uy, 1, P.bc_x, 1)),
                "y": (ghost(ux, 0, P.bc_y, 1), ghost(uy, 0, P.bc_y, 1))}
    cdx = lambda a: (a[:, 2:nx + 2] - a[:, 0:nx]) / (2.0 * P.dx)
    cdy = lambda a: (a[2:ny + 2, :] - a[0:ny, :]) / (2.0 * P.dy)
    dux_dx, dux_dy = cdx(upad["x"][0]), cdy(upad["y"][0])
    duy_dx, duy_dy = cdx(upad["x"][1]), cdy(upad["y"][1])
    R5, R7, R8, R9 = tab.R[4], tab.R[6], tab.R[7], tab.R[8]
    A8 = rho * T * (R5 - R8) / R5 * (
        4.0 * ux * (dux_dx - dux_dx / (D + I) - duy_dy / (D + I))
        + 2.0 * uy * (duy_dx + dux_dy))
    A9 = rho * T * (R7 - R9) / R7 * (
        4.0 * uy * (duy_dy - dux_dx / (D + I) - duy_dy / (D + I))
        + 2.0 * ux * (duy_dx + dux_dy))
    return A8, A9


def collision(fhat, feq_hat, A8, A9, tab: Tables):
    """Omega_i = M^-1_il [R_l (f_hat_l - f_hat^eq_l) - A_hat_l] (Eq. Boltzmann_chemical
    with the moment-space sign of A_hat of Eq. CE_LB), Delta_1..4 set to zero."""
    delta = fhat - feq_hat
    delta = torch.cat([torch.zeros_like(delta[:4]), delta[4:]], dim=0)
    g = _b(tab.R, delta) * delta
    g = torch.cat([g[:7], (g[7] - A8).unsqueeze(0), (g[8] - A9).unsqueeze(0), g[9:]], dim=0)
    return torch.einsum("il,l...->i...", tab.Minv, g)


def collision_srt(f, feq, tau: float):
    """Omega_i = (f_i - M^-1_il f_hat^eq_l) / tau (Eq. SRT): one relaxation time for all
    24 distribution functions, towards the discrete equilibrium; no A_hat."""
    return (f - feq) / tau


def cochran_increment(lam, p, T, P: Params, tab: Tables):
    """Reaction increment of lambda over one step (Eq. lambda_equation, Cochran rate,
    temporal part solved analytically with p frozen).

    With a = omega_1 p^m, b = omega_2 p^n and y = 1 - lambda, dy/dt = -y (a + b (1-y))
    has the exact solution y1 = (a+b) y0 / (b y0 + (a+b-b y0) exp((a+b) dt)).
    Returns dlambda = y0 - y1 where T > T_ig, lambda < 1 and a + b > 0, else 0."""
    a = tab.omega1 * p ** P.m
    b = tab.omega2 * p ** P.n
    c = a + b
    active = (T > P.T_ig) & (lam < 1.0) & (c > 0)
    one = torch.ones_like(c)
    c_s = torch.where(active, c, one)           # keeps inactive cells finite
    b_s = torch.where(active, b, one * 0.0)
    y0 = 1.0 - lam
    E = torch.exp(c_s * P.dt)
    y1 = c_s * y0 / (b_s * y0 + (c_s - b_s * y0) * E)
    return torch.where(active, y0 - y1, torch.zeros_like(y0))


def chemical_term(feq, ux, uy, T, F, P: Params, tab: Tables):
    """C_i = f_i^eq Q [-(1+D) I T + I |v_i - u|^2 + eta_i^2] F / (I (D+I) T^2)
    (Eq. C_i), with f^eq the discrete equilibrium M^-1 f_hat^eq."""
    I = P.I
    vx, vy, eta = _b(tab.vx, feq), _b(tab.vy, feq), _b(tab.eta, feq)
    c2 = (vx - ux) ** 2 + (vy - uy) ** 2
    return feq * tab.Q * (-(1.0 + D) * I * T + I * c2 + eta * eta) * F / (I * (D + I) * T * T)


# --------------------------------------------------------------------------
# The time step
# --------------------------------------------------------------------------

def euler_update(f: torch.Tensor, lam: torch.Tensor, P: Params, tab: Tables):
    """One forward-Euler step of Eq. Boltzmann_chemical (or, with P.tau > 0, of Eq. SRT)
    for f and of Eq. lambda_equation for lambda, every term evaluated at level n.

    f^{n+1} = f^n + dt [ -v_i.grad_NND f_i - Omega_i + C_i ]
    lambda^{n+1} = lambda^n + dlambda_chem - dt u.grad_NND lambda
    """
    fhat = moment_transform(f, tab)
    rho, ux, uy, T = macroscopic(fhat, P.I)
    p = rho * T
    feq_hat = equilibrium_moments(rho, ux, uy, T, P.I)
    feq = torch.einsum("ik,k...->i...", tab.Minv, feq_hat)
    fx = fy = lx = ly = upad = None
    if P.walls:
        # ghost layers from the boundary rules; the velocity at a ghost is the velocity
        # moment of its distributions
        fx, lx = padded(f, lam, P, tab, "x")
        fy, ly = padded(f, lam, P, tab, "y")
        nx, ny = f.shape[2], f.shape[1]
        ux_x, uy_x = macroscopic(moment_transform(fx[:, :, 1:nx + 3], tab), P.I)[1:3]
        ux_y, uy_y = macroscopic(moment_transform(fy[:, 1:ny + 3, :], tab), P.I)[1:3]
        upad = {"x": (ux_x, uy_x), "y": (ux_y, uy_y)}
    if P.tau > 0:
        omega = collision_srt(f, feq, P.tau)
    else:
        A8, A9 = modification_terms(rho, ux, uy, T, P, tab, upad)
        omega = collision(fhat, feq_hat, A8, A9, tab)

    dlam = cochran_increment(lam, p, T, P, tab)
    F = dlam / P.dt
    C = chemical_term(feq, ux, uy, T, F, P, tab)

    adv = streaming(f, P, tab, fx, fy)
    f_new = f + P.dt * (-adv - omega + C)

    lx = ghost(lam, 1, P.bc_x) if lx is None else lx
    ly = ghost(lam, 0, P.bc_y) if ly is None else ly
    dlx = torch.where(ux > 0, nnd_from_padded(lx, 1, True, P.dx), nnd_from_padded(lx, 1, False, P.dx))
    dly = torch.where(uy > 0, nnd_from_padded(ly, 0, True, P.dy), nnd_from_padded(ly, 0, False, P.dy))
    lam_new = lam + dlam - P.dt * (ux * dlx + uy * dly)
    return f_new, lam_new


def step(f: torch.Tensor, lam: torch.Tensor, P: Params, tab: Tables):
    """One time step.  P.rk = 1: forward Euler (euler_update).  P.rk = 2, 3: the strong-
    stability-preserving Runge-Kutta schemes of Shu and Osher (1988) written as convex
    combinations of forward-Euler updates E of the whole right-hand side (the reaction
    increment over dt standing for dt times the rate):
        RK2: g1 = E(f);  f' = f/2 + E(g1)/2
        RK3: g1 = E(f);  g2 = 3/4 f + 1/4 E(g1);  f' = 1/3 f + 2/3 E(g2)
    and the same combinations for lambda."""
    if P.rk == 1:
        return euler_update(f, lam, P, tab)
    g1, l1 = euler_update(f, lam, P, tab)
    e1, m1 = euler_update(g1, l1, P, tab)
    if P.rk == 2:
        return 0.5 * f + 0.5 * e1, 0.5 * lam + 0.5 * m1
    g2, l2 = 0.75 * f + 0.25 * e1, 0.75 * lam + 0.25 * m1
    e2, m2 = euler_update(g2, l2, P, tab)
    a, b = 1.0 / 3.0, 2.0 / 3.0
    return a * f + b * e2, a * lam + b * m2


def run(f, lam, P: Params, tab: Tables, nsteps: int):
    for _ in range(nsteps):
        f, lam = step(f, lam, P, tab)
    return f, lam


def init_f(rho, ux, uy, T, P: Params, tab: Tables) -> torch.Tensor:
    """Initial distribution f = M^-1 f_hat^eq(rho, u, T) (Eq. moment12 solved for f^eq)."""
    return torch.einsum("ik,k...->i...", tab.Minv, equilibrium_moments(rho, ux, uy, T, P.I))


# --------------------------------------------------------------------------
# Readouts
# --------------------------------------------------------------------------

def moments(f, lam, P: Params, tab: Tables):
    """rho, u_x, u_y, T, p = rho T, lambda (Sec. II)."""
    rho, ux, uy, T = macroscopic(moment_transform(f, tab), P.I)
    return {"rho": rho, "ux": ux, "uy": uy, "T": T, "p": rho * T, "lam": lam}


def tne(f, P: Params, tab: Tables):
    """Thermodynamic non-equilibrium measures (Sec. VI): Delta_k = f_hat_k - f_hat^eq_k
    for k = 5..24 (shape [20, Ny, Nx]; Delta_1..4 are zero) and the distance
    d = sqrt(sum_k Delta_k^2)."""
    fhat = moment_transform(f, tab)
    rho, ux, uy, T = macroscopic(fhat, P.I)
    delta = (fhat - equilibrium_moments(rho, ux, uy, T, P.I))[4:]
    return delta, torch.sqrt((delta * delta).sum(0))


def ignition_margin(f, lam, P: Params, tab: Tables):
    """min |T - T_ig| over the cells with lambda < 1 (+inf if none): the distance of the
    state from the one discontinuity of the step, the ignition test T > T_ig of the rate
    law (Sec. II)."""
    _, _, _, T = macroscopic(moment_transform(f, tab), P.I)
    live = lam < 1.0
    if not bool(live.any()):
        return float("inf")
    return float((T[live] - P.T_ig).abs().min())


def reductions(f, lam, P: Params, tab: Tables):
    """[sum rho, sum rho u_x, sum rho u_y, sum E_tot, sum_cells sum_k Delta_k^2,
    (dx / Ny) sum |Delta_5|, min lambda, max lambda]; E_tot = f_hat_4 / 2 is the total
    (kinetic + internal) energy density and the sixth entry is the row average of
    the integral of |Delta_{v_x v_x}| over x (the global TNE area of Sec. VI)."""
    fhat = moment_transform(f, tab)
    rho, ux, uy, T = macroscopic(fhat, P.I)
    delta = (fhat - equilibrium_moments(rho, ux, uy, T, P.I))[4:]
    ny = f.shape[1]
    return torch.stack([
        fhat[0].sum(), fhat[1].sum(), fhat[2].sum(), 0.5 * fhat[3].sum(),
        (delta * delta).sum(), delta[0].abs().sum() * P.dx / ny, lam.min(), lam.max()])
