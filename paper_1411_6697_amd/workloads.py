"""Seeded synthetic workloads: parameters and initial macroscopic fields.

This module is shared by the GPU path and by the tests that drive the CPU
reference; it holds none of the kinetic model's arithmetic (no moments, no
equilibria, no collision).  It only states the parameter sets and builds the
initial (rho, u_x, u_y, T, lambda) fields as NumPy float64 arrays of shape
[ny, nx], cell-centred (x_j = (j + 1/2) dx), with sharp interfaces assigned to
the left state when x_j < x_interface.

Parameter sets follow the paper where it gives them (Sec. IV, Sec. VI) and a
fixed project choice where it does not (the Cochran rate constants are never
printed; nominal omega_1 = 2, omega_2 = 100 are used).

Seeds: KH noise 14116697, batched lengths/parameters 14116698, detonation
rate constants 14116699, adjoint noise 14116700 (numpy default_rng).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Callable, Dict, Optional, Tuple

import numpy as np

OUTFLOW = "outflow"
PERIODIC = "periodic"

OMEGA1_NOMINAL = 2.0
OMEGA2_NOMINAL = 100.0

# Velocity models quoted in the paper (v_a, v_b, v_c, eta_a, eta_b, eta_c).
DVM_SOD = (2.5, 2.2, 1.2, 6.5, 3.0, 0.0)            # Sec. IV B 1 (Sod)
DVM_STEADY_DET = (2.7, 2.2, 1.2, 5.0, 3.0, 1.1)     # Sec. IV A (steady detonation)
DVM_UNSTEADY_DET = (2.7, 2.2, 1.2, 1.5, 0.5, 5.0)   # Sec. VI A (unsteady detonation)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    steps: int
    dvm: Tuple[float, ...]
    gamma: float
    I: float
    R: Tuple[float, ...]
    Q: float = 0.0
    omega1: float = 0.0
    omega2: float = 0.0
    m: float = 1.0
    n: float = 1.0
    T_ig: float = 1.1
    bc_x: str = OUTFLOW
    bc_y: str = PERIODIC
    tau: float = 0.0                  # > 0: single-relaxation-time collision (Sec. V)
    rk: int = 1                       # time scheme: 1 forward Euler, 2/3 SSP Runge-Kutta
    walls: Optional[dict] = None      # per-side wall boundaries overriding bc_x / bc_y
    make_fields: Optional[Callable[["Workload"], Dict[str, np.ndarray]]] = field(default=None, repr=False)
    meta: dict = field(default_factory=dict)

    def fields(self) -> Dict[str, np.ndarray]:
        return self.make_fields(self)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def rates(base: float = 1e5, **override) -> Tuple[float, ...]:
    """R_1..R_24 = base except the 1-based indices given as r5=..., r8=..."""
    r = [base] * 24
    for k, v in override.items():
        r[int(k[1:]) - 1] = v
    return tuple(r)


def cj_state(rho0: float, p0: float, Q: float, g: float) -> dict:
    """Chapman-Jouguet state for a quiescent ideal gas with heat release Q
    (closed form: M_CJ = sqrt(1+H) + sqrt(H), H = (g^2-1) Q / (2 c0^2))."""
    c0 = math.sqrt(g * p0 / rho0)
    H = (g * g - 1.0) * Q / (2.0 * c0 * c0)
    M = math.sqrt(1.0 + H) + math.sqrt(H)
    D = M * c0
    p1 = p0 * (1.0 + g * M * M) / (g + 1.0)
    rho1 = rho0 * (g + 1.0) * M * M / (1.0 + g * M * M)
    return {"D": D, "rho": rho1, "p": p1, "T": p1 / rho1, "u": D * (1.0 - rho0 / rho1)}


def _blank(w: Workload):
    shape = (w.ny, w.nx)
    return {k: np.zeros(shape) for k in ("rho", "ux", "uy", "T", "lam")}


def _xc(w: Workload) -> np.ndarray:
    return (np.arange(w.nx) + 0.5) * w.dx


def _yc(w: Workload) -> np.ndarray:
    return (np.arange(w.ny) + 0.5) * w.dy


# --------------------------------------------------------------------------
# Riemann problems
# --------------------------------------------------------------------------

def _riemann_fields(left, right, x_interface):
    def make(w: Workload):
        f = _blank(w)
        L = _xc(w)[None, :] < x_interface(w)
        for k, (a, b) in zip(("rho", "ux", "uy", "T"), zip(left, right)):
            f[k][...] = np.where(L, a, b)
        return f
    return make


def sod(nx: int = 400, ny: int = 1, steps: int = 2000, paper_rates: bool = False) -> Workload:
    """Sod shock tube (Sec. IV B 1): (rho, T, u_x, u_y) = (1, 1, 0, 0) | (0.125, 0.8, 0, 0),
    dx = dy = 1e-3, dt = 1e-5, I = 3, DVM (2.5, 2.2, 1.2, 6.5, 3, 0).  The default rate set
    is the Pr = 1 one (R_5..R_9 = 1.2e4, the rest 1e5); paper_rates=True takes the paper's
    literal set (R_5..R_7 = 1.2e4, all others 1e5, so A_hat is active)."""
    if paper_rates:
        R = rates(1e5, r5=1.2e4, r6=1.2e4, r7=1.2e4)
    else:
        R = rates(1e5, r5=1.2e4, r6=1.2e4, r7=1.2e4, r8=1.2e4, r9=1.2e4)
    return Workload(
        name="sod" + ("_paper_rates" if paper_rates else ""), nx=nx, ny=ny, dx=1e-3, dy=1e-3,
        dt=1e-5, steps=steps, dvm=DVM_SOD, gamma=1.4, I=3.0, R=R,
        bc_x=OUTFLOW, bc_y=PERIODIC,
        make_fields=_riemann_fields((1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.8),
                                    lambda w: 0.5 * w.nx * w.dx))


# Velocity models of the Lax and Sjogren runs (Sec. IV B 2 and 3).
DVM_LAX = (4.7, 3.3, 1.0, 6.0, 2.5, 0.9)
DVM_SJOGREN = (0.4, 1.0, 1.8, 0.3, 1.9, 1.5)


def lax(nx: int = 2000, ny: int = 1, steps: int = 15000) -> Workload:
    """Lax shock tube (Sec. IV B 2): (rho, T, u_x, u_y) = (0.445, 7.928, 0.698, 0) on [-1, 0)
    and (0.5, 1.142, 0, 0) on [0, 1]; dx = dy = 1e-3, dt = 1e-5, I = 1 (gamma = 5/3),
    DVM (4.7, 3.3, 1, 6, 2.5, 0.9), R_5..R_7 = 2e4, R_8 = R_9 = 8e4 (Pr = 4, A_hat active),
    other R_k = 1e5; t = 0.15 after 15000 steps.  The domain is cell-centred on
    [0, nx dx] with the interface at its middle."""
    R = rates(1e5, r5=2e4, r6=2e4, r7=2e4, r8=8e4, r9=8e4)
    return Workload(
        name="lax", nx=nx, ny=ny, dx=1e-3, dy=1e-3, dt=1e-5, steps=steps, dvm=DVM_LAX,
        gamma=5.0 / 3.0, I=1.0, R=R, bc_x=OUTFLOW, bc_y=PERIODIC,
        make_fields=_riemann_fields((0.445, 0.698, 0.0, 7.928), (0.5, 0.0, 0.0, 1.142),
                                    lambda w: 0.5 * w.nx * w.dx))


def sjogren(nx: int = 500, ny: int = 1, steps: int = 1500) -> Workload:
    """Sjogren's problem (Sec. IV B 3), two receding streams: (rho, T, u_x, u_y) =
    (1, 0.5, -1.2, 0) on [-0.5, 0) and (1, 0.5, 1.2, 0) on [0, 0.5]; dx = dy = 2e-3,
    dt = 2e-5, I = 4 (gamma = 4/3), DVM (0.4, 1.0, 1.8, 0.3, 1.9, 1.5), R_8 = R_9 = 2e4,
    other R_k = 5e4 (Pr = 0.4, A_hat active); t = 0.03 after 1500 steps."""
    R = rates(5e4, r8=2e4, r9=2e4)
    return Workload(
        name="sjogren", nx=nx, ny=ny, dx=2e-3, dy=2e-3, dt=2e-5, steps=steps, dvm=DVM_SJOGREN,
        gamma=4.0 / 3.0, I=4.0, R=R, bc_x=OUTFLOW, bc_y=PERIODIC,
        make_fields=_riemann_fields((1.0, -1.2, 0.0, 0.5), (1.0, 1.2, 0.0, 0.5),
                                    lambda w: 0.5 * w.nx * w.dx))


DVM_SHOCK_REFLECTION = (1.0, 2.7, 2.9, 1.0, 2.9, 0.96)    # Sec. IV C


def shock_reflection(nx: int = 300, ny: int = 100, steps: int = 100000) -> Workload:
    """Regular shock reflection (Sec. IV C): a 0.3 x 0.1 channel, dx = dy = 1e-3,
    dt = 5e-6, I = 2 (gamma = 3/2), DVM (1.0, 2.7, 2.9, 1.0, 2.9, 0.96), R_5..R_7 = 1.8e5,
    R_8 = R_9 = 2e5, other R_k = 1e5; reflecting wall at the bottom, supersonic outflow at
    the right, Dirichlet inflow (rho, T, u_x, u_y) = (1, 0.5, 2, 0) at the left and the
    post-shock state (1.25, 0.56, 1.9, -0.173205) at the top; t = 0.5 after 100000 steps.
    The initial field (not given) is the inflow state everywhere."""
    R = rates(1e5, r5=1.8e5, r6=1.8e5, r7=1.8e5, r8=2e5, r9=2e5)

    def make(w: Workload):
        f = _blank(w)
        f["rho"][...] = 1.0
        f["T"][...] = 0.5
        f["ux"][...] = 2.0
        return f
    return Workload(
        name="shock_reflection", nx=nx, ny=ny, dx=1e-3, dy=1e-3, dt=5e-6, steps=steps,
        dvm=DVM_SHOCK_REFLECTION, gamma=1.5, I=2.0, R=R, bc_x=OUTFLOW, bc_y=OUTFLOW,
        walls={"x_lo": ("dirichlet", 1.0, 0.5, 2.0, 0.0, 0.0), "y_lo": ("reflect",),
               "y_hi": ("dirichlet", 1.25, 0.56, 1.9, -0.173205, 0.0)},
        make_fields=make)


# --------------------------------------------------------------------------
# Detonation
# --------------------------------------------------------------------------

def _detonation_fields(n_driver: int, noise_seed: Optional[int] = None, noise: float = 0.0):
    def make(w: Workload):
        cj = cj_state(1.0, 1.0, w.Q, w.gamma)
        f = _blank(w)
        drv = np.arange(w.nx)[None, :] < n_driver
        f["rho"][...] = np.where(drv, cj["rho"], 1.0)
        f["T"][...] = np.where(drv, cj["T"], 1.0)
        f["ux"][...] = np.where(drv, cj["u"], 0.0)
        f["lam"][...] = np.where(drv, 1.0, 0.0)
        if noise_seed is not None:
            f["uy"][...] = np.random.default_rng(noise_seed).normal(0.0, noise, size=(w.ny, w.nx))
        return f
    return make


def detonation(nx: int = 8000, ny: int = 4, steps: int = 20000, seed: int = 14116699) -> Workload:
    """1D unsteady detonation with one-step Cochran chemistry, the grid and rates of
    Sec. VI A case (iii): dx = dy = 1e-4, dt = 1e-6, R_i = 100, I = 3, Q = 1,
    DVM (2.7, 2.2, 1.2, 1.5, 0.5, 5.0).  Unburnt (rho, u, p, lambda) = (1, 0, 1, 0);
    the first 200 cells hold the CJ state (lambda = 1).  omega_1, omega_2 are the
    nominal values scaled by one U[0.9, 1.1] draw each."""
    rng = np.random.default_rng(seed)
    s1, s2 = rng.uniform(0.9, 1.1, size=2)
    return Workload(
        name="detonation", nx=nx, ny=ny, dx=1e-4, dy=1e-4, dt=1e-6, steps=steps,
        dvm=DVM_UNSTEADY_DET, gamma=1.4, I=3.0, R=rates(100.0), Q=1.0,
        omega1=OMEGA1_NOMINAL * s1, omega2=OMEGA2_NOMINAL * s2,
        bc_x=OUTFLOW, bc_y=PERIODIC, make_fields=_detonation_fields(200))


def steady_detonation(nx: int = 1000, dx: float = 5e-4, dt: float = 1e-5, steps: int = 10000) -> Workload:
    """Steady detonation of Sec. IV A (paper: 0 <= x <= 1, dx = 2e-4, dt = 5e-6, t = 0.39):
    DVM (2.7, 2.2, 1.2, 5, 3, 1.1), I = 3, Q = 1, R_5..R_7 = 1e4, the rest 1e5; CJ state
    on x <= 0.2, (1, 1, 0, 0, 0) to the right."""
    def make(w: Workload):
        cj = cj_state(1.0, 1.0, w.Q, w.gamma)
        f = _blank(w)
        L = _xc(w)[None, :] <= 0.2
        f["rho"][...] = np.where(L, cj["rho"], 1.0)
        f["T"][...] = np.where(L, cj["T"], 1.0)
        f["ux"][...] = np.where(L, cj["u"], 0.0)
        f["lam"][...] = np.where(L, 1.0, 0.0)
        return f
    return Workload(
        name="steady_detonation", nx=nx, ny=1, dx=dx, dy=dx, dt=dt, steps=steps,
        dvm=DVM_STEADY_DET, gamma=1.4, I=3.0, R=rates(1e5, r5=1e4, r6=1e4, r7=1e4), Q=1.0,
        omega1=OMEGA1_NOMINAL, omega2=OMEGA2_NOMINAL, bc_x=OUTFLOW, bc_y=PERIODIC,
        make_fields=make)


# --------------------------------------------------------------------------
# Kelvin-Helmholtz double shear layer
# --------------------------------------------------------------------------

def kh(n: int = 2048, steps: int = 1000, reactive: bool = True, seed: int = 14116697) -> Workload:
    """Doubly periodic Kelvin-Helmholtz shear layers on [0,1]^2, dx = dy = 1/n,
    dt = 0.2 dx / max|v| (CFL 0.2), rho = 1, T = p = 2.5, lambda = 0,
    u_x = -1/2 + [tanh((y - 1/4)/0.02) - tanh((y - 3/4)/0.02)]/2, u_y ~ N(0, 1e-3^2) per
    cell.  DVM of Sec. VI A, R_k = 2e4 (R_k dt = 0.72; with R_k = 1e4 the reactive run
    loses positivity after ~700 steps and the inert one after ~2800: the white-noise seed
    feeds the high-wavenumber growth of the D2V24 model).  Reactive: Q = 1 with nominal
    Cochran constants; non-reactive: Q = 0, omega = 0."""
    dvm = DVM_UNSTEADY_DET
    dx = 1.0 / n
    dt = 0.2 * dx / max(dvm[:3])

    def make(w: Workload):
        f = _blank(w)
        y = _yc(w)[:, None]
        f["rho"][...] = 1.0
        f["T"][...] = 2.5
        f["ux"][...] = -0.5 + 0.5 * (np.tanh((y - 0.25) / 0.02) - np.tanh((y - 0.75) / 0.02))
        f["uy"][...] = np.random.default_rng(seed).normal(0.0, 1e-3, size=(w.ny, w.nx))
        return f
    return Workload(
        name="kh" + ("_reactive" if reactive else "_inert"), nx=n, ny=n, dx=dx, dy=dx, dt=dt,
        steps=steps, dvm=dvm, gamma=1.4, I=3.0, R=rates(2e4),
        Q=1.0 if reactive else 0.0,
        omega1=OMEGA1_NOMINAL if reactive else 0.0, omega2=OMEGA2_NOMINAL if reactive else 0.0,
        bc_x=PERIODIC, bc_y=PERIODIC, make_fields=make)


# --------------------------------------------------------------------------
# Adjoint strip and batched instances
# --------------------------------------------------------------------------

def adjoint_strip(nx: int = 2048, ny: int = 256, steps: int = 500, seed: int = 14116700) -> Workload:
    """2D detonation strip for the gradient runs: dx = dy = 1e-4, dt = 1e-6, x outflow,
    y periodic, first 200 columns at the CJ state, u_y noise sigma = 1e-3,
    R_5..R_7 = 100, R_8 = R_9 = 200 (Pr = 2, A_hat active), other R = 100, Q = 1."""
    return Workload(
        name="adjoint_strip", nx=nx, ny=ny, dx=1e-4, dy=1e-4, dt=1e-6, steps=steps,
        dvm=DVM_UNSTEADY_DET, gamma=1.4, I=3.0, R=rates(100.0, r8=200.0, r9=200.0), Q=1.0,
        omega1=OMEGA1_NOMINAL, omega2=OMEGA2_NOMINAL, bc_x=OUTFLOW, bc_y=PERIODIC,
        make_fields=_detonation_fields(min(200, nx // 4), noise_seed=seed, noise=1e-3))


@dataclass
class BatchSpec:
    """Ragged batch of 1D detonations sharing the grid spacing and velocity model."""
    nx: np.ndarray          # [n] cells per instance
    R: np.ndarray           # [n, 24] rates per instance
    Pr: np.ndarray          # [n] Prandtl number per instance (R_8 = R_9 = Pr R_5)
    base: Workload          # common grid/physics; nx of the base is unused

    def instance(self, k: int) -> Workload:
        return self.base.with_(name=f"batch[{k}]", nx=int(self.nx[k]), R=tuple(self.R[k]))


def batched(n_inst: int = 128, nx_lo: int = 1000, nx_hi: int = 8000, steps: int = 5000,
            seed: int = 14116698) -> BatchSpec:
    """Batch of independent 1D detonations (Ny = 1) of lengths U{nx_lo..nx_hi};
    per instance R_5..R_7 = 100 s1 and Pr = s2 with s1, s2 ~ logU[0.5, 5];
    R_8 = R_9 = Pr R_5; other R_k = 100.  dx = 1e-4, dt = 1e-6, Q = 1, gamma = 1.4,
    DVM of Sec. VI A, 200-cell CJ driver, outflow at both ends."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(nx_lo, nx_hi + 1, size=n_inst)
    s = np.exp(rng.uniform(math.log(0.5), math.log(5.0), size=(n_inst, 2)))
    R = np.full((n_inst, 24), 100.0)
    R[:, 4:7] = 100.0 * s[:, :1]
    R[:, 7:9] = s[:, 1:2] * R[:, 4:5]
    base = detonation(nx=int(nx_hi), ny=1, steps=steps).with_(
        name="batched", omega1=OMEGA1_NOMINAL, omega2=OMEGA2_NOMINAL)
    return BatchSpec(nx=nx, R=R, Pr=s[:, 1].copy(), base=base)
