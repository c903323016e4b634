"""Thin ctypes binding of liblbkm (C ABI in include/lbkm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of the
library.  PyTorch supplies device memory (caller-owned state buffers) and the stream.
The binding refuses to run if the library is missing; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# LBKM_LIBRARY may point at another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("LBKM_LIBRARY", os.path.join(HERE, "liblbkm.so"))

LBKM_BC_PERIODIC = 0
LBKM_BC_OUTFLOW = 1
BC = {"periodic": LBKM_BC_PERIODIC, "outflow": LBKM_BC_OUTFLOW}

STATUS = {0: "LBKM_OK", -1: "LBKM_EINVAL", -2: "LBKM_ESINGULAR", -3: "LBKM_ENOMEM",
          -4: "LBKM_EDEVICE", -5: "LBKM_ESTATE", -6: "LBKM_ENONFINITE"}


class LbkmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Dvm(ctypes.Structure):
    _fields_ = [("va", ctypes.c_double), ("vb", ctypes.c_double), ("vc", ctypes.c_double),
                ("eta_a", ctypes.c_double), ("eta_b", ctypes.c_double), ("eta_c", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dt", ctypes.c_double), ("bc_x", ctypes.c_int32),
                ("bc_y", ctypes.c_int32), ("dvm", Dvm)]


class Rates(ctypes.Structure):
    _fields_ = [("omega1", ctypes.c_double), ("omega2", ctypes.c_double), ("m", ctypes.c_double),
                ("n", ctypes.c_double), ("T_ig", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "lbkm_create": [ctypes.POINTER(Grid), _P, ctypes.POINTER(_P)],
    "lbkm_bind_buffers": [_P, _P, _P, _P, _P, ctypes.c_int64],
    "lbkm_set_params": [_P, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Rates)],
    "lbkm_init_fields": [_P, _P, _P, _P, _P, _P],
    "lbkm_step": [_P, ctypes.c_int64],
    "lbkm_get_moments": [_P, _P, _P, _P, _P, _P, _P],
    "lbkm_get_tne": [_P, _P, _P],
    "lbkm_reduce": [_P, _D],
    "lbkm_check": [_P],
    "lbkm_ignition_margin": [_P, _D],
    "lbkm_get_state": [_P, _P, _P],
    "lbkm_set_state": [_P, _P, _P],
    "lbkm_get_step_count": [_P, ctypes.POINTER(ctypes.c_int64)],
    "lbkm_get_matrices": [_P, _D, _D, _D],
    "lbkm_set_tile": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "lbkm_set_tile_order": [_P, ctypes.c_int32],
    "lbkm_set_srt": [_P, ctypes.c_double],
    "lbkm_set_time_scheme": [_P, ctypes.c_int32],
    "lbkm_set_boundary": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "lbkm_autotune": [_P, ctypes.POINTER(ctypes.c_int32)],
    "lbkm_adjoint_step": [_P, _P, _P, _P, _P, _P, _P, _P],
    "lbkm_adjoint_init": [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "lbkm_tne_loss": [_P, _P, _P, _P],
    "lbkm_tne_loss_noalloc": [_P, _P, _P, _P],
    "lbkm_destroy": [_P],
    "lbkm_copy_kernel": [_P, _P, ctypes.c_int64, _P],
    "lbkm_batch_create": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Grid), _P,
                          ctypes.POINTER(_P)],
    "lbkm_batch_set_params": [_P, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Rates)],
    "lbkm_batch_init_fields": [_P, _P, _P, _P, _P, _P],
    "lbkm_batch_autotune": [_P, ctypes.POINTER(ctypes.c_int32)],
    "lbkm_batch_step": [_P, ctypes.c_int64],
    "lbkm_batch_get_moments": [_P, _P, _P, _P, _P, _P, _P],
    "lbkm_batch_total_cells": [_P, ctypes.POINTER(ctypes.c_int64)],
    "lbkm_batch_status": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "lbkm_batch_set_launch": [_P, ctypes.c_int32],
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblbkm.so (built by paper_1411_6697_amd.build).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1411_6697_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lbkm_last_error.argtypes = [_P]
    lib.lbkm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dev(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def pad_pitch(nx: int, align: int = 64) -> int:
    return (nx + align - 1) // align * align


class Sim:
    """One grid.  State buffers are torch tensors owned by this object."""

    def __init__(self, nx: int, ny: int, dx: float, dy: float, dt: float, dvm: Sequence[float],
                 bc_x: str = "outflow", bc_y: str = "periodic", device="cuda:0",
                 pitch: Optional[int] = None):
        self.lib = load()
        self.device = torch.device(device)
        self.nx, self.ny = int(nx), int(ny)
        g = Grid(nx=self.nx, ny=self.ny, dx=dx, dy=dy, dt=dt, bc_x=BC[bc_x], bc_y=BC[bc_y],
                 dvm=Dvm(*[float(v) for v in dvm]))
        self._grid = g
        h = ctypes.c_void_p()
        st = self.lib.lbkm_create(ctypes.byref(g), _stream_handle(self.device), ctypes.byref(h))
        self.h = h
        if st != 0:
            msg = self.lib.lbkm_last_error(h).decode() if h.value else "lbkm_create failed"
            if h.value:
                self.lib.lbkm_destroy(h)
                self.h = ctypes.c_void_p()
            raise LbkmError(st, msg)
        self.pitch = int(pitch) if pitch is not None else pad_pitch(self.nx)
        kw = dict(dtype=torch.float64, device=self.device)
        self.f = [torch.zeros(24, self.ny, self.pitch, **kw), torch.zeros(24, self.ny, self.pitch, **kw)]
        self.lam = [torch.zeros(self.ny, self.pitch, **kw), torch.zeros(self.ny, self.pitch, **kw)]
        self._call("lbkm_bind_buffers", _ptr(self.f[0]), _ptr(self.f[1]), _ptr(self.lam[0]),
                   _ptr(self.lam[1]), ctypes.c_int64(self.pitch))

    # -- plumbing
    def _call(self, name, *args):
        st = getattr(self.lib, name)(self.h, *args)
        if st != 0:
            raise LbkmError(st, self.lib.lbkm_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lbkm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API
    def set_params(self, S: Sequence[float], gamma: float, Pr: float = 0.0, Q: float = 0.0,
                   omega1: float = 0.0, omega2: float = 0.0, m: float = 1.0, n: float = 1.0,
                   T_ig: float = 1.1):
        arr = (ctypes.c_double * 24)(*[float(v) for v in S])
        r = Rates(omega1=omega1, omega2=omega2, m=m, n=n, T_ig=T_ig)
        self._call("lbkm_set_params", arr, ctypes.c_double(gamma), ctypes.c_double(Pr),
                   ctypes.c_double(Q), ctypes.byref(r))

    def init_fields(self, rho, ux, uy, T, lam):
        t = [_dev(a, self.device).reshape(self.ny, self.nx).contiguous() for a in (rho, ux, uy, T, lam)]
        self._call("lbkm_init_fields", *[_ptr(a) for a in t])
        self._keep = t          # keep inputs alive until the stream has consumed them

    def step(self, n: int = 1):
        self._call("lbkm_step", ctypes.c_int64(int(n)))

    def moments(self) -> Dict[str, torch.Tensor]:
        out = {k: torch.empty(self.ny, self.nx, dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "T", "p", "lam")}
        self._call("lbkm_get_moments", *[_ptr(out[k]) for k in ("rho", "ux", "uy", "T", "p", "lam")])
        return out

    def tne(self):
        delta = torch.empty(20, self.ny, self.nx, dtype=torch.float64, device=self.device)
        d = torch.empty(self.ny, self.nx, dtype=torch.float64, device=self.device)
        self._call("lbkm_get_tne", _ptr(delta), _ptr(d))
        return delta, d

    def reduce(self) -> np.ndarray:
        out = (ctypes.c_double * 8)()
        self._call("lbkm_reduce", out)
        return np.array(out[:], dtype=np.float64)

    def ignition_margin(self) -> float:
        """min |T - T_ig| over the cells with lambda < 1 (inf when there is none)."""
        out = ctypes.c_double()
        self._call("lbkm_ignition_margin", ctypes.byref(out))
        return float(out.value)

    def check(self) -> bool:
        st = self.lib.lbkm_check(self.h)
        if st == -6:
            return False
        if st != 0:
            raise LbkmError(st, self.lib.lbkm_last_error(self.h).decode())
        return True

    def get_state(self):
        f = torch.empty(24, self.ny, self.nx, dtype=torch.float64, device=self.device)
        lam = torch.empty(self.ny, self.nx, dtype=torch.float64, device=self.device)
        self._call("lbkm_get_state", _ptr(f), _ptr(lam))
        return f, lam

    def set_state(self, f, lam):
        f = _dev(f, self.device).reshape(24, self.ny, self.nx).contiguous()
        lam = _dev(lam, self.device).reshape(self.ny, self.nx).contiguous()
        self._call("lbkm_set_state", _ptr(f), _ptr(lam))
        self._keep = (f, lam)

    def set_tile(self, tile_x: int, tile_y: int, lds: int = 1):
        self._call("lbkm_set_tile", ctypes.c_int32(tile_x), ctypes.c_int32(tile_y), ctypes.c_int32(lds))

    def set_tile_order(self, vertical: int):
        self._call("lbkm_set_tile_order", ctypes.c_int32(int(vertical)))

    WALL_SIDES = {"x_lo": 0, "x_hi": 1, "y_lo": 2, "y_hi": 3}
    WALL_TYPES = {"none": 0, "reflect": 1, "dirichlet": 2, "nee": 3}

    def set_boundary(self, side: str, spec):
        """Wall side: spec = ("reflect",), ("dirichlet", rho, T, u_x, u_y, lambda),
        ("nee", T, u_x, u_y) or ("none",)."""
        kind = spec[0]
        vals = [0.0] * 5
        if kind == "dirichlet":
            vals = [float(v) for v in spec[1:6]]
        elif kind == "nee":
            vals = [0.0, float(spec[1]), float(spec[2]), float(spec[3]), 0.0]
        arr = (ctypes.c_double * 5)(*vals)
        self._call("lbkm_set_boundary", ctypes.c_int32(self.WALL_SIDES[side]),
                   ctypes.c_int32(self.WALL_TYPES[kind]), arr)

    def set_time_scheme(self, order: int):
        """1: forward Euler (default); 2, 3: SSP Runge-Kutta of that order."""
        self._call("lbkm_set_time_scheme", ctypes.c_int32(int(order)))

    def set_srt(self, tau: float):
        """tau > 0: single-relaxation-time collision (Eq. SRT); tau = 0: MRT (the default)."""
        self._call("lbkm_set_srt", ctypes.c_double(float(tau)))

    def autotune(self):
        """Pick the fastest launch shape on this device; returns (tile_x, tile_y, lds, vertical)."""
        out = (ctypes.c_int32 * 4)()
        self._call("lbkm_autotune", out)
        return tuple(out[:])

    def step_count(self) -> int:
        v = ctypes.c_int64()
        self._call("lbkm_get_step_count", ctypes.byref(v))
        return v.value

    # -- adjoint (dense [24][ny][nx] / [ny][nx] device tensors)
    def set_theta(self, theta, gamma: float, m: float = 1.0, n: float = 1.0, T_ig: float = 1.1):
        """Parameters from theta = (R_1..R_24, Q, omega_1, omega_2), with R_8, R_9 taken as
        given (the parameter vector of the gradient entry points)."""
        th = [float(v) for v in (theta.detach().cpu().tolist() if isinstance(theta, torch.Tensor) else theta)]
        if len(th) != NUM_GRAD:
            raise ValueError(f"theta needs {NUM_GRAD} entries")
        self.set_params(th[:24], gamma, 0.0, th[24], th[25], th[26], m, n, T_ig)

    def adjoint_step(self, f_n, lam_n, af_np1, alam_np1, grad: torch.Tensor):
        """Adjoint of one step: returns (af_n, alam_n) and adds the parameter gradient of
        this step to grad (27 doubles on the device)."""
        af_n = torch.empty_like(af_np1)
        alam_n = torch.empty_like(alam_np1)
        self._call("lbkm_adjoint_step", _ptr(f_n), _ptr(lam_n), _ptr(af_np1), _ptr(alam_np1),
                   _ptr(af_n), _ptr(alam_n), _ptr(grad))
        return af_n, alam_n

    def adjoint_init(self, rho, ux, uy, T, af):
        t = [_dev(a, self.device).reshape(self.ny, self.nx).contiguous() for a in (rho, ux, uy, T)]
        out = [torch.empty(self.ny, self.nx, dtype=torch.float64, device=self.device) for _ in range(4)]
        self._call("lbkm_adjoint_init", *[_ptr(a) for a in t], _ptr(af), *[_ptr(o) for o in out])
        self._keep = t
        return tuple(out)

    def tne_loss(self, f, grad: bool = True):
        """L = sum_cells sum_{k=5..24} Delta_k^2 of a dense state, and dL/df if grad."""
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(f) if grad else None
        self._call("lbkm_tne_loss", _ptr(f), _ptr(loss), _ptr(g))
        return loss[0], g

    def tne_loss_into(self, f, loss, grad=None):
        """The same loss into caller buffers through lbkm_tne_loss_noalloc (no device
        allocation by the library or by this call): loss is a 1-element float64 device
        tensor, grad None or a tensor shaped like f."""
        self._call("lbkm_tne_loss_noalloc", _ptr(f), _ptr(loss), _ptr(grad))


NUM_GRAD = 27   # R_1..R_24, Q, omega_1, omega_2


class LBKMRun(torch.autograd.Function):
    """(f^N, lambda^N) after `steps` steps from the initial fields, differentiable with
    respect to theta = (R_1..R_24, Q, omega_1, omega_2) and the initial rho, u_x, u_y, T,
    lambda.  The forward pass keeps a checkpoint every `every` steps; the backward pass
    re-runs each segment from its checkpoint, keeps the segment's states, and applies the
    library's adjoint step to them in reverse order.  The Sim must not be used by anything
    else between the forward and the backward pass."""

    @staticmethod
    def forward(ctx, theta, rho, ux, uy, T, lam, sim: "Sim", steps: int, gamma: float,
                every: int = 50, m: float = 1.0, n: float = 1.0, T_ig: float = 1.1):
        sim.set_theta(theta, gamma, m, n, T_ig)
        sim.init_fields(rho, ux, uy, T, lam)
        ckpts, done = [], 0
        while done < steps:
            ckpts.append(sim.get_state())
            k = min(every, steps - done)
            sim.step(k)
            done += k
        fN, lN = sim.get_state()
        ctx.sim, ctx.ckpts, ctx.steps, ctx.every = sim, ckpts, steps, every
        ctx.fields = tuple(_dev(a, sim.device).reshape(sim.ny, sim.nx) for a in (rho, ux, uy, T))
        ctx.theta_meta = (theta.dtype, theta.device)
        return fN, lN

    @staticmethod
    def backward(ctx, gf, gl):
        sim = ctx.sim
        kw = dict(dtype=torch.float64, device=sim.device)
        af = gf.contiguous() if gf is not None else torch.zeros(24, sim.ny, sim.nx, **kw)
        al = gl.contiguous() if gl is not None else torch.zeros(sim.ny, sim.nx, **kw)
        grad = torch.zeros(NUM_GRAD, **kw)
        for seg in reversed(range(len(ctx.ckpts))):
            f0, l0 = ctx.ckpts[seg]
            k = min(ctx.every, ctx.steps - seg * ctx.every)
            sim.set_state(f0, l0)
            stash = [(f0, l0)]
            for _ in range(k - 1):
                sim.step(1)
                stash.append(sim.get_state())
            for s in reversed(range(k)):
                af, al = sim.adjoint_step(stash[s][0], stash[s][1], af, al, grad)
            del stash
        arho, aux, auy, aT = sim.adjoint_init(*ctx.fields, af)
        dt, dev = ctx.theta_meta
        return (grad.to(dtype=dt, device=dev), arho, aux, auy, aT, al) + (None,) * 7


class TNELoss(torch.autograd.Function):
    """L = sum_cells sum_{k=5..24} Delta_k^2 of a dense state f (Sec. VI)."""

    @staticmethod
    def forward(ctx, f, sim: "Sim"):
        loss, g = sim.tne_loss(f.contiguous(), grad=True)
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return g * gout, None


class Batch:
    """Ragged batch of 1D instances advanced together (library-owned packed state)."""

    def __init__(self, nx: Sequence[int], dx: float, dt: float, dvm: Sequence[float], device="cuda:0"):
        self.lib = load()
        self.device = torch.device(device)
        self.nx = [int(v) for v in nx]
        self.offsets = np.concatenate([[0], np.cumsum(self.nx)]).astype(np.int64)
        g = Grid(nx=1, ny=1, dx=dx, dy=dx, dt=dt, bc_x=LBKM_BC_OUTFLOW, bc_y=LBKM_BC_PERIODIC,
                 dvm=Dvm(*[float(v) for v in dvm]))
        arr = (ctypes.c_int32 * len(self.nx))(*self.nx)
        h = ctypes.c_void_p()
        st = self.lib.lbkm_batch_create(ctypes.c_int32(len(self.nx)), arr, ctypes.byref(g),
                                        _stream_handle(self.device), ctypes.byref(h))
        self.h = h
        if st != 0:
            msg = self.lib.lbkm_last_error(h).decode() if h.value else "lbkm_batch_create failed"
            self.close()
            raise LbkmError(st, msg)
        self.total = int(self.offsets[-1])

    _call = Sim._call
    close = Sim.close
    __del__ = Sim.__del__

    def set_params(self, R, gamma: float, Pr=None, Q: float = 0.0, omega1: float = 0.0,
                   omega2: float = 0.0, m: float = 1.0, n: float = 1.0, T_ig: float = 1.1):
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(len(self.nx), 24)
        S = R.ctypes.data_as(_D)
        P = None
        if Pr is not None:
            Pr = np.ascontiguousarray(Pr, dtype=np.float64).reshape(len(self.nx))
            P = Pr.ctypes.data_as(_D)
        r = Rates(omega1=omega1, omega2=omega2, m=m, n=n, T_ig=T_ig)
        self._call("lbkm_batch_set_params", S, P, ctypes.c_double(gamma), ctypes.c_double(Q),
                   ctypes.byref(r))

    def init_fields(self, rho, ux, uy, T, lam):
        t = [_dev(a, self.device).reshape(self.total).contiguous() for a in (rho, ux, uy, T, lam)]
        self._call("lbkm_batch_init_fields", *[_ptr(a) for a in t])
        self._keep = t

    def autotune(self) -> int:
        v = ctypes.c_int32()
        self._call("lbkm_batch_autotune", ctypes.byref(v))
        return v.value

    def set_launch(self, wgs_per_cu: int):
        """0: one launch per step; 1..16: the persistent kernel at that many work-groups per CU."""
        self._call("lbkm_batch_set_launch", ctypes.c_int32(int(wgs_per_cu)))

    def step(self, n: int = 1):
        self._call("lbkm_batch_step", ctypes.c_int64(int(n)))

    def status(self):
        """(work-groups per launch, work-groups per CU or 0 with one launch per step); raises
        if a neighbour wait ran out."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        self._call("lbkm_batch_status", ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def moments(self) -> Dict[str, torch.Tensor]:
        out = {k: torch.empty(self.total, dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "T", "p", "lam")}
        self._call("lbkm_batch_get_moments", *[_ptr(out[k]) for k in ("rho", "ux", "uy", "T", "p", "lam")])
        return out

    def split(self, packed: torch.Tensor):
        """Per-instance views of a packed field."""
        return [packed[self.offsets[k]:self.offsets[k + 1]] for k in range(len(self.nx))]


def batch_from_spec(spec, device="cuda:0", instances=None) -> Batch:
    """Create, parameterise and initialise a Batch from a workloads.BatchSpec (or a subset
    of its instances)."""
    idx = list(range(len(spec.nx))) if instances is None else list(instances)
    ws = [spec.instance(k) for k in idx]
    b0 = spec.base
    b = Batch([w.nx for w in ws], b0.dx, b0.dt, b0.dvm, device=device)
    b.set_params(np.stack([np.asarray(w.R, dtype=np.float64) for w in ws]), b0.gamma, None, b0.Q,
                 b0.omega1, b0.omega2, b0.m, b0.n, b0.T_ig)
    F = [w.fields() for w in ws]
    b.init_fields(*[np.concatenate([np.asarray(f[k], dtype=np.float64).reshape(-1) for f in F])
                    for k in ("rho", "ux", "uy", "T", "lam")])
    return b


def sim_from_workload(w, device="cuda:0", pitch=None, fields=None) -> Sim:
    """Create, parameterise and initialise a Sim for a workload of
    paper_1411_6697_amd.workloads (input generation only)."""
    s = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.dvm, w.bc_x, w.bc_y, device=device, pitch=pitch)
    s.set_params(w.R, w.gamma, 0.0, w.Q, w.omega1, w.omega2, w.m, w.n, w.T_ig)
    if getattr(w, "tau", 0.0) > 0.0:
        s.set_srt(w.tau)
    if getattr(w, "rk", 1) != 1:
        s.set_time_scheme(w.rk)
    for side, spec in (getattr(w, "walls", None) or {}).items():
        s.set_boundary(side, spec)
    F = fields if fields is not None else w.fields()
    s.init_fields(F["rho"], F["ux"], F["uy"], F["T"], F["lam"])
    return s
