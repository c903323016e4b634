"""Shared test helpers: convert a workload to the oracle's parameter set, run the
oracle, and the parity metric used against the GPU path."""

from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1411_6697_amd import workloads as W


def oracle_params(w: W.Workload, **over) -> oracle.Params:
    kw = dict(dvm=oracle.DVM(*w.dvm), I=w.I, R=tuple(w.R), dx=w.dx, dy=w.dy, dt=w.dt, Q=w.Q,
              omega1=w.omega1, omega2=w.omega2, m=w.m, n=w.n, T_ig=w.T_ig,
              bc_x=w.bc_x, bc_y=w.bc_y, tau=w.tau, rk=w.rk, walls=w.walls)
    kw.update(over)
    return oracle.Params(**kw)


def oracle_init(w: W.Workload, fields=None, **over):
    P = oracle_params(w, **over)
    tab = oracle.make_tables(P)
    F = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in (fields or w.fields()).items()}
    f = oracle.init_f(F["rho"], F["ux"], F["uy"], F["T"], P, tab)
    return P, tab, f, F["lam"].clone()


def oracle_run(w: W.Workload, steps=None, fields=None, **over):
    P, tab, f, lam = oracle_init(w, fields, **over)
    f, lam = oracle.run(f, lam, P, tab, w.steps if steps is None else steps)
    return P, tab, f, lam


def max_rel_err(a: np.ndarray, b: np.ndarray, kind: str, scale: float = 0.0) -> float:
    """Parity metric.  rho, T ("pointwise"): max |a-b|/|b|.  Fields that may vanish
    ("scaled": u_x, u_y, lambda): max |a-b| / max(|b|, S) with S = max(||b||_inf, scale);
    for the velocity components `scale` is the flow-speed scale max(||u_x||, ||u_y||) so
    that a component that is zero up to rounding (u_y in a 1D run) is measured against
    the flow speed.  If S < 1e-300 the absolute error is returned."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    if kind == "pointwise":
        return float(np.max(np.abs(a - b) / np.abs(b)))
    S = max(float(np.max(np.abs(b))), float(scale))
    if S < 1e-300:
        return float(np.max(np.abs(a - b)))
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), S)))


PARITY_KIND = {"rho": "pointwise", "T": "pointwise", "ux": "scaled", "uy": "scaled", "lam": "scaled"}


def parity_errors(gpu: dict, ref: dict) -> dict:
    """max_rel_err for rho, u_x, u_y, T, lambda with the velocity scale of `ref`."""
    us = max(float(np.max(np.abs(np.asarray(ref["ux"])))), float(np.max(np.abs(np.asarray(ref["uy"])))))
    return {k: max_rel_err(gpu[k], np.asarray(ref[k]), PARITY_KIND[k],
                           us if k in ("ux", "uy") else 0.0) for k in PARITY_KIND}
