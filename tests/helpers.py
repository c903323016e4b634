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
              bc_x=w.bc_x, bc_y=w.bc_y)
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


def max_rel_err(a: np.ndarray, b: np.ndarray, kind: str) -> float:
    """Parity metric.  rho, T: pointwise |a-b|/|b|.  Fields that may vanish (u_x, u_y,
    lambda): |a-b| / max(|b|, ||b||_inf); if ||b||_inf < 1e-300 the absolute error."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if kind == "pointwise":
        return float(np.max(np.abs(a - b) / np.abs(b)))
    nb = float(np.max(np.abs(b))) if b.size else 0.0
    if nb < 1e-300:
        return float(np.max(np.abs(a - b))) if b.size else 0.0
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), nb)))


PARITY_KIND = {"rho": "pointwise", "T": "pointwise", "ux": "scaled", "uy": "scaled", "lam": "scaled"}
