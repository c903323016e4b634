"""Benchmark of the MRT-LBKM step on one MI355X.

Workload: the doubly periodic 2048 x 2048 Kelvin-Helmholtz configuration (reactive, Q = 1;
the inert Q = 0 run is reported beside it), float64.  One step = one full time step of the
method over the grid (macroscopic moments, f_hat = M f, equilibrium, A_hat, collision,
chemistry and C_i, M^-1, NND streaming, forward Euler, lambda update), i.e. one launch of
the fused step kernel.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
BYTES_PER_CELL = 400            # 24 f read + 24 f written + lambda read + lambda written, 8 B each
PMC_FILE = os.path.join(ROOT, "profiles", "k_step_kh2048_pmc.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1411_6697_amd", "csrc", n)
                  for n in ("step.hip", "lbkm_device.h", "lbkm_internal.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the step kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    if not os.path.exists(PMC_FILE):
        return None
    vals = {}
    with open(PMC_FILE) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(sim, steps, warmup):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    sim.step(steps)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps       # ms per step (= per step-kernel launch)


def copy_ceiling_gbs(n_bytes=1 << 31):
    """Achievable HBM bandwidth of the library's plain copy kernel (read + write bytes)."""
    import ctypes
    import torch
    from paper_1411_6697_amd import lbkm
    lib = lbkm.load()
    n = n_bytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(3):
        lib.lbkm_copy_kernel(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        lib.lbkm_copy_kernel(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def cpu_baseline(w, tile=1024, steps=8):
    """Oracle timing on the host cores: a tile x tile periodic cut of the same initial fields,
    `steps` steps after one untimed step."""
    import numpy as np
    import torch
    import oracle
    F = w.fields()
    cut = {k: np.ascontiguousarray(v[:tile, :tile]) for k, v in F.items()}
    P = oracle.Params(dvm=oracle.DVM(*w.dvm), I=w.I, R=w.R, dx=w.dx, dy=w.dy, dt=w.dt, Q=w.Q,
                      omega1=w.omega1, omega2=w.omega2, m=w.m, n=w.n, T_ig=w.T_ig,
                      bc_x="periodic", bc_y="periodic")
    tab = oracle.make_tables(P)
    t = {k: torch.from_numpy(v) for k, v in cut.items()}
    f = oracle.init_f(t["rho"], t["ux"], t["uy"], t["T"], P, tab)
    lam = t["lam"]
    f, lam = oracle.step(f, lam, P, tab)
    t0 = time.perf_counter()
    f, lam = oracle.run(f, lam, P, tab, steps)
    dt = time.perf_counter() - t0
    return {"value": round(tile * tile * steps / dt / 1e6, 4), "unit": "MLUPS",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{tile}x{tile} periodic cut of the 2048^2 KH initial fields (reactive), "
                      f"{steps} steps after 1 untimed step, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-inert", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_1411_6697_amd import lbkm
    from paper_1411_6697_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = W.kh(n=args.n, steps=args.steps, reactive=True)
    cells = w.nx * w.ny
    sim = lbkm.sim_from_workload(w)
    ms = time_steps(sim, args.steps, args.warmup)
    ok = sim.check()
    del sim
    torch.cuda.empty_cache()
    value = cells / (ms * 1e-3) / 1e6

    inert = None
    if not args.no_inert:
        w0 = W.kh(n=args.n, steps=args.steps, reactive=False)
        s0 = lbkm.sim_from_workload(w0)
        ms0 = time_steps(s0, args.steps, args.warmup)
        del s0
        torch.cuda.empty_cache()
        inert = {"mlups": round(cells / (ms0 * 1e-3) / 1e6, 2), "ms_per_step": round(ms0, 5)}

    achieved = BYTES_PER_CELL * cells / (ms * 1e-3) / 1e9
    ceiling = copy_ceiling_gbs()
    traffic = measured_traffic()
    out = {
        "metric": "MLUPS (cell updates/s) FP64 at 2048^2",
        "value": round(value, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"kelvin_helmholtz_{w.nx}x{w.ny}_reactive_Q1_periodic",
                   "nx": w.nx, "ny": w.ny, "dt": w.dt, "velocities": "D2V24",
                   "state_finite_after_run": bool(ok)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_step",
                     "algorithmic_bytes_per_cell": BYTES_PER_CELL,
                     "copy_kernel_gbs": round(ceiling, 1)},
        "inert_Q0": inert,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
