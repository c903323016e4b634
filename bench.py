"""Benchmark of the MRT-LBKM step on one MI355X.

Workload: the doubly periodic 2048 x 2048 Kelvin-Helmholtz configuration (reactive, Q = 1;
the inert Q = 0 run is reported beside it), float64.  One step = one full time step of the
method over the grid (macroscopic moments, f_hat = M f, equilibrium, A_hat, collision,
chemistry and C_i, M^-1, NND streaming, forward Euler, lambda update), i.e. one launch of
the fused step kernel.  Reported beside it on the same GPU: the batched form (128 ragged
1D detonations, one persistent launch per graph replay) and the adjoint form (gradient of
the non-equilibrium loss over a 2048 x 256 detonation strip, 500 steps, checkpoints every
50), each against the plain step's time per cell-update, and the reactive run with the
single-relaxation-time collision (Sec. V, the MRT/SRT cost ratio of Table I), with the
SSP Runge-Kutta time schemes, and between reflecting walls; and the two small
configurations (Sod 400 x 1, the detonation 8000 x 4) as whole runs with the oracle's rates
beside them.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--no-cpu-baseline]
                  [--no-inert] [--no-batched] [--no-adjoint] [--no-srt] [--no-rk] [--no-walls]
                  [--no-small]
                  [--launch TXxTY[l|s|h]:ORDER]   (fix the step's launch instead of autotuning it)
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


STEP_KERNELS = {0: "k_step", 1: "k_step_lds", 2: "k_step_sf", 3: "k_step_sh"}    # launch mode -> kernel


def step_kernel_name(tile) -> str:
    """Name of the step kernel a launch (tile_x, tile_y, mode) runs, as the profiler shows
    it up to the specialisation flags."""
    return f"{STEP_KERNELS[int(tile[2])]}<{int(tile[0])},{int(tile[1])}>"


def measured_traffic(tile):
    """HBM bytes per launch of the step kernel at launch `tile` = (tile_x, tile_y, mode) or
    (tile_x, tile_y, mode, column_bands), from the committed rocprofv3 counter summary, if
    that was taken on the current kernel source and holds that launch shape (and, when
    given, that tile order); else None."""
    if not os.path.exists(PMC_FILE):
        return None
    src_hash, per_kernel = None, {}
    with open(PMC_FILE) as fh:
        for line in fh:
            parts = line.split()
            if not parts or line.startswith("#"):
                continue
            if parts[0] == "kernel_source_sha256" and len(parts) > 1:
                src_hash = parts[1]
            elif parts[0] == "kernel" and len(parts) > 2:
                kv = dict(zip(parts[2::2], parts[3::2]))
                per_kernel[parts[1]] = kv
    if src_hash != kernel_source_hash():
        return None
    want = STEP_KERNELS[int(tile[2])] + f"<{int(tile[0])},{int(tile[1])},"
    for name, kv in per_kernel.items():
        if name.startswith(want):
            if len(tile) > 3 and kv.get("launch", "").rpartition(":")[2] != str(int(tile[3])):
                return None
            try:
                return float(kv["hbm_bytes_per_launch"])
            except (KeyError, ValueError):
                return None
    return None


def _finite_or_none(v):
    """A float for the JSON line, None where it is not finite (the margin of a state
    without unburnt cells is +inf)."""
    import math
    return v if math.isfinite(v) else None


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


COPY_BYTES = 25 * 2048 * 2048 * 8      # one 2048^2 step's state: 24 planes + lambda


def copy_ceiling_gbs(n_bytes=COPY_BYTES):
    """Achievable HBM bandwidth of the library's plain copy kernel (read + write bytes) over
    as many bytes as one 2048^2 step reads."""
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
    cores = torch.get_num_threads()
    # the same oracle on one thread, on a 256^2 corner of the cut for 4 steps
    small = 256
    f1 = oracle.init_f(*(t[k][:small, :small].contiguous() for k in ("rho", "ux", "uy", "T")), P, tab)
    l1 = t["lam"][:small, :small].contiguous()
    torch.set_num_threads(1)
    try:
        f1, l1 = oracle.step(f1, l1, P, tab)
        t1 = time.perf_counter()
        f1, l1 = oracle.run(f1, l1, P, tab, 4)
        dt1 = time.perf_counter() - t1
    finally:
        torch.set_num_threads(cores)
    return {"value": round(tile * tile * steps / dt / 1e6, 4), "unit": "MLUPS",
            "cores": cores, "kind": "oracle",
            "sample": f"{tile}x{tile} periodic cut of the 2048^2 KH initial fields (reactive), "
                      f"{steps} steps after 1 untimed step, {dt:.1f} s",
            "one_thread_value": round(small * small * 4 / dt1 / 1e6, 4),
            "one_thread_sample": f"{small}x{small} corner of the same cut, 4 steps after 1 untimed step, "
                                 f"{dt1:.1f} s"}


def bench_batched(ns_per_cell_plain, steps=5000, chunk=500, launch=None):
    """Config of 128 ragged 1D detonations: autotune (one launch per step, or the persistent
    kernel at 1-8 work-groups per CU), then `steps` steps in calls of `chunk` steps each
    (each call replays captured graphs).  `launch` fixes the mode instead (0: one launch per
    step, 1..8: persistent at that many work-groups per CU)."""
    import torch
    from paper_1411_6697_amd import lbkm
    from paper_1411_6697_amd import workloads as W
    spec = W.batched(steps=steps)
    b = lbkm.batch_from_spec(spec)
    if launch is None:
        cells_per_wg = b.autotune()
    else:
        b.set_launch(launch)
        cells_per_wg = -(-b.total // b.status()[0])
    b.step(chunk)                                  # captures the replayed graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps // chunk):
        b.step(chunk)
    e1.record()
    torch.cuda.synchronize()
    wgs, per_cu = b.status()
    ms = e0.elapsed_time(e1) / (steps // chunk * chunk)
    mlups = b.total / (ms * 1e-3) / 1e6
    m = b.moments()
    good = (torch.isfinite(m["rho"]) & (m["T"] > 0)).cpu().numpy()
    ok = [bool(good[b.offsets[k]:b.offsets[k + 1]].all()) for k in range(len(spec.nx))]
    lost = [k for k in range(len(spec.nx)) if not ok[k]]
    # steps 500..1500 timed alone (every instance is physical until about step 2000; the
    # oracle goldens cover the first 1000), and the number of physical instances as the run
    # goes on
    b2 = lbkm.batch_from_spec(spec)
    b2.set_launch(per_cu)
    b2.step(chunk)                                 # captures the graph
    torch.cuda.synchronize()
    window = 1000
    e0.record()
    for _ in range(window // chunk):
        b2.step(chunk)
    e1.record()
    torch.cuda.synchronize()
    ms_w = e0.elapsed_time(e1) / window
    physical = {}
    done = chunk + window
    physical[done] = _physical_count(b2, spec)
    while done < steps:
        b2.step(chunk)
        done += chunk
        physical[done] = _physical_count(b2, spec)
    b2.close()
    # the same instances as separate single-grid runs, one launch per instance and step
    sims = [lbkm.sim_from_workload(spec.instance(k)) for k in range(len(spec.nx))]
    for s_ in sims:
        s_.step(2)
    torch.cuda.synchronize()
    sep_steps = 20
    t0 = time.perf_counter()
    for _ in range(sep_steps):
        for s_ in sims:
            s_.step(1)
    torch.cuda.synchronize()
    sep_ms = (time.perf_counter() - t0) * 1e3 / sep_steps
    del sims
    gbs = BYTES_PER_CELL * b.total / (ms * 1e-3) / 1e9
    return {"workload": f"batched_{len(spec.nx)}_detonations_nx_1000_8000_outflow", "instances": len(spec.nx),
            "cells": int(b.total), "steps": steps // chunk * chunk, "ms_per_step": round(ms, 5),
            "mlups": round(mlups, 2), "algorithmic_gbs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "ns_per_cell_update": round(ms * 1e6 / b.total, 5),
            "vs_plain_step_time_per_cell": round(ms * 1e6 / b.total / ns_per_cell_plain, 3),
            "launch_mode": "one launch per step" if per_cu == 0 else "persistent",
            "work_groups": wgs, "work_groups_per_cu": per_cu, "cells_per_work_group": cells_per_wg,
            "steps_per_call": chunk,
            "instances_physical_after_run": sum(ok),
            # instances whose temperature turned non-positive (the explicit scheme loses
            # stability near the driver when Pr approaches 5; the CPU oracle does the same)
            "instances_lost": {int(k): round(float(spec.Pr[k]), 3) for k in lost},
            "physical_window": {"steps": [chunk, chunk + window], "ms_per_step": round(ms_w, 5),
                                "mlups": round(b.total / (ms_w * 1e-3) / 1e6, 2),
                                "hbm_frac": round(BYTES_PER_CELL * b.total / (ms_w * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                "vs_plain_step_time_per_cell": round(ms_w * 1e6 / b.total / ns_per_cell_plain, 3)},
            "physical_instances_after_step": {str(k): v for k, v in physical.items()},
            "separate_launches_mlups": round(b.total / (sep_ms * 1e-3) / 1e6, 2)}


def _physical_count(b, spec):
    import torch
    m = b.moments()
    good = (torch.isfinite(m["rho"]) & (m["T"] > 0)).cpu().numpy()
    return int(sum(bool(good[b.offsets[k]:b.offsets[k + 1]].all()) for k in range(len(spec.nx))))


def _oracle_rate(w, steps, threads):
    """The oracle's cell-update rate (MLUPS) on `threads` host threads over `steps` steps of
    workload w from its initial fields, after one untimed step."""
    import numpy as np
    import torch
    import oracle
    P = oracle.Params(dvm=oracle.DVM(*w.dvm), I=w.I, R=w.R, dx=w.dx, dy=w.dy, dt=w.dt, Q=w.Q,
                      omega1=w.omega1, omega2=w.omega2, m=w.m, n=w.n, T_ig=w.T_ig, bc_x=w.bc_x, bc_y=w.bc_y)
    tab = oracle.make_tables(P)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in w.fields().items()}
    before = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        f = oracle.init_f(t["rho"], t["ux"], t["uy"], t["T"], P, tab)
        f, lam = oracle.step(f, t["lam"], P, tab)
        t0 = time.perf_counter()
        f, lam = oracle.run(f, lam, P, tab, steps)
        dt = time.perf_counter() - t0
    finally:
        torch.set_num_threads(before)
    return w.nx * w.ny * steps / dt / 1e6, dt


def bench_small_configs(ns_per_cell_plain, oracle_rates=True):
    """The two small configurations, each as a whole run from its initial fields on the GPU
    (launch shape autotuned first): Sod 400 x 1 for 2000 steps and the detonation 8000 x 4
    for 20000 steps; beside them the oracle's rate on one host thread and on all of them,
    over a bounded number of steps of the same run."""
    import torch
    from paper_1411_6697_amd import lbkm
    from paper_1411_6697_amd import workloads as W
    out = {}
    for name, w, osteps in (("sod_400x1_2000_steps", W.sod(), 200),
                            ("detonation_8000x4_20000_steps", W.detonation(), 20)):
        s = lbkm.sim_from_workload(w)
        launch = s.autotune()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(w.steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        cells = w.nx * w.ny
        gbs = BYTES_PER_CELL * cells * w.steps / (ms * 1e-3) / 1e9
        r = {"cells": cells, "steps": w.steps, "run_ms": round(ms, 3), "ms_per_step": round(ms / w.steps, 5),
             "mlups": round(cells * w.steps / (ms * 1e-3) / 1e6, 2), "algorithmic_gbs": round(gbs, 1),
             "hbm_frac": round(gbs / HBM_PEAK_GBS, 5), "launch": list(launch), "finite": bool(s.check()),
             "ignition_margin_after_run": _finite_or_none(s.ignition_margin())}
        s.close()
        if oracle_rates:
            r1, d1 = _oracle_rate(w, osteps, 1)
            ra, da = _oracle_rate(w, osteps, torch.get_num_threads())
            r["oracle_mlups_1_thread"] = round(r1, 4)
            r["oracle_mlups_all_threads"] = round(ra, 4)
            r["oracle_threads"] = torch.get_num_threads()
            r["oracle_sample"] = f"{osteps} steps of the same run after 1 untimed step ({d1:.1f} s, {da:.1f} s)"
        out[name] = r
    return out


def bench_adjoint(ns_per_cell_plain):
    """Gradient of the non-equilibrium loss of the 2048 x 256 strip after 500 steps with
    respect to (R_1..R_24, Q, omega_1, omega_2) and the initial fields: checkpointed
    forward, recomputation and the adjoint steps, wall time of the whole backward pass;
    the adjoint step alone timed with events over 100 calls."""
    import torch
    from paper_1411_6697_amd import lbkm
    from paper_1411_6697_amd import workloads as W
    w = W.adjoint_strip()
    cells = w.nx * w.ny
    plain = lbkm.sim_from_workload(w)
    plain.autotune()
    ms_plain = time_steps(plain, 200, 10)
    del plain
    s = lbkm.Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.dvm, w.bc_x, w.bc_y)
    F = w.fields()
    theta = torch.tensor(list(w.R) + [w.Q, w.omega1, w.omega2], dtype=torch.float64, requires_grad=True)
    ts = [torch.tensor(F[k], dtype=torch.float64, device=s.device, requires_grad=True)
          for k in ("rho", "ux", "uy", "T", "lam")]
    times = []
    for _ in range(2):                             # the first pass warms up allocations
        theta.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fN, lN = lbkm.LBKMRun.apply(theta, *ts, s, w.steps, w.gamma, 50, w.m, w.n, w.T_ig)
        loss = lbkm.TNELoss.apply(fN, s)
        loss.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    f, lam = s.get_state()
    af = torch.ones_like(f)
    al = torch.ones_like(lam)
    grad = torch.zeros(lbkm.NUM_GRAD, dtype=torch.float64, device=s.device)
    s.adjoint_step(f, lam, af, al, grad)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 100
    e0.record()
    for _ in range(reps):
        af, al = s.adjoint_step(f, lam, af, al, grad)
    e1.record()
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1) / reps
    return {"workload": f"detonation_strip_{w.nx}x{w.ny}_{w.steps}_steps_checkpoint_50",
            "loss": float(loss.detach()), "gradient_wall_s": round(times[-1], 4),
            "plain_step_ms": round(ms_plain, 5), "adjoint_step_ms": round(ms_adj, 5),
            "adjoint_step_vs_plain_step": round(ms_adj / ms_plain, 3),
            "gradient_vs_plain_run": round(times[-1] / (w.steps * ms_plain * 1e-3), 3),
            "plain_ns_per_cell_update": round(ms_plain * 1e6 / cells, 5),
            "vs_kh_plain_step_time_per_cell": round(ms_adj * 1e6 / cells / ns_per_cell_plain, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-inert", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-srt", action="store_true")
    ap.add_argument("--no-rk", action="store_true")
    ap.add_argument("--no-walls", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="fix the KH step's launch instead of autotuning it: TXxTY[l|s|h]:ORDER, e.g. 64x4s:1 "
                         "(l = LDS-staged stencil, s = stream-first kernel, h = centre values shared in LDS, ORDER 1 = "
                         "column bands); used to "
                         "profile a stated shape")
    ap.add_argument("--batch-launch", type=int, default=None,
                    help="fix the batched run's launch instead of autotuning it: 0 = one launch per step, "
                         "1..8 = the persistent kernel at that many work-groups per CU")
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
    if args.launch:
        shape, order = args.launch.split(":")
        lds = {"l": 1, "s": 2, "h": 3}.get(shape[-1], 0)
        tx, ty = (int(v) for v in shape.rstrip("lsh").split("x"))
        sim.set_tile(tx, ty, lds)
        sim.set_tile_order(int(order))
        launch = (tx, ty, lds, int(order))
    else:
        launch = sim.autotune()                 # launch shape: tile, LDS staging, tile order
    ms = time_steps(sim, args.steps, args.warmup)
    ok = sim.check()
    margin = _finite_or_none(sim.ignition_margin())
    del sim
    torch.cuda.empty_cache()
    value = cells / (ms * 1e-3) / 1e6

    inert = None
    if not args.no_inert:
        w0 = W.kh(n=args.n, steps=args.steps, reactive=False)
        s0 = lbkm.sim_from_workload(w0)
        s0.autotune()
        ms0 = time_steps(s0, args.steps, args.warmup)
        del s0
        torch.cuda.empty_cache()
        inert = {"mlups": round(cells / (ms0 * 1e-3) / 1e6, 2), "ms_per_step": round(ms0, 5)}

    srt = None
    if not args.no_srt:
        # the same reactive run with the single-relaxation-time collision (Eq. SRT), tau = 1/R_k
        ws = w.with_(tau=1.0 / w.R[4])
        s1 = lbkm.sim_from_workload(ws)
        launch_srt = s1.autotune()
        ms1 = time_steps(s1, args.steps, args.warmup)
        del s1
        torch.cuda.empty_cache()
        srt = {"tau": ws.tau, "mlups": round(cells / (ms1 * 1e-3) / 1e6, 2), "ms_per_step": round(ms1, 5),
               "launch": list(launch_srt), "mrt_over_srt_time": round(ms / ms1, 4),
               "paper_table_I_mrt_over_srt_time": round(2293.93 / 2221.58, 4)}

    schemes = None
    if not args.no_rk:
        # the same reactive run with the SSP Runge-Kutta schemes (2 and 3 stage launches per step)
        schemes = {}
        for rk in (2, 3):
            s2 = lbkm.sim_from_workload(w.with_(rk=rk))
            s2.set_tile(*launch[:3])
            s2.set_tile_order(launch[3])
            ms2 = time_steps(s2, max(args.steps // rk, 1), args.warmup)
            schemes[f"rk{rk}"] = {"ms_per_step": round(ms2, 5), "mlups": round(cells / (ms2 * 1e-3) / 1e6, 2),
                                  "time_over_euler": round(ms2 / ms, 4), "finite": bool(s2.check())}
            del s2
            torch.cuda.empty_cache()

    walls = None
    if not args.no_walls:
        # the same reactive run between reflecting walls at both y sides (ghost layers filled
        # before each step, the ghost-aware step specialisation)
        ww = w.with_(bc_y="outflow", walls={"y_lo": ("reflect",), "y_hi": ("reflect",)})
        s3 = lbkm.sim_from_workload(ww)
        launch_w = s3.autotune()                   # the wall shape is fixed; this picks the tile order
        ms3 = time_steps(s3, args.steps, args.warmup)
        walls = {"ms_per_step": round(ms3, 5), "mlups": round(cells / (ms3 * 1e-3) / 1e6, 2),
                 "time_over_periodic": round(ms3 / ms, 4), "launch": list(launch_w), "finite": bool(s3.check())}
        del s3
        torch.cuda.empty_cache()

    achieved = BYTES_PER_CELL * cells / (ms * 1e-3) / 1e9
    ceiling = copy_ceiling_gbs()
    traffic = measured_traffic(launch[:4])
    out = {
        "metric": "MLUPS (cell updates/s) FP64 at 2048\u00b2; batched & adjoint vs plain step time",
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
                   "nx": w.nx, "ny": w.ny, "dx": w.dx, "dt": w.dt, "velocities": "D2V24",
                   "dvm_va_vb_vc_eta_a_eta_b_eta_c": list(w.dvm), "gamma": w.gamma, "Q": w.Q,
                   "rates": "R_1..R_24 = %g (all equal)" % w.R[4] if len(set(w.R)) == 1 else list(w.R),
                   "omega1_omega2": [w.omega1, w.omega2],
                   "launch": {"tile": [launch[0], launch[1]], "lds": launch[2], "column_bands": launch[3]},
                   "state_finite_after_run": bool(ok), "ignition_margin_after_run": margin},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": step_kernel_name(launch[:3]),
                     "algorithmic_bytes_per_cell": BYTES_PER_CELL,
                     "copy_kernel_gbs": round(ceiling, 1)},
        "inert_Q0": inert,
        "srt_collision": srt,
        "runge_kutta": schemes,
        "reflecting_walls_y": walls,
    }
    ns_cell = ms * 1e6 / cells
    if not args.no_batched:
        out["batched"] = bench_batched(ns_cell, launch=args.batch_launch)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(ns_cell)
        torch.cuda.empty_cache()
    if not args.no_small:
        out["small_configs"] = bench_small_configs(ns_cell, oracle_rates=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
