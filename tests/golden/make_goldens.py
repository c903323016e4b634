"""Write the oracle's end states of the long configurations as test goldens.

Every stored value comes from the CPU oracle (package `oracle`) run on the seeded
initial fields of `paper_1411_6697_amd.workloads`; nothing here touches the GPU
library.  The GPU parity tests load these files and compare the HIP path's end state
with them element by element.

    python tests/golden/make_goldens.py det8000     # 1D detonation, 8000 x 1, 20000 steps
    python tests/golden/make_goldens.py kh-cut      # KH cut 250 x 256, 1000 steps, reactive and inert
    python tests/golden/make_goldens.py batch128    # all 128 batched detonations, 1000 steps

Recipes (the configurations' own grids, rates, velocity models and seeds):

* det8000: the unsteady detonation (Sec. VI A case iii) on its full 8000-cell length.
  Its rows in y are identical (y-periodic, y-uniform data; the GPU test checks that the
  four rows stay bitwise equal), so one row stands for the 8000 x 4 grid.
* kh-cut: columns 0..249 and rows 384..639 of the 2048^2 Kelvin-Helmholtz fields (the
  rows across the lower shear layer), at the configuration's dx = 1/2048, dt and R_k;
  periodic in x (the initial fields do not depend on x apart from the i.i.d. noise),
  zero-gradient outflow in y.  250 columns leave a ragged last tile.  This run amplifies
  any difference in rounding by about ten times per hundred steps (the grid-scale modes
  that the white-noise seed excites grow, and minmod switches on them), so two float64
  implementations that round differently agree to 1e-10 only for about 250 steps.  The
  file holds the state after 200 steps in float64 (compared element by element) and the
  state after all 1000 steps in float32 (compared through quantities that do not depend
  on the amplified small scales).
* batch128: the 128 instances of the batched configuration, each advanced on its own,
  stored packed back to back in instance order.  1000 steps: the instances with the
  largest Prandtl numbers start an oscillation near the driver after about 2000 steps.

Files: `<name>.npz` with float64 arrays rho, ux, uy, T, lam (shape [ny, nx], or [P] for
the packed batch) and the step count (kh-cut adds end_rho ... end_lam, float32, and
end_steps); written with numpy's compressed format (the
undisturbed parts of the 1D runs are bitwise uniform and compress to almost nothing).
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle                                              # noqa: E402
from paper_1411_6697_amd import workloads as W             # noqa: E402

KH_ROWS = (384, 640)
KH_COLS = (0, 250)
KH_EXACT_STEPS = 200
BATCH_STEPS = 1000


def _params(w: W.Workload) -> oracle.Params:
    return oracle.Params(dvm=oracle.DVM(*w.dvm), I=w.I, R=tuple(w.R), dx=w.dx, dy=w.dy, dt=w.dt, Q=w.Q,
                         omega1=w.omega1, omega2=w.omega2, m=w.m, n=w.n, T_ig=w.T_ig,
                         bc_x=w.bc_x, bc_y=w.bc_y)


def _run(w: W.Workload, fields: dict, steps, label: str):
    """The oracle's moments after `steps` steps (an int), or after each of a list of step
    counts (then a list of results)."""
    P = _params(w)
    tab = oracle.make_tables(P)
    F = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)) for k, v in fields.items()}
    f = oracle.init_f(F["rho"], F["ux"], F["uy"], F["T"], P, tab)
    lam = F["lam"].clone()
    t0 = time.time()
    done, outs = 0, []
    for target in ([steps] if isinstance(steps, int) else list(steps)):
        while done < target:
            k = min(500, target - done)
            f, lam = oracle.run(f, lam, P, tab, k)
            done += k
            print(f"{label}: {done}/{target} steps, {time.time() - t0:.0f} s", flush=True)
        m = oracle.moments(f, lam, P, tab)
        out = {k: m[k].numpy().copy() for k in ("rho", "ux", "uy", "T", "lam")}
        for k, v in out.items():
            assert np.all(np.isfinite(v)), (label, k)
        assert np.all(out["rho"] > 0) and np.all(out["T"] > 0), label
        outs.append(out)
    return outs[0] if isinstance(steps, int) else outs


def det8000() -> None:
    w = W.detonation()
    F = {k: v[:1] for k, v in w.fields().items()}
    out = _run(w.with_(ny=1), F, w.steps, "det8000")
    np.savez_compressed(os.path.join(HERE, "det8000.npz"), steps=w.steps, **out)


def kh_cut() -> None:
    for reactive in (True, False):
        w = W.kh(n=2048, reactive=reactive)
        (y0, y1), (x0, x1) = KH_ROWS, KH_COLS
        F = {k: v[y0:y1, x0:x1] for k, v in w.fields().items()}
        wc = w.with_(nx=x1 - x0, ny=y1 - y0, bc_x="periodic", bc_y="outflow")
        early, end = _run(wc, F, (KH_EXACT_STEPS, w.steps), f"kh-cut reactive={reactive}")
        name = "kh_cut_reactive.npz" if reactive else "kh_cut_inert.npz"
        np.savez_compressed(os.path.join(HERE, name), steps=KH_EXACT_STEPS, end_steps=w.steps,
                            rows=np.array(KH_ROWS), cols=np.array(KH_COLS), **early,
                            **{"end_" + k: v.astype(np.float32) for k, v in end.items()})


def batch128() -> None:
    spec = W.batched()
    parts = {k: [] for k in ("rho", "ux", "uy", "T", "lam")}
    for i in range(len(spec.nx)):
        w = spec.instance(i)
        out = _run(w, w.fields(), BATCH_STEPS, f"batch[{i}] nx={w.nx}")
        for k in parts:
            parts[k].append(out[k].reshape(-1))
    packed = {k: np.concatenate(v) for k, v in parts.items()}
    np.savez_compressed(os.path.join(HERE, "batch128.npz"), steps=BATCH_STEPS, nx=np.asarray(spec.nx),
                        **packed)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["det8000", "kh-cut", "batch128"])
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads:
        torch.set_num_threads(a.threads)
    {"det8000": det8000, "kh-cut": kh_cut, "batch128": batch128}[a.which]()
