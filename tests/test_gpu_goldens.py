"""Full-run parity of the HIP path with the oracle on the long configurations.

The oracle's end states were written by tests/golden/make_goldens.py (CPU only, from the
seeded inputs of paper_1411_6697_amd.workloads); here the GPU runs the same configurations
through the C ABI and its end state is compared element by element.  Bar: max relative
error <= 1e-10 on rho, u_x, u_y, T and lambda (rho, T pointwise; u and lambda scaled by
max(|b|, ||b||_inf), the velocity components by the flow speed).
"""

import os

import numpy as np
import pytest
import torch

from paper_1411_6697_amd import workloads as W
from tests.helpers import PARITY_KIND, parity_errors

pytestmark = pytest.mark.gpu
TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lbkm():
    from paper_1411_6697_amd import lbkm
    return lbkm


def _load(name):
    with np.load(os.path.join(GOLDEN, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _check(g, ref, label):
    errs = parity_errors({k: g[k] for k in PARITY_KIND}, {k: ref[k] for k in PARITY_KIND})
    print(label, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= TOL, (label, k, e)


def test_detonation_8000x4_full_run_matches_oracle():
    """The unsteady detonation configuration (Sec. VI A case iii), 8000 x 4 cells, all 20000
    steps: the four rows stay bitwise identical and row 0 matches the oracle's 8000-cell
    run everywhere."""
    ref = _load("det8000.npz")
    w = W.detonation()
    assert int(ref["steps"]) == w.steps
    s = _lbkm().sim_from_workload(w)
    s.step(w.steps)
    assert s.check()
    g = {k: v.cpu().numpy() for k, v in s.moments().items()}
    for k in g:
        for r in range(1, w.ny):
            assert np.array_equal(g[k][0], g[k][r]), (k, r)
    _check({k: g[k][0] for k in g}, {k: ref[k][0] for k in PARITY_KIND}, "det8000 step 20000")
    # the reaction has spread beyond the 200-cell driver (burnt past cell 300, the leading
    # shock near cell 790), the far part of the tube is still undisturbed
    assert np.nonzero(g["lam"][0] > 0.5)[0].max() > 300 and g["lam"][0, 1000:].max() == 0.0


def _kh_cut(reactive, ref, perturb=0.0):
    w = W.kh(n=2048, reactive=reactive)
    (y0, y1), (x0, x1) = ref["rows"], ref["cols"]
    F = {k: np.ascontiguousarray(v[y0:y1, x0:x1]) for k, v in w.fields().items()}
    if perturb:
        F["uy"] = F["uy"] * (1.0 + perturb)
    wc = w.with_(nx=int(x1 - x0), ny=int(y1 - y0), bc_x="periodic", bc_y="outflow")
    return _lbkm().sim_from_workload(wc, fields=F)


def _moments(s):
    return {k: v.cpu().numpy() for k, v in s.moments().items()}


@pytest.mark.parametrize("reactive", [True, False])
def test_kelvin_helmholtz_cut_matches_oracle(reactive):
    """The Kelvin-Helmholtz configuration's fields, dx = 1/2048, dt and R_k, on a 250 x 256
    cut across the lower shear layer (periodic in x, outflow in y), with the launch shape and
    tile order the autotuner picks for the cut.

    After 200 steps: element by element at 1e-10.  This run amplifies differences of
    rounding by about ten times per hundred steps (the grid-scale modes that the white-noise
    seed excites grow, and minmod switches on them), so after all 1000 steps two float64
    implementations that round differently no longer agree pointwise (measured: GPU and
    oracle apart by 1e-11 at step 200, 1e-9 at 400, 1e-3 at 800 in the reactive run).  At
    step 1000 the test asks instead that the HIP result stay as close to the oracle's as
    the HIP run itself moves when its initial u_y is changed by one part in 1e10: the
    difference is then of the size the conditioning of the run gives to a 1e-10 change of
    the input."""
    ref = _load("kh_cut_reactive.npz" if reactive else "kh_cut_inert.npz")
    s = _kh_cut(reactive, ref)
    launch = s.autotune()
    print("launch", launch, flush=True)
    s.step(int(ref["steps"]))
    assert s.check()
    _check(_moments(s), ref, f"kh-cut reactive={reactive} step {int(ref['steps'])}")
    s.step(int(ref["end_steps"]) - int(ref["steps"]))
    assert s.check()
    a = _moments(s)
    end = {k: ref["end_" + k].astype(np.float64) for k in PARITY_KIND}
    d_oracle = parity_errors(a, end)
    p = _kh_cut(reactive, ref, perturb=1e-10)
    p.set_tile(*launch[:3])
    p.set_tile_order(launch[3])
    p.step(int(ref["end_steps"]))
    d_input = parity_errors(_moments(p), a)
    print("step", int(ref["end_steps"]), "vs oracle", {k: f"{v:.2e}" for k, v in d_oracle.items()},
          "vs input change 1e-10", {k: f"{v:.2e}" for k, v in d_input.items()}, flush=True)
    assert max(d_oracle.values()) <= max(d_input.values())


def test_batch_all_128_instances_match_oracle():
    """The batched configuration (128 ragged detonations, one persistent launch per step
    call, autotuned work-group count, hipGraph replays): every instance against the oracle
    after 1000 steps."""
    ref = _load("batch128.npz")
    spec = W.batched()
    assert np.array_equal(ref["nx"], spec.nx)
    b = _lbkm().batch_from_spec(spec)
    print("autotuned cells per work-group:", b.autotune(), flush=True)
    steps = int(ref["steps"])
    for n in (500, 500):
        b.step(n)
    assert sum((500, 500)) == steps
    print("launch shape:", b.status(), flush=True)
    m = b.moments()
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in m.items()}
    off = b.offsets
    worst = {k: 0.0 for k in PARITY_KIND}
    for i in range(len(spec.nx)):
        sl = slice(off[i], off[i + 1])
        errs = parity_errors({k: g[k][sl] for k in PARITY_KIND}, {k: ref[k][sl] for k in PARITY_KIND})
        for k, e in errs.items():
            worst[k] = max(worst[k], e)
            assert e <= TOL, (i, int(spec.nx[i]), k, e)
    print("batch128 step", steps, "worst over instances", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
