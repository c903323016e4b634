"""Batched 1D path (a ragged batch of independent detonation tubes advanced by one
persistent launch per lbkm_batch_step call, or by one launch per step): parity with the CPU
oracle instance by instance (max relative error <= 1e-10, same metric as the single-grid
tests), agreement with the single-grid path, and invariance under the launch mode and
shape, the autotuner and the way the steps are chunked.
"""

import numpy as np
import pytest
import torch

from paper_1411_6697_amd import workloads as W
from tests.helpers import PARITY_KIND, oracle_run, parity_errors

pytestmark = pytest.mark.gpu
TOL = 1e-10
# the batched cell update performs the same operations as the single-grid one with the
# y-differences dropped (they are exact zeros there); allow a few ulps of slack in case the
# compiler contracts a multiply-add differently
SAME_TOL = 1e-13


def _lbkm():
    from paper_1411_6697_amd import lbkm
    return lbkm


def _edge_spec():
    """Nine instances: single-cell, two-cell and odd lengths, lengths around one and two
    work-group ranges, per-instance rates (Pr != 1, so A_hat is active) from the batch
    recipe."""
    s = W.batched(n_inst=9, nx_lo=1, nx_hi=400, seed=7)
    nx = np.array([1, 2, 3, 5, 64, 65, 257, 300, 400])
    return W.BatchSpec(nx=nx, R=s.R, Pr=s.Pr, base=s.base)


def _moments(b):
    m = b.moments()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in m.items()}


def _split(b, m):
    return [{k: v[b.offsets[i]:b.offsets[i + 1]] for k, v in m.items()} for i in range(len(b.nx))]


def _assert_parity_with_oracle(spec, k, g, steps, label):
    import oracle
    P, tab, f, lam = oracle_run(spec.instance(k), steps=steps)
    om = oracle.moments(f, lam, P, tab)
    ref = {q: om[q].numpy().reshape(-1) for q in PARITY_KIND}
    errs = parity_errors({q: g[q].reshape(-1) for q in PARITY_KIND}, ref)
    print(label, k, spec.nx[k], {q: f"{v:.2e}" for q, v in errs.items()}, flush=True)
    for q, e in errs.items():
        assert e <= TOL, (label, k, q, e)


def _single_grid(spec, k, steps):
    s = _lbkm().sim_from_workload(spec.instance(k))
    s.step(steps)
    m = s.moments()
    torch.cuda.synchronize()
    out = {q: v.cpu().numpy().reshape(-1) for q, v in m.items()}
    s.close()
    return out


def _max_rel_diff(a, b):
    """Largest difference relative to each field's magnitude; the velocity components are
    measured against the flow speed (u_y of a 1D run is rounding noise, as in the parity
    metric)."""
    speed = max(float(np.max(np.abs(b["ux"]))), float(np.max(np.abs(b["uy"]))), 1e-300)
    worst = 0.0
    for q in ("rho", "ux", "uy", "T", "lam"):
        x, y = np.asarray(a[q]).reshape(-1), np.asarray(b[q]).reshape(-1)
        scale = speed if q in ("ux", "uy") else max(float(np.max(np.abs(y))), 1e-300)
        worst = max(worst, float(np.max(np.abs(x - y))) / scale)
    return worst


@pytest.mark.parametrize("wgs_per_cu", [2, 0])
def test_ragged_edge_batch_matches_oracle_per_instance(wgs_per_cu):
    """Persistent kernel (2 work-groups per CU) and one launch per step (0)."""
    spec = _edge_spec()
    b = _lbkm().batch_from_spec(spec)
    b.set_launch(wgs_per_cu)
    b.step(120)
    b.step(180)
    print("launch shape (wgs, wgs/CU):", b.status(), flush=True)
    per = _split(b, _moments(b))
    for k in range(len(spec.nx)):
        _assert_parity_with_oracle(spec, k, per[k], 300, "edge batch")


def test_launch_per_step_gives_the_persistent_kernels_bits():
    """One launch per step (graphs of 64 launches and a remainder) against the persistent
    kernel at 1 and 2 work-groups per CU: the same cells, bit for bit, including waves that
    hold several short instances and calls whose step counts cross the 64-step chunks."""
    spec = _edge_spec()
    runs = {}
    for mode in (0, 1, 2):
        b = _lbkm().batch_from_spec(spec)
        b.set_launch(mode)
        for n in (77, 53, 64, 1):
            b.step(n)
        assert b.status()[1] == mode
        runs[mode] = _moments(b)
    for mode in (1, 2):
        for q in ("rho", "ux", "uy", "T", "lam"):
            assert np.array_equal(runs[0][q], runs[mode][q]), (mode, q)


def test_batch_refuses_the_srt_switch_and_runge_kutta():
    """The single-relaxation-time form and the Runge-Kutta schemes are single-grid options;
    a batched context refuses them (ESTATE) and keeps stepping in the MRT form."""
    L = _lbkm()
    b = L.batch_from_spec(_edge_spec())
    assert b.lib.lbkm_set_srt(b.h, 1e-3) == -5
    assert "batched" in b.lib.lbkm_last_error(b.h).decode()
    assert b.lib.lbkm_set_time_scheme(b.h, 2) == -5
    b.step(2)
    b.status()


def test_batch_agrees_with_single_grid_path():
    spec = _edge_spec()
    b = _lbkm().batch_from_spec(spec)
    b.step(200)
    b.status()
    per = _split(b, _moments(b))
    for k in range(len(spec.nx)):
        d = _max_rel_diff(per[k], _single_grid(spec, k, 200))
        print("batch vs single grid", k, spec.nx[k], f"{d:.1e}", flush=True)
        assert d <= SAME_TOL, (k, d)


def test_step_chunking_and_autotune_do_not_change_results():
    spec = W.batched(n_inst=24, nx_lo=50, nx_hi=3000, seed=11)
    a = _lbkm().batch_from_spec(spec)
    a.step(64)
    a.status()
    ra = _moments(a)
    b = _lbkm().batch_from_spec(spec)
    cells = b.autotune()                      # trial steps run on a saved copy of the state
    print("autotuned cells per work-group:", cells, "shape:", b.status(), flush=True)
    for n in (1, 1, 2, 3, 5, 8, 13, 31):      # 64 steps, both buffer parities, several graphs
        b.step(n)
    b.status()
    rb = _moments(b)
    for q in ("rho", "ux", "uy", "T", "lam"):
        assert np.array_equal(ra[q], rb[q]), q


def test_full_size_batch_sampled_instances():
    """The 128-instance batch (lengths U{1000..8000}): every instance finite after 400
    steps; the shortest instance against the oracle; the shortest, longest and a middle
    one against the single-grid path."""
    spec = W.batched()
    b = _lbkm().batch_from_spec(spec)
    b.autotune()
    b.step(200)
    b.step(200)
    print("full batch shape:", b.status(), "cells:", b.total, flush=True)
    m = _moments(b)
    for q in ("rho", "ux", "T", "lam"):
        assert np.all(np.isfinite(m[q])), q
    assert np.all(m["rho"] > 0) and np.all(m["T"] > 0)
    per = _split(b, m)
    order = np.argsort(spec.nx)
    short, long_, mid = int(order[0]), int(order[-1]), int(order[len(order) // 2])
    _assert_parity_with_oracle(spec, short, per[short], 400, "full batch")
    for k in (short, mid, long_):
        d = _max_rel_diff(per[k], _single_grid(spec, k, 400))
        print("full batch vs single grid", k, spec.nx[k], f"{d:.1e}", flush=True)
        assert d <= SAME_TOL, (k, d)


@pytest.mark.parametrize("wgs_per_cu", [2, 0])
def test_batch_with_rate_exponents_and_without_modification(wgs_per_cu):
    """Two more specialisations of the batch kernels (persistent, and one launch per step):
    rate exponents m = 2, n = 0.5, and a batch whose instances all have Pr = 1 (A_hat off);
    both against the single-grid path and the shortest instance against the oracle."""
    for tweak in ("exponents", "pr1"):
        s = W.batched(n_inst=6, nx_lo=20, nx_hi=700, seed=23)
        if tweak == "exponents":
            spec = W.BatchSpec(nx=s.nx, R=s.R, Pr=s.Pr, base=s.base.with_(m=2.0, n=0.5))
        else:
            R = s.R.copy()
            R[:, 7] = R[:, 4]
            R[:, 8] = R[:, 6]
            spec = W.BatchSpec(nx=s.nx, R=R, Pr=np.ones(len(s.nx)), base=s.base)
        b = _lbkm().batch_from_spec(spec)
        b.set_launch(wgs_per_cu)
        b.step(150)
        assert b.status()[1] == wgs_per_cu
        per = _split(b, _moments(b))
        k0 = int(np.argmin(spec.nx))
        _assert_parity_with_oracle(spec, k0, per[k0], 150, "batch " + tweak)
        for k in range(len(spec.nx)):
            d = _max_rel_diff(per[k], _single_grid(spec, k, 150))
            assert d <= SAME_TOL, (tweak, k, d)
