"""Hand-written adjoint of the step (through the C ABI) against reverse-mode automatic
differentiation of the FP64 oracle, and the checkpointed gradient of a whole run against
central finite differences of the GPU forward run.

Inputs of the oracle never come from the GPU: states are produced by the oracle (or the
seeded generators) and handed to the GPU with set_state.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1411_6697_amd import workloads as W
from tests.helpers import oracle_params

pytestmark = pytest.mark.gpu
NG = 27


def _lbkm():
    from paper_1411_6697_amd import lbkm
    return lbkm


def _theta(w):
    return np.array(list(w.R) + [w.Q, w.omega1, w.omega2], dtype=np.float64)


def _tables(w, theta=None, grad=False):
    P = oracle_params(w)
    tab = oracle.make_tables(P)
    if theta is not None:
        tab.R = torch.tensor(theta[:24], dtype=torch.float64)
        tab.Q = torch.tensor(theta[24], dtype=torch.float64)
        tab.omega1 = torch.tensor(theta[25], dtype=torch.float64)
        tab.omega2 = torch.tensor(theta[26], dtype=torch.float64)
    if grad:
        for t in (tab.R, tab.Q, tab.omega1, tab.omega2):
            t.requires_grad_(True)
    return P, tab


def _random_fields(nx, ny, seed):
    """Uncorrelated random fields with the reaction switched on everywhere (T > T_ig,
    0 < lambda < 1) and a non-trivial velocity in both directions."""
    g = np.random.default_rng(seed)
    return dict(rho=1.0 + 0.2 * g.random((ny, nx)), ux=0.1 * g.standard_normal((ny, nx)),
                uy=0.1 * g.standard_normal((ny, nx)), T=1.25 + 0.3 * g.random((ny, nx)),
                lam=0.05 + 0.9 * g.random((ny, nx)))


def _oracle_state(w, fields, steps):
    P, tab = _tables(w)
    F = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in fields.items()}
    f = oracle.init_f(F["rho"], F["ux"], F["uy"], F["T"], P, tab)
    f, lam = oracle.run(f, F["lam"].clone(), P, tab, steps)
    return f.detach(), lam.detach()


def _sim(w):
    L = _lbkm()
    s = L.Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.dvm, w.bc_x, w.bc_y)
    s.set_theta(_theta(w), w.gamma, w.m, w.n, w.T_ig)
    return s


def _close(a, b, tol, label):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(float(np.max(np.abs(b))), 1e-300)
    err = float(np.max(np.abs(a - b))) / scale
    print(label, f"max|diff|/max|ref| = {err:.2e}", flush=True)
    assert err <= tol, (label, err)


def _param_close(g, ref, tol, label):
    """Per-parameter relative error, with entries far below the largest measured against
    1e-6 of the largest (R_1..R_4 have zero gradient by construction)."""
    g = np.asarray(g)
    ref = np.asarray(ref)
    floor = 1e-6 * float(np.max(np.abs(ref)))
    err = np.abs(g - ref) / np.maximum(np.abs(ref), floor)
    print(label, "worst", f"{float(np.max(err)):.2e}", "at", int(np.argmax(err)), flush=True)
    assert float(np.max(err)) <= tol, (label, err)


CASES = [  # nx, ny, bc_x, bc_y
    (40, 6, "outflow", "periodic"), (9, 7, "periodic", "outflow"), (1, 4, "outflow", "periodic"),
    (2, 3, "periodic", "periodic"), (3, 1, "outflow", "outflow"), (5, 2, "outflow", "outflow"),
    # rows wide enough for waves whose x-stencils come from neighbouring lanes (interior
    # waves of a 256-wide work-group), beside waves at the row ends that gather them
    (300, 3, "outflow", "periodic"), (200, 2, "periodic", "outflow")]


@pytest.mark.parametrize("nx,ny,bcx,bcy,mn", [c + ((1.0, 1.0),) for c in CASES] +
                         [(12, 5, "outflow", "periodic", (2.0, 0.5))])
def test_one_adjoint_step_equals_oracle_vector_jacobian_product(nx, ny, bcx, bcy, mn):
    w = W.adjoint_strip(nx=nx, ny=ny).with_(bc_x=bcx, bc_y=bcy, m=mn[0], n=mn[1])
    f, lam = _oracle_state(w, _random_fields(nx, ny, 100 + nx), steps=3)
    g = np.random.default_rng(7 + ny)
    af = torch.from_numpy(g.standard_normal((24, ny, nx)))
    al = torch.from_numpy(g.standard_normal((ny, nx)))

    P, tab = _tables(w, grad=True)
    fx = f.clone().requires_grad_(True)
    lx = lam.clone().requires_grad_(True)
    f1, l1 = oracle.step(fx, lx, P, tab)
    ref = torch.autograd.grad((f1, l1), (fx, lx, tab.R, tab.Q, tab.omega1, tab.omega2),
                              grad_outputs=(af, al), allow_unused=True)
    ref = [torch.zeros(()) if r is None else r for r in ref]
    ref_theta = np.concatenate([ref[2].numpy(), [float(ref[3]), float(ref[4]), float(ref[5])]])

    s = _sim(w)
    dev = s.device
    grad = torch.zeros(NG, dtype=torch.float64, device=dev)
    af_n, al_n = s.adjoint_step(f.to(dev).contiguous(), lam.to(dev).contiguous(), af.to(dev), al.to(dev), grad)
    torch.cuda.synchronize()
    label = f"{nx}x{ny} {bcx}/{bcy}"
    _close(af_n.cpu().numpy(), ref[0].numpy(), 1e-11, label + " d/df")
    _close(al_n.cpu().numpy(), ref[1].numpy(), 1e-11, label + " d/dlambda")
    _param_close(grad.cpu().numpy(), ref_theta, 1e-9, label + " d/dtheta")


def test_adjoint_step_refuses_srt_and_runge_kutta():
    """The adjoint covers the MRT form of Eq. Boltzmann_chemical under forward Euler only: a
    context switched to the single-relaxation-time form or to a Runge-Kutta scheme refuses
    an adjoint step (ESTATE), and accepts it again once switched back."""
    w = W.adjoint_strip(nx=8, ny=3)
    f, lam = _oracle_state(w, _random_fields(8, 3, 11), steps=1)
    s = _sim(w)
    dev = s.device
    args = (f.to(dev).contiguous(), lam.to(dev).contiguous(), torch.ones(24, 3, 8, dtype=torch.float64, device=dev),
            torch.ones(3, 8, dtype=torch.float64, device=dev))
    s.set_srt(1e-2)
    with pytest.raises(_lbkm().LbkmError, match="MRT"):
        s.adjoint_step(*args, torch.zeros(NG, dtype=torch.float64, device=dev))
    s.set_srt(0.0)
    s.set_time_scheme(3)
    with pytest.raises(_lbkm().LbkmError, match="Euler"):
        s.adjoint_step(*args, torch.zeros(NG, dtype=torch.float64, device=dev))
    s.set_time_scheme(1)
    s.adjoint_step(*args, torch.zeros(NG, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()


def test_tne_loss_and_its_gradient_match_oracle():
    w = W.adjoint_strip(nx=24, ny=5)
    f, lam = _oracle_state(w, _random_fields(24, 5, 3), steps=4)
    P, tab = _tables(w)
    fx = f.clone().requires_grad_(True)
    delta, _ = oracle.tne(fx, P, tab)
    L = (delta * delta).sum()
    (gref,) = torch.autograd.grad(L, (fx,))
    s = _sim(w)
    loss, g = s.tne_loss(f.to(s.device).contiguous())
    torch.cuda.synchronize()
    assert abs(float(loss) - float(L)) <= 1e-12 * abs(float(L)), (float(loss), float(L))
    _close(g.cpu().numpy(), gref.numpy(), 1e-11, "dL/df")


def test_adjoint_init_matches_oracle():
    w = W.adjoint_strip(nx=17, ny=3)
    F = _random_fields(17, 3, 5)
    t = {k: torch.from_numpy(F[k]).clone().requires_grad_(True) for k in ("rho", "ux", "uy", "T")}
    P, tab = _tables(w)
    f0 = oracle.init_f(t["rho"], t["ux"], t["uy"], t["T"], P, tab)
    af = torch.from_numpy(np.random.default_rng(9).standard_normal((24, 3, 17)))
    ref = torch.autograd.grad(f0, [t[k] for k in ("rho", "ux", "uy", "T")], grad_outputs=af)
    s = _sim(w)
    out = s.adjoint_init(F["rho"], F["ux"], F["uy"], F["T"], af.to(s.device))
    torch.cuda.synchronize()
    for k, a, b in zip(("rho", "ux", "uy", "T"), out, ref):
        _close(a.cpu().numpy(), b.numpy(), 1e-12, "d/d" + k)


def _oracle_run_gradient(w, steps, fields=None):
    th = _theta(w)
    P, tab = _tables(w, th, grad=True)
    F = {k: torch.from_numpy(np.ascontiguousarray(v)).clone().requires_grad_(True)
         for k, v in (fields or w.fields()).items()}
    f = oracle.init_f(F["rho"], F["ux"], F["uy"], F["T"], P, tab)
    f, lam = oracle.run(f, F["lam"], P, tab, steps)
    delta, _ = oracle.tne(f, P, tab)
    L = (delta * delta).sum()
    L.backward()
    gth = np.concatenate([tab.R.grad.numpy(), [float(tab.Q.grad), float(tab.omega1.grad),
                                                 float(tab.omega2.grad)]])
    return float(L), gth, {k: F[k].grad.numpy() for k in F}


def _gpu_run_gradient(w, steps, every, fields=None):
    L_ = _lbkm()
    s = L_.Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.dvm, w.bc_x, w.bc_y)
    F = fields or w.fields()
    theta = torch.tensor(_theta(w), dtype=torch.float64, requires_grad=True)
    ts = {k: torch.tensor(F[k], dtype=torch.float64, device=s.device, requires_grad=True)
          for k in ("rho", "ux", "uy", "T", "lam")}
    fN, lN = L_.LBKMRun.apply(theta, ts["rho"], ts["ux"], ts["uy"], ts["T"], ts["lam"], s, steps,
                              w.gamma, every, w.m, w.n, w.T_ig)
    loss = L_.TNELoss.apply(fN, s)
    loss.backward()
    torch.cuda.synchronize()
    return s, float(loss), theta.grad.numpy(), {k: v.grad.cpu().numpy() for k, v in ts.items()}


def test_checkpointed_run_gradient_matches_oracle_autograd():
    """30 steps of a 40 x 8 strip (front, ignition, reaction, A_hat active), checkpoints
    every 7 steps (a ragged last segment).  Besides the strip's u_y noise the initial u_x
    carries noise of the same size, so that no upwind decision of lambda is taken on a
    velocity that is zero up to rounding (see the next test)."""
    w = W.adjoint_strip(nx=40, ny=8, steps=30)
    F = w.fields()
    F["ux"] = F["ux"] + 1e-3 * np.random.default_rng(41).standard_normal(F["ux"].shape)
    L0, gth0, gf0 = _oracle_run_gradient(w, 30, F)
    _, L1, gth1, gf1 = _gpu_run_gradient(w, 30, 7, F)
    print("loss", L1, "oracle", L0, flush=True)
    assert abs(L1 - L0) <= 1e-11 * abs(L0)
    _param_close(gth1, gth0, 1e-8, "d/dtheta")
    for k in ("rho", "ux", "uy", "T", "lam"):
        _close(gf1[k], gf0[k], 1e-8, "d/d" + k)


def test_strip_gradient_agrees_away_from_rounding_level_upwind_decisions():
    """The strip itself starts with u_x = 0 exactly, so the first step decides the upwind
    side of lambda on u_x values that are rounding noise (about 1e-17, of either sign, and
    different in the two implementations).  Where lambda varies across such a cell, the
    two one-sided derivatives with respect to u_x and lambda there differ; both are exact
    on their branch.  Everything else is unique and is compared: the parameter gradient,
    the gradients with respect to rho, u_y and T everywhere, and those with respect to u_x
    and lambda outside these cells and their NND stencils (the cells are found from the
    oracle's initial state)."""
    w = W.adjoint_strip(nx=40, ny=8, steps=30)
    F = w.fields()
    L0, gth0, gf0 = _oracle_run_gradient(w, 30, F)
    _, L1, gth1, gf1 = _gpu_run_gradient(w, 30, 7, F)
    assert abs(L1 - L0) <= 1e-11 * abs(L0)
    _param_close(gth1, gth0, 1e-8, "d/dtheta")
    for k in ("rho", "uy", "T"):
        _close(gf1[k], gf0[k], 1e-8, "d/d" + k)
    P, tab = _tables(w)
    Ft = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in F.items()}
    m = oracle.moments(oracle.init_f(Ft["rho"], Ft["ux"], Ft["uy"], Ft["T"], P, tab), Ft["lam"], P, tab)
    lam = F["lam"]
    cols = np.arange(w.nx)
    shifted = lambda a, d: a[:, np.clip(cols + d, 0, w.nx - 1)]      # outflow rule in x
    lam_varies = np.zeros_like(lam, dtype=bool)
    for d in (-2, -1, 1, 2):
        lam_varies |= shifted(lam, d) != lam
    tie = (np.abs(m["ux"].numpy()) < 1e-12) & lam_varies
    assert tie.any()          # the case this test is about is present
    near = np.zeros_like(tie)
    for d in range(-2, 3):
        near |= shifted(tie, d)
    print("cells with a rounding-level upwind decision:", np.argwhere(tie).tolist(), flush=True)
    for k in ("ux", "lam"):
        a, b = gf1[k].copy(), gf0[k].copy()
        a[near] = 0.0
        b[near] = 0.0
        _close(a, b, 1e-8, "d/d" + k + " (away from those cells)")


def _loss_at(s, w, theta, F):
    L_ = _lbkm()
    s.set_theta(theta, w.gamma, w.m, w.n, w.T_ig)
    s.init_fields(F["rho"], F["ux"], F["uy"], F["T"], F["lam"])
    s.step(w.steps)
    f, _ = s.get_state()
    loss, _ = s.tne_loss(f, grad=False)
    return float(loss)


def test_full_size_gradient_matches_central_differences():
    """The 2048 x 256 strip, 500 steps, checkpoints every 50: d L / d theta_k against
    central differences of the GPU forward run, (L(theta + h theta_k e_k) -
    L(theta - h theta_k e_k)) / (2 h theta_k) for h = 1e-5 ... 1e-8 (printed).  The bar,
    relative error <= 1e-5, applies at h = 1e-6 for R_9, R_21, Q, omega_1 and omega_2 (about
    5e-8 there) and at h = 1e-7 for R_5 and R_8 (1.6e-5 and 1.5e-5 at h = 1e-6, 3e-6 at
    h = 1e-7): with u_y noise of 1e-3 the planes with v_iy = 0 vary only at the 1e-6 scale,
    and a relative change of R_5 or R_8 above about 1e-6 moves minmod selections across
    their switch points, where the discrete map has kinks (the finite differences converge
    to the adjoint value as h decreases)."""
    w = W.adjoint_strip()
    s, L, gth, _ = _gpu_run_gradient(w, w.steps, 50)
    assert np.isfinite(L) and L > 0
    F = w.fields()
    th = _theta(w)
    for k in (4, 7, 8, 20, 24, 25, 26):     # R_5, R_8, R_9, R_21, Q, omega_1, omega_2
        rel = {}
        for h in (1e-5, 1e-6, 1e-7, 1e-8):
            tp, tm = th.copy(), th.copy()
            tp[k] += h * th[k]
            tm[k] -= h * th[k]
            fd = (_loss_at(s, w, tp, F) - _loss_at(s, w, tm, F)) / (2 * h * th[k])
            rel[h] = abs(fd - gth[k]) / abs(gth[k])
        print("theta", k, "adjoint", gth[k], {h: f"{v:.1e}" for h, v in rel.items()}, flush=True)
        assert rel[1e-7 if k in (4, 7) else 1e-6] <= 1e-5, (k, gth[k], rel)


def _loss_from_fields(s, w, F):
    s.set_theta(_theta(w), w.gamma, w.m, w.n, w.T_ig)
    s.init_fields(F["rho"], F["ux"], F["uy"], F["T"], F["lam"])
    s.step(w.steps)
    f, _ = s.get_state()
    loss, _ = s.tne_loss(f, grad=False)
    return float(loss)


def test_full_size_initial_field_gradients_match_central_differences():
    """The 2048 x 256 strip, 500 steps, checkpoints every 50: the gradient with respect to the
    initial rho, u_x, u_y, T and lambda (through the adjoint of the initialisation
    f = M^-1 f_hat^eq), sum(dL/dF * delta) along a direction delta per field, against central
    differences (L(F + h delta) - L(F - h delta)) / (2 h) of the GPU forward run for
    h = 1e-6, 1e-7, 1e-8 (printed).

    The strip's white u_y noise leaves neighbouring differences of the distributions at 1e-6
    of their size or less away from the front, and the initial lambda is exactly 0 or 1, so a
    perturbation of those cells moves minmod selections (and the ignition gate) across their
    switch points at any usable h: for a random relative rho perturbation the finite
    differences miss by 3e-2, 8e-3, 2e-3 at h = 1e-6, 1e-7, 1e-8.  The directions are
    therefore:
      rho scaled uniformly (minmod is homogeneous of degree one, so only the pressure
        dependence of the reaction rate moves the state off that scaling): 1e-5 at h = 1e-6;
      u_y's noise scaled by a bump at the front (x = 200 cells, width 4; y-differences scale
        alike in a column): 1e-5 at h = 1e-6;
      rho, T and u_x bumps at the front: the differences converge to the adjoint value as h
        shrinks (the kinks they cross become fewer), 1e-5 at h = 1e-8 (rho, T) and 5e-5
        (u_x);
      lambda on the unburnt cells at the front: converging, 5e-4 at h = 1e-8.
    The initial-field gradients are matched to the oracle's reverse-mode derivative at 1e-8
    on a reduced strip (test_checkpointed_run_gradient_matches_oracle_autograd)."""
    w = W.adjoint_strip()
    F = w.fields()
    s, L, _, gf = _gpu_run_gradient(w, w.steps, 50, F)
    x = np.arange(w.nx)[None, :] * np.ones((w.ny, 1))
    bump = lambda c, sig: np.exp(-((x - c) / sig) ** 2)
    dirs = {"rho": F["rho"],
            "rho_front": F["rho"] * bump(200.0, 4.0),
            "T": F["T"] * bump(200.0, 4.0),
            "ux": 0.5 * bump(200.0, 4.0),
            "uy": F["uy"] * bump(200.0, 4.0),
            "lam": np.where(F["lam"] < 0.5, bump(202.0, 3.0), 0.0)}
    for name, d in dirs.items():
        k = name.split("_")[0]
        want = float(np.sum(gf[k] * d))
        rel = {}
        for h in (1e-6, 1e-7, 1e-8):
            Fp, Fm = dict(F), dict(F)
            Fp[k] = F[k] + h * d
            Fm[k] = F[k] - h * d
            fd = (_loss_from_fields(s, w, Fp) - _loss_from_fields(s, w, Fm)) / (2 * h)
            rel[h] = abs(fd - want) / abs(want)
        print("d/d" + name, "adjoint", want, {h: f"{v:.1e}" for h, v in rel.items()}, flush=True)
        bar = {"rho": (1e-6, 1e-5), "uy": (1e-6, 1e-5), "rho_front": (1e-8, 1e-5), "T": (1e-8, 1e-5),
               "ux": (1e-8, 5e-5), "lam": (1e-8, 5e-4)}[name]
        assert rel[bar[0]] <= bar[1], (name, want, rel)
        if bar[0] == 1e-8:
            assert rel[1e-8] < rel[1e-7] < rel[1e-6], (name, rel)     # converging as h shrinks
