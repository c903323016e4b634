"""The allocation-free TNE loss (lbkm_tne_loss_noalloc) against lbkm_tne_loss.

Both run the same kernels; the allocation-free entry point keeps its per-work-group
partial sums in a fixed device array instead of the context's adjoint scratch, so the
loss and its gradient must agree bitwise.  Two calls in a row on different contexts, the
second on a smaller grid (the array keeps the first call's partial sums), and the size
limit of the array.
"""

import pytest
import torch

from paper_1411_6697_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lbkm():
    from paper_1411_6697_amd import lbkm
    return lbkm


def test_noalloc_loss_equals_tne_loss_on_two_calls_second_smaller():
    lbkm = _lbkm()
    for w in (W.adjoint_strip(nx=700, ny=40, steps=25), W.adjoint_strip(nx=130, ny=7, steps=25)):
        s = lbkm.sim_from_workload(w)
        s.step(w.steps)
        f, _ = s.get_state()
        loss = torch.full((1,), float("nan"), dtype=torch.float64, device=f.device)
        grad = torch.full_like(f, float("nan"))
        loss_only = torch.full((1,), float("nan"), dtype=torch.float64, device=f.device)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        s.tne_loss_into(f, loss, grad)          # first: the context has no adjoint scratch yet
        s.tne_loss_into(f, loss_only, None)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        # the adjoint scratch that lbkm_tne_loss allocates here is 10 planes (>= 0.5 MiB)
        assert free0 - free1 < (1 << 19), (free0, free1)
        ref_loss, ref_grad = s.tne_loss(f, grad=True)
        torch.cuda.synchronize()
        print(w.nx, w.ny, "loss", loss.item(), ref_loss.item(), flush=True)
        assert torch.isfinite(loss).all() and loss.item() > 0.0
        assert torch.equal(loss, ref_loss.reshape(1))
        assert torch.equal(loss_only, ref_loss.reshape(1))
        assert torch.equal(grad, ref_grad)
        s.close()


def test_noalloc_loss_refuses_grids_beyond_its_array():
    """ceil(nx/256) * ny partial sums must fit the 65536 of the fixed array: 1 x 65537 does
    not, and the call returns EINVAL before launching anything."""
    lbkm = _lbkm()
    s = lbkm.Sim(1, 65537, 1e-4, 1e-4, 1e-6, W.DVM_UNSTEADY_DET, bc_x="outflow", bc_y="periodic")
    s.set_params(W.rates(100.0), 1.4)
    f = torch.zeros((24, 65537, 1), dtype=torch.float64, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    st = s.lib.lbkm_tne_loss_noalloc(s.h, lbkm._ptr(f), lbkm._ptr(loss), None)
    assert st == -1
    assert "65536" in s.lib.lbkm_last_error(s.h).decode()
    s.close()
