"""The wave operator as a torch.autograd.Function (the paper's rrule for F*q): gradients of a
misfit with respect to the squared slowness and to the source, against the oracle and
against central finite differences of the GPU misfit itself."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_05592_amd as A
import workloads as W
from helpers import make_plan, oracle_adjoint, oracle_forward, oracle_gradient, rel_l2

pytestmark = pytest.mark.gpu


def _setup(storage):
    wl = W.small_2d(nshot=2)
    plan = make_plan(wl, storage=storage)
    # 0.3 x the oracle data of the true model: the residual does not cancel, so the forward's
    # rounding is not amplified in it and the 1e-5 bar applies to the whole pullback
    d_obs = plan.pack([0.3 * d for d in oracle_forward(wl)], "d")
    m0 = plan.pack([wl.m(0, background=True)], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    return wl, plan, d_obs, m0, q


@pytest.mark.parametrize("storage", [A.Storage(A.STORE_FULL), A.Storage(A.STORE_CHECKPOINT, 4)])
def test_autograd_gradients_match_the_oracle(storage):
    wl, plan, d_obs, m0, q = _setup(storage)
    m = m0.clone().requires_grad_(True)
    qq = q.clone().requires_grad_(True)
    d = A.wave_forward(m, qq, plan)
    loss = 0.5 * ((d - d_obs) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    ms = [wl.m(0, background=True)]
    dds = [(a - b).astype(np.float32) for a, b in zip(oracle_forward(wl, ms=ms), plan.unpack(d_obs, "d"))]
    e_m = rel_l2(plan.unpack(m.grad, "m"), oracle_gradient(wl, dds, ms=ms))
    e_q = rel_l2(plan.unpack(qq.grad, "q"), oracle_adjoint(wl, dds, ms=ms))
    print(f"autograd dphi/dm rel-L2 {e_m:.3e}, dphi/dq rel-L2 {e_q:.3e}", flush=True)
    assert e_m <= 1e-5 and e_q <= 1e-5


def test_autograd_gradient_against_finite_differences():
    """Central differences of the GPU misfit on 8 smooth random directions; eps = 1e-2 of the
    model scale.  FP32 misfit noise limits the agreement to ~1e-3 (gate 1e-2)."""
    wl, plan, d_obs, m0, q = _setup(A.Storage(A.STORE_CHECKPOINT, 4))
    m = m0.clone().requires_grad_(True)
    d = A.wave_forward(m, q, plan)
    loss = 0.5 * ((d.double() - d_obs.double()) ** 2).sum()
    loss.backward()
    g = m.grad.double()

    def phi(mm):
        dd = plan.forward(mm, q)
        return 0.5 * ((dd.double() - d_obs.double()) ** 2).sum().item()

    errs = []
    for k in range(8):
        dm = plan.pack([W.random_field(wl.comp_shape(0), 100 + k, smooth_cells=3.0)], "m")
        eps = 1e-2 * m0.abs().max().item() / dm.abs().max().item()
        fd = (phi(m0 + eps * dm) - phi(m0 - eps * dm)) / (2 * eps)
        ad = torch.dot(g, dm.double()).item()
        errs.append(abs(fd - ad) / abs(fd))
    print("finite-difference relative errors:", ", ".join(f"{e:.2e}" for e in errs), flush=True)
    assert max(errs) <= 1e-2


def test_physical_grid_parameterisation_folds_the_border():
    """extend_edge's backward is the adjoint of edge replication: d phi / d m_phys = E^T g."""
    wl, plan, d_obs, m0, q = _setup(A.Storage(A.STORE_FULL))
    nbl = wl.nbl
    m_phys = m0.view(wl.comp_shape(0))[nbl:-nbl, nbl:-nbl].clone().requires_grad_(True)
    m = A.extend_edge(m_phys, nbl).reshape(-1)
    d = A.wave_forward(m, q, plan)
    (0.5 * ((d - d_obs) ** 2).sum()).backward()
    mc = m0.clone().requires_grad_(True)
    d2 = A.wave_forward(mc, q, plan)
    (0.5 * ((d2 - d_obs) ** 2).sum()).backward()
    folded = O.fold_edge(mc.grad.view(wl.comp_shape(0)).double().cpu().numpy(), nbl)
    assert rel_l2(m_phys.grad.double().cpu().numpy(), folded) <= 1e-6
