"""Time-lapse batched gradient with the wavespeed parameterisation (the block-diagonal operator
diag(F^i(v^i) q^i) of "Putting it all together"): every vintage is a model window, a few shots
per vintage run in one plan, and the gradient with respect to each vintage's wavespeed is
checked against the oracle (rel-L2 <= 1e-5)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_05592_amd as A
import workloads as W
from helpers import make_plan, oracle_gradient, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _survey():
    return W.timelapse_survey(nx=96, nz=64, h=10.0, T=320.0, nvint=3, nsrc=5, nrec=40,
                              shots_per_vintage=2, nbl=12, iteration=3)


@pytest.mark.parametrize("groups", [0, 3])
def test_timelapse_velocity_gradient_matches_the_oracle(groups):
    wl = _survey()
    v32 = [W.extend_edge(wl.v0[w].astype(np.float32), wl.nbl) for w in range(wl.nwindow)]
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 40 + i) for i, s in enumerate(wl.shots)]
    plan = make_plan(wl, A.Storage(A.STORE_FULL))
    plan.set_groups(groups)
    v = plan.pack(v32, "m").requires_grad_(True)
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    dd = plan.pack(dds, "d")
    d = A.wave_forward(A.slowness2_from_velocity(v), q, plan)
    (d * dd).sum().backward()          # pullback of dd: J^T dd, then the chain rule of m = 1/v^2
    torch.cuda.synchronize()
    got = plan.unpack(v.grad, "m")
    ms = [O.slowness2(v32[w]) for w in range(wl.nwindow)]
    g_m = oracle_gradient(wl, dds, ms=ms)
    ref = [O.velocity_gradient(v32[w], g_m[w]) for w in range(wl.nwindow)]
    err = rel_l2(got, ref)
    print(f"time-lapse velocity gradient ({wl.nwindow} vintages, {wl.nshot} shots, groups {groups}): "
          f"rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
    # vintages differ only inside the plume: their gradients are not all equal
    assert rel_l2(got[0], got[-1]) > 1e-3


def test_slowness_kernels_match_their_definitions():
    x = torch.linspace(1.4, 4.6, 10001, device="cuda", dtype=torch.float32)
    m = A.slowness2(x)
    g = torch.randn(10001, device="cuda", dtype=torch.float32)
    gv = A.velocity_gradient(x, g)
    torch.cuda.synchronize()
    xd = x.cpu().numpy()
    assert np.array_equal(m.cpu().numpy(), O.slowness2(xd).astype(np.float32))
    np.testing.assert_allclose(gv.cpu().numpy(), O.velocity_gradient(xd, g.cpu().numpy()), rtol=2e-7, atol=0)
