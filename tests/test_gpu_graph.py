"""A whole gradient step (forward with storage, residual, reverse sweep) captured in a HIP
graph and replayed: every replay, with eager work and synchronisations in between, must
reproduce the eager result bitwise (the library records no memset nodes: it clears memory
with its own fill kernel)."""
import numpy as np
import pytest
import torch

import paper_2304_05592_amd as A
import workloads as W
from helpers import gpu_inputs, make_plan

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", [A.Storage(A.STORE_FULL), A.Storage(A.STORE_CHECKPOINT, 3),
                                     A.Storage(A.STORE_FULL, 0, A.PREC_BF16)])
def test_graph_replays_match_eager(storage):
    wl = W.small_2d(nshot=2)
    plan = make_plan(wl, storage=storage)
    m, q = gpu_inputs(wl, plan, background=True)
    m_true, _ = gpu_inputs(wl, plan)
    ws = plan.workspace()
    d_obs = plan.forward(m_true, q, ws=ws)
    d = torch.empty_like(d_obs)
    r = torch.empty_like(d_obs)
    g = torch.empty(plan.layout.m_size, dtype=torch.float64, device="cuda")

    def step():
        plan.forward(m, q, d=d, keep=True, ws=ws)
        _, loss = A.residual(d, d_obs, r=r)
        plan.backward(m, q, r, g=g, v=None, ws=ws)
        return loss

    loss = step()
    torch.cuda.synchronize()
    g_ref, loss_ref = g.clone(), loss.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        loss_g = step()
    torch.cuda.synchronize()
    for it in range(3):
        g.zero_()
        d.zero_()
        _ = plan.forward(m_true, q, ws=plan.workspace())   # unrelated eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), it
        assert torch.equal(loss_g, loss_ref), it
