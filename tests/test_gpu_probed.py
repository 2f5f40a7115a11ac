"""GPU parity of the probed gradient (PROBED storage, awe_gradient_probed) against the oracle's
gradient_probed, through the C ABI: Rademacher probes, an on-the-fly DFT table and the identity
table (the exact gradient) on a 2D batch of uneven shots, at rel-L2 <= 1e-5; bitwise invariance
under launch shape and shot grouping; the workspace against FULL storage."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_05592_amd as A
import workloads as W
from helpers import gpu_inputs, make_plan, rel_l2, shot_kwargs

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _batch(short=False):
    # short: nt <= 64, so that the identity table (one probe per level) fits the probe limit
    wl = W.small_2d(windows=[70, 130, 96], T_per_shot=[60.0, 36.0, 48.0] if short else [160.0, 100.0, 130.0])
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 3 + i) for i, s in enumerate(wl.shots)]
    return wl, dds


def _oracle(wl, dds, C, s):
    gs = [np.zeros(wl.comp_shape(w)) for w in range(wl.nwindow)]
    for i, sh in enumerate(wl.shots):
        gs[sh.window] += O.gradient_probed(wl.m(sh.window), wl.q(i), dds[i], C=C[:, :sh.nt].astype(np.float64),
                                           s=s, **shot_kwargs(wl, i))
    return gs


def _tables(max_nt):
    return {"rademacher": W.probe_table("rademacher", max_nt, r=8, seed=21),
            "dft": W.probe_table("dft", max_nt, freqs=[0, 3, 7, 12, 20]),
            "identity": W.probe_table("identity", max_nt)}


@pytest.mark.parametrize("kind", ["rademacher", "dft", "identity"])
def test_probed_gradient_matches_the_oracle(kind):
    wl, dds = _batch(short=kind == "identity")
    max_nt = max(s.nt for s in wl.shots)
    C, s = _tables(max_nt)[kind]
    plan = make_plan(wl, storage=A.Storage(A.STORE_PROBED, C.shape[0]))
    m, q = gpu_inputs(wl, plan)
    g, v, d = plan.gradient_probed(m, q, plan.pack(dds, "d"), C, s, v=True, d=True)
    torch.cuda.synchronize()
    err = max(rel_l2(a, b) for a, b in zip(plan.unpack(g, "m"), _oracle(wl, dds, C, s)))
    print(f"probed gradient ({kind}, r = {C.shape[0]}): rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
    if kind == "identity":   # the exact gradient, and the same traces and F^T dd as FULL storage
        full = make_plan(wl, storage=A.Storage(A.STORE_FULL))
        g_f, v_f, d_f = full.gradient(m, q, full.pack(dds, "d"), v=True, d=True)
        torch.cuda.synchronize()
        assert rel_l2(g.cpu().numpy(), g_f.cpu().numpy()) <= TOL
        assert torch.equal(d, d_f) and torch.equal(v, v_f)


def test_probed_gradient_does_not_depend_on_shape_or_grouping():
    wl, dds = _batch()
    max_nt = max(s.nt for s in wl.shots)
    C, s = _tables(max_nt)["rademacher"]
    plan = make_plan(wl, storage=A.Storage(A.STORE_PROBED, C.shape[0]))
    m, q = gpu_inputs(wl, plan)
    dd = plan.pack(dds, "d")
    Cd = torch.from_numpy(C).cuda()
    ref = plan.gradient_probed(m, q, dd, Cd, s)[0]
    for tz, fusion, groups in ((8, 0, 3), (32, 3, 1), (64, 0, 2), (16, 1, 0), (24, 3, 2)):
        plan.set_tiles(tz)
        plan.set_fusion(fusion)
        plan.set_groups(groups)
        assert torch.equal(plan.gradient_probed(m, q, dd, Cd, s)[0], ref), (tz, fusion, groups)


def test_autotuner_on_a_probed_plan_keeps_the_result():
    """The autotuner times the probe kernels on a PROBED plan (their coefficients read from the
    workspace); whatever shape and fusion it keeps, the gradient is bitwise the one before."""
    wl, dds = _batch()
    max_nt = max(s.nt for s in wl.shots)
    C, s = _tables(max_nt)["rademacher"]
    plan = make_plan(wl, storage=A.Storage(A.STORE_PROBED, C.shape[0]))
    m, q = gpu_inputs(wl, plan)
    dd = plan.pack(dds, "d")
    Cd = torch.from_numpy(C).cuda()
    ref = plan.gradient_probed(m, q, dd, Cd, s)[0].clone()
    choice, ms = plan.autotune(m, q, dd, probe_steps=8)
    torch.cuda.synchronize()
    print(f"probed autotune: {choice}, {ms:.3f} ms", flush=True)
    assert ms > 0
    assert torch.equal(plan.gradient_probed(m, q, dd, Cd, s)[0], ref)


def test_probed_storage_refusals_and_workspace():
    wl, dds = _batch()
    r = 8
    full = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    plan = make_plan(wl, storage=A.Storage(A.STORE_PROBED, r))
    npts = sum(-(-sh.nx // 64) * 64 * sh.nz for sh in plan._cshots)
    assert plan.ws_bytes < full.ws_bytes and plan.ws_bytes >= 2 * r * npts * 8
    m, q = gpu_inputs(wl, plan)
    with pytest.raises(A.AweError, match="awe_gradient_probed"):
        plan.gradient(m, q, plan.pack(dds, "d"))
    with pytest.raises(A.AweError, match="not PROBED"):
        _raw_probed(full, m, q, dds)
    with pytest.raises(A.AweError):
        make_plan(wl, storage=A.Storage(A.STORE_PROBED, 65))


def _raw_probed(plan, m, q, dds):
    """awe_gradient_probed on a plan whose storage is not PROBED (the binding would refuse the
    table shape first)."""
    import ctypes
    from paper_2304_05592_amd import binding as B
    dd = plan.pack(dds, "d")
    C = torch.zeros(8 * max(s.nt for s in plan.shots), device="cuda")
    s = np.ones(8)
    g = torch.empty(plan.layout.m_size, dtype=torch.float64, device="cuda")
    ws = plan.workspace()
    B.check(B.lib().awe_gradient_probed(plan._h, B._ptr(m), B._ptr(q), B._ptr(dd), B._ptr(C),
                                        s.ctypes.data_as(ctypes.c_void_p), B._ptr(g), None, None, B._ptr(ws),
                                        plan.ws_bytes, B._stream_ptr(None)))


def test_probed_gradient_3d_matches_the_oracle():
    """3D: one shot whose receivers the post-step injection pass adds (it also adds its part of
    the probe sums A_j), 8 Rademacher probes, against the oracle; two launch shapes give the
    same bits."""
    wl = W.small_3d(n=(26, 20, 30), nbl=8, T=60.0, nrec_side=6)
    sh = wl.shots[0]
    dd = W.synthetic_residual(sh.nt, len(sh.rec), wl.dt, wl.f0, 5)
    C, s = W.probe_table("rademacher", sh.nt, r=8, seed=13)
    plan = make_plan(wl, storage=A.Storage(A.STORE_PROBED, 8))
    m, q = gpu_inputs(wl, plan)
    ddt = plan.pack([dd], "d")
    g = plan.gradient_probed(m, q, ddt, C, s)[0]
    plan.set_tiles(32, 4, 7)
    g2 = plan.gradient_probed(m, q, ddt, C, s)[0]
    torch.cuda.synchronize()
    ref = O.gradient_probed(wl.m(0), wl.q(0), dd, C=C.astype(np.float64), s=s, **shot_kwargs(wl, 0))
    err = rel_l2(plan.unpack(g, "m")[0], ref)
    print(f"probed gradient 3D (r = 8): rel-L2 {err:.3e}", flush=True)
    assert err <= TOL and torch.equal(g, g2)
