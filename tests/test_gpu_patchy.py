"""Patchy-saturation rock physics R ("Putting it all together") on the GPU against the oracle.

The forward kernel evaluates R in FP64 and rounds once, so it must agree with the oracle's
FP64 values rounded to float32 to within one float32 unit; the pullback kernel (analytic
derivative) must agree with the oracle's complex-step pullback to float32 rounding.  The
composition sw -> R -> m = 1/v^2 -> F of a small time-lapse survey is checked end to end
against the oracle chain (rel-L2 <= 1e-5)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_05592_amd as A
import workloads as W
from helpers import make_plan, oracle_gradient, rel_l2

pytestmark = pytest.mark.gpu
ULP = 2.0 ** -23


def _inputs(shape, seed):
    """Seeded rock and saturation; 1-D sizes are cut from a longer draw (a field of a handful
    of cells has no spread to normalise)."""
    gen = (max(shape[0], 4096),) if len(shape) == 1 else shape
    vp, rho, phi = W.reservoir_rock(gen, seed)
    sw = W.saturation_field(gen, seed + 1)
    return tuple(a[:shape[0]] if len(shape) == 1 else a for a in (sw, vp, rho, phi))


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a).ravel()).cuda() for a in arrs]


def _check_forward(sw, vp, rho, phi, consts=None):
    tsw, tvp, trho, tphi = _dev(sw, vp, rho, phi)
    vp_new, rho_new = A.patchy(tsw, tvp, trho, tphi, consts=consts)
    torch.cuda.synchronize()
    ref_v, ref_r = O.patchy(sw.ravel(), vp.ravel(), rho.ravel(), phi.ravel(), consts)
    for got, ref, name in ((vp_new, ref_v, "vp_new"), (rho_new, ref_r, "rho_new")):
        g = got.cpu().numpy().astype(np.float64)
        rel = np.abs(g - ref) / np.abs(ref)
        print(f"patchy {name} n={sw.size}: max rel {rel.max():.2e}", flush=True)
        assert rel.max() <= ULP, name
    return vp_new, rho_new


@pytest.mark.parametrize("n", [1, 63, 64, 257, 100003])
def test_patchy_forward_matches_the_oracle(n):
    sw, vp, rho, phi = _inputs((n,), 11)
    _check_forward(sw, vp, rho, phi)


def test_patchy_forward_with_other_constants_and_empty_input():
    sw, vp, rho, phi = _inputs((37, 53), 12)
    consts = dict(O.PATCHY_CONSTANTS, k_co2=0.3e9, rho_co2=600.0, k_min=38.0e9)
    _check_forward(sw, vp, rho, phi, consts)
    e = torch.empty(0, device="cuda", dtype=torch.float32)
    v, r = A.patchy(e, e, e, e)
    g = A.patchy_vjp(e, e, e, e, e)
    torch.cuda.synchronize()
    assert v.numel() == r.numel() == g.numel() == 0


def test_zero_saturation_returns_the_brine_rock():
    _, vp, rho, phi = _inputs((4099,), 13)
    sw = np.zeros_like(vp)
    vp_new, rho_new = _check_forward(sw, vp, rho, phi)
    assert np.array_equal(rho_new.cpu().numpy(), rho)
    d = np.abs(vp_new.cpu().numpy().astype(np.float64) - vp) / vp
    assert d.max() <= ULP


@pytest.mark.parametrize("with_rho", [False, True])
def test_patchy_pullback_matches_the_oracle(with_rho):
    shape = (301, 517)                       # ragged against any block size
    sw, vp, rho, phi = _inputs(shape, 14)
    rng = np.random.default_rng(3)
    g_vp = rng.standard_normal(shape).astype(np.float32)
    g_rho = rng.standard_normal(shape).astype(np.float32) * 1e-3 if with_rho else None
    t = _dev(sw, vp, rho, phi, g_vp)
    tg_rho = _dev(g_rho)[0] if with_rho else None
    g = A.patchy_vjp(*t, g_rho=tg_rho)
    torch.cuda.synchronize()
    ref = O.patchy_vjp(sw, vp, rho, phi, g_vp, g_rho).ravel()
    # scale: the sum of the magnitudes of the two terms (they can cancel)
    scale = np.abs(O.patchy_vjp(sw, vp, rho, phi, np.abs(g_vp))).ravel()
    if with_rho:
        scale += np.abs(O.patchy_vjp(sw, vp, rho, phi, np.zeros_like(g_vp), np.abs(g_rho))).ravel()
    err = np.abs(g.cpu().numpy().astype(np.float64) - ref) / scale
    print(f"patchy pullback (g_rho {with_rho}): max scaled err {err.max():.2e}", flush=True)
    assert err.max() <= 2 * ULP


def _survey():
    return W.timelapse_survey(nx=96, nz=64, h=10.0, T=320.0, nvint=3, nsrc=5, nrec=40,
                              shots_per_vintage=2, nbl=12, iteration=4)


def test_saturation_gradient_through_rock_physics_matches_the_oracle():
    """g_sw of <F(m(R(sw))) q, dd> for a 3-vintage survey: R, m = 1/v^2, the batched wave
    pullback and the two chain rules, against the oracle's FP64 chain."""
    wl = _survey()
    shape = wl.comp_shape(0)
    vp, rho, phi = W.reservoir_rock(shape, 21)
    sws = [(0.8 * W.extend_edge(W.plume_mask(wl.v[0].shape, wl.h, i + 1, wl.nwindow), wl.nbl))
           .astype(np.float32) for i in range(wl.nwindow)]
    assert float(vp.max()) <= wl.vmax
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 60 + i) for i, s in enumerate(wl.shots)]
    plan = make_plan(wl, A.Storage(A.STORE_FULL))
    sw = plan.pack(sws, "m").requires_grad_(True)
    tvp, trho, tphi = (plan.pack([a] * wl.nwindow, "m") for a in (vp, rho, phi))
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    dd = plan.pack(dds, "d")
    v_new, _ = A.patchy_rock_physics(sw, tvp, trho, tphi)
    d = A.wave_forward(A.slowness2_from_velocity(v_new), q, plan)
    (d * dd).sum().backward()
    torch.cuda.synchronize()
    got = plan.unpack(sw.grad, "m")
    v_o = [O.patchy(sws[w], vp, rho, phi)[0] for w in range(wl.nwindow)]
    g_m = oracle_gradient(wl, dds, ms=[O.slowness2(v) for v in v_o])
    ref = [O.patchy_vjp(sws[w], vp, rho, phi, O.velocity_gradient(v_o[w], g_m[w]))
           for w in range(wl.nwindow)]
    err = rel_l2(got, ref)
    print(f"saturation gradient through R ({wl.nwindow} vintages, {wl.nshot} shots): rel-L2 {err:.3e}",
          flush=True)
    assert err <= 1e-5


def test_rock_kernels_at_the_benchmark_sizes():
    """The two sizes the benchmark times: all vintages of the 15-vintage crosswell workload
    (every output compared) and 2^28 cells (grid-stride path; 200k sampled outputs compared)."""
    wl = W.make_config("c7_timelapse_rock")
    ext = lambda a: W.extend_edge(np.asarray(a, dtype=np.float32), wl.nbl)
    plan = make_plan(wl, A.Storage(A.STORE_NONE))
    vp, rho, phi = (ext(wl.extra[k]) for k in ("vp", "rho", "phi"))
    sws = [ext(a) for a in wl.extra["sat"]]
    tvp, trho, tphi = (plan.pack([a] * wl.nwindow, "m") for a in (vp, rho, phi))
    tsw = plan.pack(sws, "m")
    v_new, r_new = A.patchy(tsw, tvp, trho, tphi)
    g = A.patchy_vjp(tsw, tvp, trho, tphi, torch.ones_like(tvp))
    torch.cuda.synchronize()
    got_v, got_r, got_g = (plan.unpack(t, "m") for t in (v_new, r_new, g))
    for w in range(wl.nwindow):
        ref_v, ref_r = O.patchy(sws[w], vp, rho, phi)
        assert np.max(np.abs(got_v[w] - ref_v) / ref_v) <= ULP
        assert np.max(np.abs(got_r[w] - ref_r) / ref_r) <= ULP
        ref_g = O.patchy_vjp(sws[w], vp, rho, phi, np.ones_like(vp))
        assert np.max(np.abs(got_g[w] - ref_g) / np.abs(ref_g)) <= 2 * ULP
    del plan, tvp, trho, tphi, tsw, v_new, r_new, g
    # 2^28 cells built as in the benchmark: a 4096-cell pattern repeated
    n, side = 1 << 28, 4096
    base = [*W.reservoir_rock((side,), 7)]
    base.insert(0, W.saturation_field((side,), 8))
    tsw, tvp, trho, tphi = (torch.from_numpy(a.ravel()).cuda().repeat(n // side) for a in base)
    v_new, r_new = A.patchy(tsw, tvp, trho, tphi)
    g = A.patchy_vjp(tsw, tvp, trho, tphi, torch.ones_like(tvp))
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(5).choice(n, 200_000, replace=False))
    ti = torch.from_numpy(idx).cuda()
    got_v, got_r, got_g = (t[ti].cpu().numpy().astype(np.float64) for t in (v_new, r_new, g))
    sw, vp, rho, phi = (a.ravel()[idx % side] for a in base)
    ref_v, ref_r = O.patchy(sw, vp, rho, phi)
    ref_g = O.patchy_vjp(sw, vp, rho, phi, np.ones_like(vp))
    assert np.max(np.abs(got_v - ref_v) / ref_v) <= ULP
    assert np.max(np.abs(got_r - ref_r) / ref_r) <= ULP
    assert np.max(np.abs(got_g - ref_g) / np.abs(ref_g)) <= 2 * ULP
    print(f"rock kernels: c7 size {wl.nwindow} vintages and 2^28 cells (sampled) agree", flush=True)
