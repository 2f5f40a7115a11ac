"""The full-size fixtures are what the oracle computes today on the seeded inputs.

The scheme is causal: a forward run truncated to its first n time samples
reproduces the first n samples of the full run exactly.  Re-running the oracle
over a short prefix therefore checks the stored trace samples of a shot (and
with them the generators, the geometry and the oracle) without the full-length
run; the gradient samples are checked for shape and finiteness.
"""
import importlib.util
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_spec = importlib.util.spec_from_file_location("make_full_size", os.path.join(GOLD, "make_full_size.py"))
G = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(G)


@pytest.mark.parametrize("name,shot,n", [("c2_grad", 0, 240), ("c2_grad", 15, 240), ("c4_uneven", 3, 200),
                                         ("c5_crop", 0, 60)])
def test_fixture_trace_prefix(name, shot, n):
    path = os.path.join(GOLD, f"{name}_full.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gold = np.load(path)
    wl = W.make_config(name)
    sh = wl.shots[shot]
    d = O.forward(wl.m(sh.window, background=True), wl.q(shot)[:n], sh.src, sh.rec, h=wl.h, dt=wl.dt,
                  nbl=wl.nbl, vref=wl.vmax)
    ti, ri = gold[f"trace_t_{shot}"], gold[f"trace_r_{shot}"]
    keep = ti < n
    assert keep.sum() >= n // G.TIME_STRIDE
    np.testing.assert_allclose(d[np.ix_(ti[keep], ri)], gold[f"trace_value_{shot}"][keep], rtol=0,
                               atol=1e-12 * np.abs(d).max())
    for w in range(wl.nwindow):
        idx, val = gold[f"grad_index_{w}"], gold[f"grad_value_{w}"]
        assert idx.shape == val.shape and idx.max() < int(np.prod(wl.comp_shape(w)))
        assert np.isfinite(val).all()
    assert np.abs(gold["trace_value_0"]).max() > 0


@pytest.mark.parametrize("shot,n", [(0, 240), (11, 240)])
def test_born_fixture_trace_prefix(shot, n):
    path = os.path.join(GOLD, "c2_born_full.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gold = np.load(path)
    wl = W.make_config("c2_grad")
    sh = wl.shots[shot]
    d = O.born(wl.m(0, background=True), wl.q(shot)[:n], G.born_perturbation(wl), sh.src, sh.rec, h=wl.h,
               dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    ti, ri = gold[f"trace_t_{shot}"], gold[f"trace_r_{shot}"]
    keep = ti < n
    np.testing.assert_allclose(d[np.ix_(ti[keep], ri)], gold[f"trace_value_{shot}"][keep], rtol=0,
                               atol=1e-12 * np.abs(d).max())
    assert np.abs(d).max() > 0 and np.abs(gold[f"trace_value_{shot}"]).max() > 0


@pytest.mark.parametrize("name,shot,n", [("c6_timelapse", 0, 1600), ("c7_timelapse_rock", 0, 1400)])
def test_timelapse_fixture_trace_prefix(name, shot, n):
    """The time-lapse fixtures' traces at each vintage's starting wavespeed (m = 1/v^2 of the
    float32 wavespeed, in FP64); for the rock workload that wavespeed is R at zero saturation,
    which is the brine rock's own vp.  Sources and receivers sit in two wells 2.5 km apart, so
    the prefix runs past the first arrivals (the stored samples it covers are not all zero)."""
    path = os.path.join(GOLD, f"{name}_full.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gold = np.load(path)
    wl = W.make_config(name)
    par, v, rock = G.timelapse_models(wl)
    if rock is not None:
        np.testing.assert_allclose(v[0], rock[0], rtol=1e-12, atol=0)
        assert all(np.all(p == 0) for p in par)
    sh = wl.shots[shot]
    d = O.forward(O.slowness2(v[sh.window]), wl.q(shot)[:n], sh.src, sh.rec, h=wl.h, dt=wl.dt,
                  nbl=wl.nbl, vref=wl.vmax)
    ti, ri = gold[f"trace_t_{shot}"], gold[f"trace_r_{shot}"]
    keep = ti < n
    assert keep.sum() >= n // G.TIME_STRIDE
    np.testing.assert_allclose(d[np.ix_(ti[keep], ri)], gold[f"trace_value_{shot}"][keep], rtol=0,
                               atol=1e-12 * np.abs(d).max())
    stored = gold[f"trace_value_{shot}"]
    assert np.abs(stored[keep]).max() > 0.05 * np.abs(stored).max()
    assert sorted(int(k[len("grad_index_"):]) for k in gold.files if k.startswith("grad_index_")) == \
        list(range(wl.nwindow))
    for w in range(wl.nwindow):
        idx, val = gold[f"grad_index_{w}"], gold[f"grad_value_{w}"]
        assert idx.shape == val.shape and idx.max() < int(np.prod(wl.comp_shape(w)))
        assert np.isfinite(val).all() and np.abs(val).max() > 0


def test_fp32_floor_record_supports_the_gpu_gates():
    """The float32-emulated oracle's rounding floor (written by measure_fp32_floor.py, oracle
    only) is what the GPU gates lean on: the Born trace bar of 2e-5 and the probed-gradient bars of
    1.5e-4 (2D) and 3e-5 (the 3D crop) sit below the operators' float32 floors, and the dot-test bar of 1e-5 above the float32
    dot-test floors; FP64 dot tests are exact to 1e-12."""
    import json
    rec = json.load(open(os.path.join(GOLD, "fp32_floor.json")))
    assert rec["c2_grad"]["born_traces_rel_l2"] > 2e-5
    assert rec["c2_grad"]["forward_traces_rel_l2"] > 1e-5
    assert rec["c9_probed"]["gradient_rel_l2"] > 1.5e-4      # the full-size probed gradient's bar
    assert rec["c9_probed_crop"]["gradient_rel_l2"] > 3e-5   # the 3D crop's probed gradient's bar
    dots = rec["small_2d_dot_tests"]
    assert dots["F_dot_rel_fp32"] < 1e-5 and dots["J_dot_rel_fp32"] < 1e-5
    assert dots["F_dot_rel_fp64"] < 1e-12 and dots["J_dot_rel_fp64"] < 1e-12
