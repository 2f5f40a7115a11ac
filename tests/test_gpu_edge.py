"""Degenerate cases against the oracle, through the C ABI: a computational grid smaller than
one tile (2D and 3D), a single time step (nt = 2; 2D and 3D), a shot without receivers in a
batch, and sources and receivers exactly on grid nodes (one interpolation weight 1).

Each 2D case runs traces, F^T dd and the gradient with one and with two time levels per
launch (odd step counts included) and compares them with the oracle at rel-L2 <= 1e-5; the
CHECKPOINT gradient must be bitwise the FULL one.  The 3D cases run two launch shapes (the
whole depth in one z-block, and 8-plane z-blocks with a ragged last one)."""
import numpy as np
import pytest
import torch

import paper_2304_05592_amd as A
import workloads as W
from helpers import gpu_inputs, make_plan, oracle_adjoint, oracle_forward, oracle_gradient, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _residuals(wl, seed=3):
    return [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, seed + i) if len(s.rec)
            else np.zeros((s.nt, 0), np.float32) for i, s in enumerate(wl.shots)]


def _run(wl, dds, fuse, storage=None):
    plan = make_plan(wl, storage=storage or A.Storage(A.STORE_FULL))
    plan.set_tiles(tz=16)
    plan.set_fusion(fuse)
    m, q = gpu_inputs(wl, plan, background=True)
    dd = plan.pack(dds, "d")
    g, v, d = plan.gradient(m, q, dd, v=True, d=True)
    va = plan.adjoint(m, dd)
    torch.cuda.synchronize()
    return plan, g, v, d, va


def _check_against_oracle(wl, dds, case):
    ms = [wl.m(w, background=True) for w in range(wl.nwindow)]
    ref_d = oracle_forward(wl, ms=ms)
    ref_v = oracle_adjoint(wl, dds, ms=ms)
    ref_g = oracle_gradient(wl, dds, ms=ms)
    outs = {}
    for fuse in (A.FUSE_NONE, A.FUSE_BOTH):
        plan, g, v, d, va = _run(wl, dds, fuse)
        got_d, got_v = plan.unpack(d, "d"), plan.unpack(v, "q")
        got_g = plan.unpack(g, "m")
        errs = (rel_l2(got_d, ref_d), rel_l2(got_v, ref_v), rel_l2(got_g, ref_g))
        print(f"{case} fusion {fuse}: traces {errs[0]:.2e}, F^T dd {errs[1]:.2e}, gradient {errs[2]:.2e}",
              flush=True)
        assert max(errs) <= TOL, (case, fuse, errs)
        assert torch.equal(va, v)
        outs[fuse] = [t.cpu() for t in (g, v, d)]
    # one and two levels per launch are bitwise the same; checkpointing changes no bit
    assert all(torch.equal(a, b) for a, b in zip(outs[A.FUSE_NONE], outs[A.FUSE_BOTH]))
    _, g, v, d, _ = _run(wl, dds, A.FUSE_NONE, A.Storage(A.STORE_CHECKPOINT, 2))
    assert all(torch.equal(a.cpu(), b) for a, b in zip((g, v, d), outs[A.FUSE_NONE]))
    return plan.unpack(v, "q"), plan.unpack(d, "d")


def test_grid_smaller_than_one_tile():
    """6 x 4 physical cells + 4-cell borders: a 14 x 12 computational grid, less than one tile
    (64 columns, 16 rows) in both directions."""
    wl = W.small_2d(nx=6, nz=4, nbl=4, T=300.0, nshot=2)
    assert wl.comp_shape(0) == (12, 14)
    _check_against_oracle(wl, _residuals(wl), "tiny grid")


def test_single_time_step():
    """nt = 2: one forward step (u^1 from the source sample q^0 alone) and one adjoint step;
    d^0 and v^{nt-1} are zero by definition."""
    wl = W.small_2d(nx=40, nz=24, nbl=4, T=1.0, nshot=2)
    assert all(s.nt == 2 for s in wl.shots)
    v, d = _check_against_oracle(wl, _residuals(wl), "nt = 2")
    assert all(not x[0].any() for x in d)           # d^0 of both shots
    assert all(x[1] == 0 for x in v)                # v^{nt-1} of both shots


def test_shot_without_receivers_in_a_batch():
    """The middle shot of three records nothing: its traces are empty, its F^T dd is exactly
    zero and it adds nothing to the gradient."""
    wl = W.small_2d(nx=40, nz=24, nbl=4, T=120.0, nshot=3)
    wl.shots[1].rec = np.zeros((0, 3))
    v, d = _check_against_oracle(wl, _residuals(wl), "no receivers")
    assert d[1].size == 0 and not v[1].any()


def test_source_and_receivers_on_grid_nodes():
    """Source and receivers exactly on grid nodes: bilinear weights (1, 0, 0, 0), the base
    node's right / lower neighbours get weight zero."""
    wl = W.small_2d(nx=40, nz=24, nbl=4, T=150.0, nshot=2)
    h = wl.h
    for i, s in enumerate(wl.shots):
        s.src = np.array([(12.0 + 9 * i) * h, 0.0, 5.0 * h])
        s.rec = s.rec.copy()
        s.rec[:, 0] = np.arange(len(s.rec)) * h
        s.rec[:, 2] = 2.0 * h
    _check_against_oracle(wl, _residuals(wl), "on-node geometry")


def _check_3d(wl, case):
    dds = _residuals(wl)
    ms = [wl.m(0, background=True)]
    ref_d, ref_v = oracle_forward(wl, ms=ms), oracle_adjoint(wl, dds, ms=ms)
    ref_g = oracle_gradient(wl, dds, ms=ms)
    outs = []
    for ty, bz in ((8, 0), (4, 8)):                 # whole depth; 8-plane blocks + a ragged one
        plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
        plan.set_tiles(tz=32, ty=ty, bz=bz)
        m, q = gpu_inputs(wl, plan, background=True)
        g, v, d = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
        torch.cuda.synchronize()
        errs = (rel_l2(plan.unpack(d, "d"), ref_d), rel_l2(plan.unpack(v, "q"), ref_v),
                rel_l2(plan.unpack(g, "m"), ref_g))
        print(f"{case} ty {ty} bz {bz}: traces {errs[0]:.2e}, F^T dd {errs[1]:.2e}, "
              f"gradient {errs[2]:.2e}", flush=True)
        assert max(errs) <= TOL, (case, ty, bz, errs)
        outs.append([t.cpu() for t in (g, v, d)])
    assert all(torch.equal(a, b) for a, b in zip(*outs))
    return plan.unpack(v, "q"), plan.unpack(d, "d")


def test_3d_grid_smaller_than_one_column_block():
    """7 x 5 x 6 physical cells + 4-cell borders: 15 x 13 columns (a block is 64 wide) and
    14 planes."""
    wl = W.small_3d(n=(6, 5, 7), h=12.5, nbl=4, T=200.0, nrec_side=2, nshot=2)
    assert wl.comp_shape(0) == (14, 13, 15)
    _check_3d(wl, "3D tiny grid")


def test_3d_single_time_step():
    """nt = 2 in 3D.  After one step u^1 is nonzero only on the source's eight nodes and w^1 only
    on the receivers' nodes, so one receiver per shot sits next to the source (otherwise every
    output is exactly zero)."""
    wl = W.small_3d(n=(6, 5, 7), h=12.5, nbl=4, T=1.0, nrec_side=2, nshot=2)
    assert all(s.nt == 2 for s in wl.shots)
    for s in wl.shots:
        s.rec = s.rec.copy()
        s.rec[0] = s.src + 0.3 * wl.h
    v, d = _check_3d(wl, "3D nt = 2")
    assert all(not x[0].any() for x in d) and all(x[1] == 0 for x in v)
