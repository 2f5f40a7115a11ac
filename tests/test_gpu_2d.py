"""GPU parity of the 2D path against the oracle, through the C ABI.

Tolerance: relative L2 <= 1e-5 for float32 traces, adjoint samples, Born data and gradients
(the float32 rounding floor of these sizes is ~1e-6).  Sizes span several 64 x 32 tiles with
ragged edges; the oracle finishes each case in about a second.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_05592_amd as A
import workloads as W
from helpers import (gpu_inputs, make_plan, oracle_adjoint, oracle_born, oracle_forward,
                     oracle_gradient, rel_l2, shot_kwargs)

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _sync():
    torch.cuda.synchronize()


def _report(name, err):
    print(f"{name}: rel-L2 {err:.3e}", flush=True)


def _residuals(wl, seed=3):
    return [W.synthetic_residual(wl.shots[s].nt, len(wl.shots[s].rec), wl.dt, wl.f0, seed + s)
            for s in range(wl.nshot)]


def _oracle_residual(wl):
    """dd = F(m0) q - F(m_true) q from the oracle (both models from the generator)."""
    d_true = oracle_forward(wl)
    d0 = oracle_forward(wl, ms=[wl.m(w, background=True) for w in range(wl.nwindow)])
    return [(a - b).astype(np.float32) for a, b in zip(d0, d_true)]


def test_forward_parity_small_survey():
    wl = W.small_2d()
    plan = make_plan(wl)
    m, q = gpu_inputs(wl, plan)
    d = plan.forward(m, q)
    _sync()
    err = rel_l2(plan.unpack(d, "d"), oracle_forward(wl))
    _report("forward small_2d", err)
    assert err <= TOL


def test_forward_parity_two_layer_full_size_mirror_and_determinism():
    wl = W.make_config("c1_fwd")
    plan = make_plan(wl)
    m, q = gpu_inputs(wl, plan)
    d1 = plan.forward(m, q)
    d2 = plan.forward(m, q)
    _sync()
    got = plan.unpack(d1, "d")[0]
    err = rel_l2(got, oracle_forward(wl)[0])
    _report("forward c1_fwd", err)
    assert err <= TOL
    assert torch.equal(d1, d2)
    assert np.array_equal(got[:, :50], got[:, 100:50:-1])


def test_adjoint_parity():
    wl = W.small_2d()
    plan = make_plan(wl)
    m, _ = gpu_inputs(wl, plan)
    dds = _residuals(wl)
    v = plan.adjoint(m, plan.pack(dds, "d"))
    _sync()
    err = rel_l2(plan.unpack(v, "q"), oracle_adjoint(wl, dds))
    _report("adjoint small_2d", err)
    assert err <= TOL


def test_born_parity():
    wl = W.small_2d()
    plan = make_plan(wl)
    m, q = gpu_inputs(wl, plan, background=True)
    dms = [W.random_field(wl.comp_shape(0), 4, smooth_cells=2.0) * np.float32(0.01)]
    dd = plan.born(m, q, plan.pack(dms, "m"))
    _sync()
    ms = [wl.m(0, background=True)]
    err = rel_l2(plan.unpack(dd, "d"), oracle_born(wl, dms, ms=ms))
    _report("born small_2d", err)
    assert err <= TOL


def test_gradient_full_storage_parity():
    wl = W.small_2d()
    plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    m, q = gpu_inputs(wl, plan, background=True)
    dds = _oracle_residual(wl)
    g, v, d = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
    _sync()
    ms = [wl.m(0, background=True)]
    g_ref = oracle_gradient(wl, dds, ms=ms)
    err = rel_l2(plan.unpack(g, "m"), g_ref)
    _report("gradient FULL small_2d", err)
    assert err <= TOL
    err_v = rel_l2(plan.unpack(v, "q"), oracle_adjoint(wl, dds, ms=ms))
    _report("gradient v small_2d", err_v)
    assert err_v <= TOL
    assert rel_l2(plan.unpack(d, "d"), oracle_forward(wl, ms=ms)) <= TOL


def test_checkpointed_gradient_is_bitwise_the_full_storage_gradient():
    wl = W.small_2d()
    dds = _residuals(wl)
    out = []
    for st in (A.Storage(A.STORE_FULL), A.Storage(A.STORE_CHECKPOINT, 3), A.Storage(A.STORE_CHECKPOINT, 1)):
        plan = make_plan(wl, storage=st)
        m, q = gpu_inputs(wl, plan, background=True)
        g, v, _ = plan.gradient(m, q, plan.pack(dds, "d"), v=True)
        _sync()
        out.append((g.cpu(), v.cpu()))
    for g, v in out[1:]:
        assert torch.equal(g, out[0][0])
        assert torch.equal(v, out[0][1])


@pytest.mark.parametrize("prec,bound", [(A.PREC_BF16, 2e-2), (A.PREC_FP16, 2e-3)])
def test_low_precision_checkpoints_error_is_reported(prec, bound):
    wl = W.small_2d()
    dds = _residuals(wl)
    ref_plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    m, q = gpu_inputs(wl, ref_plan, background=True)
    g_ref, _, _ = ref_plan.gradient(m, q, ref_plan.pack(dds, "d"))
    plan = make_plan(wl, storage=A.Storage(A.STORE_CHECKPOINT, 4, prec))
    g, _, _ = plan.gradient(m, q, plan.pack(dds, "d"))
    _sync()
    err = rel_l2(g.cpu().numpy(), g_ref.cpu().numpy())
    _report(f"gradient CHECKPOINT prec={prec} vs FP32", err)
    assert 0 < err <= bound


def test_uneven_windows_and_lengths_parity():
    wl = W.small_2d(windows=[90, 70, 113], T_per_shot=[400.0, 250.0, 330.0])
    dds = _residuals(wl)
    plan = make_plan(wl, storage=A.Storage(A.STORE_CHECKPOINT, 5))
    m, q = gpu_inputs(wl, plan)
    g, v, d = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
    _sync()
    e_d = rel_l2(plan.unpack(d, "d"), oracle_forward(wl))
    e_g = rel_l2(plan.unpack(g, "m"), oracle_gradient(wl, dds))
    e_v = rel_l2(plan.unpack(v, "q"), oracle_adjoint(wl, dds))
    _report("uneven forward", e_d)
    _report("uneven gradient", e_g)
    _report("uneven adjoint", e_v)
    assert max(e_d, e_g, e_v) <= TOL


def test_batched_equals_single_shot_bitwise():
    wl = W.small_2d(nshot=4)
    dds = _residuals(wl)
    plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    m, q = gpu_inputs(wl, plan)
    _, vb, db = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
    _sync()
    vb, db = plan.unpack(vb, "q"), plan.unpack(db, "d")
    for s in range(wl.nshot):
        p1 = make_plan(wl, storage=A.Storage(A.STORE_FULL), shots=[s])
        m1, q1 = gpu_inputs(wl, p1, shots=[s])
        _, v1, d1 = p1.gradient(m1, q1, p1.pack([dds[s]], "d"), v=True, d=True)
        _sync()
        assert np.array_equal(p1.unpack(d1, "d")[0], db[s])
        assert np.array_equal(p1.unpack(v1, "q")[0], vb[s])


def _dot_errors(a, b, na, nb):
    """|a - b| relative to |a| and to the Cauchy-Schwarz scale ||Fx|| ||y||."""
    return abs(a - b) / max(abs(a), abs(b)), abs(a - b) / (na * nb)


# Dot tests with FP32 operators and FP64 inner products: the float32-emulated oracle reaches
# 4.7e-7 (F) and 5.6e-6 (J) relative on these vectors (tests/golden/fp32_floor.json), below
# 1e-5, so the plain relative difference is held to 1e-5 for both.
DOT_TOL = 1e-5


def test_dot_tests_on_gpu_with_fp64_inner_products():
    """FP32 operators, FP64 inner products: |<Fx,y> - <x,F^T y>| / max(|a|, |b|) <= 1e-5 (and
    the difference scaled by ||Fx|| ||y|| <= 1e-6)."""
    wl = W.small_2d(nshot=2)
    plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    m, _ = gpu_inputs(wl, plan)
    rng = np.random.default_rng(0)
    x = plan.pack([rng.standard_normal(s.nt) for s in wl.shots], "q")
    y = plan.pack([rng.standard_normal((s.nt, len(s.rec))) for s in wl.shots], "d")
    fx = plan.forward(m, x)
    a = A.dot(fx, y).item()
    b = A.dot(x, plan.adjoint(m, y)).item()
    rel, scaled = _dot_errors(a, b, torch.linalg.norm(fx.double()).item(), torch.linalg.norm(y.double()).item())
    _report("GPU F dot test (relative)", rel)
    _report("GPU F dot test (scaled)", scaled)
    assert scaled <= 1e-6 and rel <= DOT_TOL
    dm = plan.pack([W.random_field(wl.comp_shape(0), 1)], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    jdm = plan.born(m, q, dm)
    a = A.dot(jdm, y).item()
    g, _, _ = plan.gradient(m, q, y)
    b = A.dot(dm.double(), g).item()
    rel, scaled = _dot_errors(a, b, torch.linalg.norm(jdm.double()).item(), torch.linalg.norm(y.double()).item())
    _report("GPU J dot test (relative)", rel)
    _report("GPU J dot test (scaled)", scaled)
    assert scaled <= 1e-6 and rel <= DOT_TOL


def test_residual_and_dot_kernels():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(1_234_567).astype(np.float32)
    b = rng.standard_normal(1_234_567).astype(np.float32)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    r, loss = A.residual(ta, tb)
    dot = A.dot(ta, tb)
    _sync()
    assert np.array_equal(r.cpu().numpy(), a - b)
    ref = 0.5 * np.sum((a - b).astype(np.float64) ** 2)
    assert abs(loss.item() - ref) <= 1e-12 * ref
    refd = np.dot(a.astype(np.float64), b.astype(np.float64))
    assert abs(dot.item() - refd) <= 1e-10 * np.abs(a.astype(np.float64) * b).sum()
    # deterministic
    assert A.dot(ta, tb).item() == dot.item()


@pytest.mark.parametrize("prec,bound", [(A.PREC_BF16, 2e-2), (A.PREC_FP16, 2e-3)])
def test_full_16bit_storage_gradient_error_is_reported(prec, bound):
    wl = W.small_2d()
    dds = _residuals(wl)
    ref = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    m, q = gpu_inputs(wl, ref, background=True)
    g32, v32, d32 = ref.gradient(m, q, ref.pack(dds, "d"), v=True, d=True)
    plan = make_plan(wl, storage=A.Storage(A.STORE_FULL, 0, prec))
    g16, v16, d16 = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
    _sync()
    err = rel_l2(g16.cpu().numpy(), g32.cpu().numpy())
    _report(f"gradient FULL prec={prec} vs FP32", err)
    assert 0 < err <= bound
    # the stored precision does not touch the forward traces or F^T dd
    assert torch.equal(d16, d32) and torch.equal(v16, v32)
    e_or = rel_l2(plan.unpack(g16, "m"), oracle_gradient(wl, dds, ms=[wl.m(0, background=True)]))
    _report(f"gradient FULL prec={prec} vs oracle", e_or)
    assert e_or <= bound


def test_results_do_not_depend_on_the_tile_shape_and_autotune_keeps_them():
    wl = W.small_2d(windows=[90, 70], T_per_shot=[300.0, 220.0])
    dds = _residuals(wl)
    plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    m, q = gpu_inputs(wl, plan)
    dd = plan.pack(dds, "d")
    outs = []
    for tz in (8, 12, 16, 20, 24, 32, 64):
        plan.set_tiles(tz=tz)
        g, v, d = plan.gradient(m, q, dd, v=True, d=True)
        outs.append((g.clone(), v.clone(), d.clone()))
    choice, ms = plan.autotune(m, q, dd, probe_steps=16)
    g, v, d = plan.gradient(m, q, dd, v=True, d=True)
    _sync()
    print(f"autotuned tile rows {choice['tz']} ({ms:.3f} ms probe)", flush=True)
    for o in outs[1:] + [(g, v, d)]:
        assert all(torch.equal(a, b) for a, b in zip(o, outs[0]))


def test_autotune_without_a_residual_injects_nothing():
    """Regression: the autotuner's adjoint probe runs with no residual (dd = NULL); tiles that
    hold receivers must then skip the injection instead of reading through the null pointer."""
    wl = W.small_2d(windows=[90, 70], T_per_shot=[200.0, 150.0])
    plan = make_plan(wl)
    m, q = gpu_inputs(wl, plan)
    choice, ms = plan.autotune(m, q, None, probe_steps=8)
    d = plan.forward(m, q)
    _sync()
    assert choice["tz"] in (8, 12, 16, 20, 24, 32, 64) and ms > 0
    assert rel_l2(plan.unpack(d, "d"), oracle_forward(wl)) <= TOL


@pytest.mark.parametrize("tz", [8, 16, 24, 32])
def test_two_levels_per_launch_is_bitwise_the_one_level_path(tz):
    """Uneven windows, per-shot nt (odd and even step counts, end-aligned offsets): forward
    traces, F^T dd and the FULL-storage gradient are bitwise identical with two time levels
    per launch and with one."""
    wl = W.small_2d(windows=[90, 70, 113], T_per_shot=[400.0, 250.0, 331.0])
    dds = _residuals(wl)
    outs = []
    # two levels per launch in both directions, forward only, reverse sweep only; then none
    for fuse in (A.FUSE_BOTH, A.FUSE_FORWARD, A.FUSE_ADJOINT, A.FUSE_NONE):
        plan = make_plan(wl, storage=A.Storage(A.STORE_FULL))
        plan.set_tiles(tz=tz)
        plan.set_fusion(fuse)
        m, q = gpu_inputs(wl, plan)
        g, v, d = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
        va = plan.adjoint(m, plan.pack(dds, "d"))
        _sync()
        outs.append((g.cpu(), v.cpu(), d.cpu(), va.cpu()))
    for other in outs[:-1]:
        for a, b in zip(other, outs[-1]):
            assert torch.equal(a, b)
    assert rel_l2(plan.unpack(outs[0][1], "q"), oracle_adjoint(wl, dds)) <= TOL


@pytest.mark.parametrize("storage", [A.Storage(A.STORE_FULL), A.Storage(A.STORE_CHECKPOINT, 3),
                                     A.Storage(A.STORE_FULL, 0, A.PREC_BF16)],
                         ids=["full32", "checkpoint3", "fullbf16"])
def test_shot_groups_do_not_change_results(storage):
    """Running the shots in groups (one time loop per group) gives bitwise the same traces,
    F^T dd, gradient, adjoint-only and Born results as one group, on uneven windows with
    per-shot nt (groups of one, two and three shots)."""
    wl = W.small_2d(windows=[90, 70, 113, 64], T_per_shot=[400.0, 250.0, 331.0, 290.0])
    dds = _residuals(wl)
    dms = [W.random_field(wl.comp_shape(w), 17 + w, 2.0) * 0.01 for w in range(wl.nwindow)]
    outs = []
    for ng in (1, 2, 3, 4):
        plan = make_plan(wl, storage=storage)
        assert plan.set_groups(ng) == ng
        m, q = gpu_inputs(wl, plan)
        dd = plan.pack(dds, "d")
        g, v, d = plan.gradient(m, q, dd, v=True, d=True)
        va = plan.adjoint(m, dd)
        b = plan.born(m, q, plan.pack(dms, "m"))
        _sync()
        outs.append([t.cpu() for t in (g, v, d, va, b)])
    for o in outs[1:]:
        assert all(torch.equal(a, b) for a, b in zip(o, outs[0]))
    assert rel_l2(plan.unpack(outs[0][2], "d"), oracle_forward(wl)) <= TOL


def test_checkpointed_gradient_with_uneven_nt_is_bitwise_the_full_storage_gradient():
    """Regression: shots of different nt start at different global steps; a checkpoint restore
    of a state before a shot's start left older levels in that shot's buffers, which its first
    steps then read.  Levels below 1 are zero by definition and are no longer read."""
    wl = W.small_2d(windows=[90, 70, 113, 64], T_per_shot=[600.0, 180.0, 400.0, 290.0])
    dds = _residuals(wl)
    out = []
    for st in (A.Storage(A.STORE_FULL), A.Storage(A.STORE_CHECKPOINT, 3), A.Storage(A.STORE_CHECKPOINT, 16)):
        plan = make_plan(wl, storage=st)
        m, q = gpu_inputs(wl, plan, background=True)
        g, v, _ = plan.gradient(m, q, plan.pack(dds, "d"), v=True)
        _sync()
        out.append((g.cpu(), v.cpu()))
    for g, v in out[1:]:
        assert torch.equal(g, out[0][0])
        assert torch.equal(v, out[0][1])


@pytest.mark.parametrize("tz,groups", [(8, 1), (16, 2), (24, 1), (32, 2)])
def test_checkpointed_gradient_with_two_level_reversals_is_bitwise(tz, groups):
    """The paired reversals of a checkpointed gradient run as two-level adjoint launches that
    image from the recomputed forward levels (or a slot read by reference): on an uneven batch
    with per-shot nt the gradient, F^T dd and traces are bitwise the FULL one-level ones with
    FP32 slots and the one-level ones with BF16 slots."""
    wl = W.small_2d(windows=[90, 70, 113, 64], T_per_shot=[600.0, 180.0, 400.0, 290.0])
    dds = _residuals(wl)

    def run(storage, fusion):
        plan = make_plan(wl, storage=storage)
        plan.set_groups(groups)
        plan.set_tiles(tz=tz)
        plan.set_fusion(fusion)
        m, q = gpu_inputs(wl, plan, background=True)
        out = plan.gradient(m, q, plan.pack(dds, "d"), v=True, d=True)
        _sync()
        return [t.cpu() for t in out]

    ref32 = run(A.Storage(A.STORE_FULL), A.FUSE_NONE)
    for slots in (3, 16):
        got = run(A.Storage(A.STORE_CHECKPOINT, slots), A.FUSE_ADJOINT)
        assert all(torch.equal(a, b) for a, b in zip(got, ref32)), f"FP32 slots {slots}"
    ref16 = run(A.Storage(A.STORE_CHECKPOINT, 3, A.PREC_BF16), A.FUSE_NONE)
    got = run(A.Storage(A.STORE_CHECKPOINT, 3, A.PREC_BF16), A.FUSE_ADJOINT)
    assert all(torch.equal(a, b) for a, b in zip(got, ref16))

def test_kernel_timing_counts_every_step_launch_of_a_checkpointed_gradient():
    """With kernel timing on, each checkpoint advance is one timed interval that counts its
    forward launches and each adjoint launch another: a checkpointed gradient of two equal shots
    (one shot group) reports exactly the schedule's forward steps and nt - 1 adjoint steps, with
    positive times, and the same gradient bits as without timing.  With FULL storage each sweep
    is one interval and counts its (two-level) launches."""
    wl = W.small_2d(windows=[90, 90], T_per_shot=[200.0, 200.0])
    dds = _residuals(wl)
    plan = make_plan(wl, storage=A.Storage(A.STORE_CHECKPOINT, 4))
    m, q = gpu_inputs(wl, plan)
    dd = plan.pack(dds, "d")
    ref = plan.gradient(m, q, dd)[0].clone()
    nt = wl.shots[0].nt
    sched = A.checkpoint_schedule(nt - 1, 4)
    fwd_steps = int(sum(b - a for op, a, b in sched if op == 0))
    plan.profile_enable(4 * nt, 1)
    g = plan.gradient(m, q, dd)[0]
    prof = plan.profile_read()
    plan.profile_disable()
    _sync()
    print(f"timed launches: {prof}; schedule forward steps {fwd_steps}", flush=True)
    assert prof["forward"][0] == fwd_steps and prof["adjoint"][0] == nt - 1
    assert prof["forward"][1] > 0 and prof["adjoint"][1] > 0
    assert torch.equal(g, ref)
    # FULL storage: each sweep's step loop is one interval; two levels per launch in both
    full = make_plan(wl, storage=A.Storage(A.STORE_FULL))
    full.set_tiles(tz=16)
    full.set_fusion(A.FUSE_BOTH)
    full.profile_enable(8, 1)
    full.gradient(m, q, dd)
    prof = full.profile_read()
    full.profile_disable()
    _sync()
    launches = (nt - 1) // 2 + (nt - 1) % 2
    assert prof["forward"][0] == launches and prof["adjoint"][0] == launches, prof
