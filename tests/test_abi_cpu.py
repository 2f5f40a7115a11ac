"""Host-side checks of the C ABI that need no GPU: exported symbols, argument validation,
and the binomial checkpoint schedule."""
import argparse
import math
import os
import re
from functools import lru_cache

import numpy as np
import pytest

import paper_2304_05592_amd as A
from paper_2304_05592_amd import binding as B


def _declared_functions():
    text = open(B.os.path.join(B._HERE, "..", "include", "awe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(awe_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = A.lib()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(A.EXPORTS)
    assert L.awe_version() == 1


def _problem(**over):
    shot = B.AweShot()
    shot.nx, shot.ny, shot.nz, shot.nt = 50, 1, 40, 100
    shot.nrec = 2
    shot.src[0], shot.src[1], shot.src[2] = 100.0, 0.0, 50.0
    rec = np.array([[10.0, 0, 20.0], [200.0, 0, 20.0]])
    p = B.AweProblem()
    p.ndim, p.nbl, p.h, p.dt, p.vmax, p.damp_vref, p.damp_R = 2, 5, 10.0, 1.0, 3.0, 3.0, 1e-3
    p.nshot = 1
    for k, v in over.items():
        if hasattr(shot, k):
            setattr(shot, k, v)
        else:
            setattr(p, k, v)
    arr = (B.AweShot * 1)(shot)
    p.shots = B.ctypes.cast(arr, B.ctypes.POINTER(B.AweShot))
    p.rec_pos = rec.ctypes.data_as(B.ctypes.POINTER(B.ctypes.c_double))
    return p, (arr, rec)


def _create(p, mode=0, nslots=0, prec=0):
    st = B.AweStorage(mode, nslots, prec, 0)
    h = B.ctypes.c_void_p()
    s = A.lib().awe_plan_create(B.ctypes.byref(p), B.ctypes.byref(st), B.ctypes.byref(h))
    if s == 0:
        A.lib().awe_plan_destroy(h)
    return s, A.lib().awe_last_error().decode()


def test_cfl_violation_is_rejected():
    lim = 2 / math.sqrt(2 * (205 / 72 + 2 * (8 / 5 + 1 / 5 + 8 / 315 + 1 / 560)))
    p, keep = _problem(dt=1.01 * lim * 10.0 / 3.0)
    s, msg = _create(p)
    assert s == 3 and "stability" in msg


def test_geometry_outside_grid_is_rejected():
    p, keep = _problem()
    keep[1][1, 0] = 1e5
    s, msg = _create(p)
    assert s == 4 and "receiver 1" in msg
    p, keep = _problem()
    p.shots[0].src[2] = -80.0
    assert _create(p)[0] == 4


@pytest.mark.parametrize("over,code", [({"ndim": 4}, 1), ({"nt": 1}, 1), ({"h": -1.0}, 1),
                                       ({"damp_R": 0.0}, 1), ({"ny": 2}, 1), ({"nshot": 0}, 1)])
def test_invalid_arguments_are_rejected(over, code):
    p, keep = _problem(**over)
    assert _create(p)[0] == code


def test_bad_storage_is_rejected():
    p, keep = _problem()
    assert _create(p, mode=2, nslots=0)[0] == 1
    assert _create(p, mode=7)[0] == 1
    p3, keep3 = _problem(ndim=3, ny=40)
    assert _create(p3, mode=2, nslots=4)[0] == 2


def _select(p, mode, nslots=0, prec=0, budget_mib=0):
    """(status, storage in effect, workspace bytes) from awe_storage_select (host only)."""
    st, out, nb = B.AweStorage(mode, nslots, prec, budget_mib), B.AweStorage(), B.ctypes.c_size_t(0)
    s = A.lib().awe_storage_select(B.ctypes.byref(p), B.ctypes.byref(st), B.ctypes.byref(out), B.ctypes.byref(nb))
    return s, (out.mode, out.nslots, out.prec), nb.value


def test_auto_storage_falls_back_to_checkpoint_under_a_memory_budget():
    """AUTO storage against a mocked budget: FULL while its workspace fits, else CHECKPOINT with
    the largest slot count whose workspace fits; WORKSPACE when not even one slot fits."""
    p, keep = _problem(nx=500, nz=400, nt=1000)
    s, full, F = _select(p, 1)
    assert s == 0 and full == (1, 0, 0)
    ck = {k: _select(p, 2, k)[2] for k in (1, 2, 16, 17, 63, 64, 65)}
    assert all(ck[a] < ck[b] for a, b in zip(sorted(ck), sorted(ck)[1:]))
    assert ck[1] < F
    mib = 1 << 20
    s, eff, nb = _select(p, 3, budget_mib=-(-F // mib))
    assert s == 0 and eff == (1, 0, 0) and nb == F
    budget = 100
    s, eff, nb = _select(p, 3, budget_mib=budget)
    assert s == 0 and eff[0] == 2 and eff[2] == 0
    k = eff[1]
    assert nb == _select(p, 2, k)[2] <= budget * mib < _select(p, 2, k + 1)[2]
    s, eff, _ = _select(p, 3, nslots=16, budget_mib=budget)
    assert s == 0 and eff == (2, 16, 0)
    s, eff, nb = _select(p, 3, prec=1, budget_mib=budget)      # BF16 slots: more of them fit
    assert s == 0 and eff[0] == 2 and eff[1] > k and nb <= budget * mib
    s, _, _ = _select(p, 3, budget_mib=ck[1] // mib)
    assert s == 5 and "budget" in A.lib().awe_last_error().decode()
    assert _select(p, 3, nslots=-1, budget_mib=10)[0] == 1
    assert _select(p, 3, budget_mib=-1)[0] == 1
    p3, keep3 = _problem(ndim=3, ny=40, nx=60, nz=60, nt=400)
    s, eff, nb = _select(p3, 3, budget_mib=4)
    assert s == 2 and "disabled in 3D" in A.lib().awe_last_error().decode()
    s, full3, F3 = _select(p3, 1)
    assert _select(p3, 3, budget_mib=-(-F3 // mib))[:2] == (0, (1, 0, 0))


def test_auto_storage_binding_reports_the_choice():
    st, nb = B.select_storage(2, 10.0, 1.0, 5, 3.0, [(400, 500)],
                              [B.ShotGeometry(0, 1000, (100.0, 0.0, 50.0), np.array([[10.0, 0, 20.0]]))],
                              B.Storage(B.STORE_AUTO, 0, B.PREC_FP32, 50))
    assert st.mode == B.STORE_CHECKPOINT and st.nslots >= 1 and nb <= 50 << 20


# ------------------------------------------------------------------------------ schedule
@lru_cache(None)
def _dp(l, s):
    """Minimal forward steps to reverse l levels from a stored start with s free slots when
    every reversal needs its own state (the classic problem)."""
    if l == 0:
        return 0
    if s == 0:
        return l * (l + 1) // 2
    best = l + _dp(l - 1, s)
    for c in range(1, l):
        best = min(best, c + _dp(l - c, s - 1) + _dp(c - 1, s))
    return best


@lru_cache(maxsize=None)
def _dp2(l, s):
    """The same when a state S_j = (u^j, u^{j-1}) serves the reversals of both its levels:
    reaching level l reverses l and l - 1; a checkpoint at c (stored, the levels above it
    reversed from there, then restored) reverses c and c - 1."""
    if l <= 0:
        return 0
    best = l + _dp2(l - 2, s)
    if s > 0:
        for c in range(1, l):
            best = min(best, c + _dp2(l - c, s - 1) + _dp2(c - 2, s))
    return best


def _simulate(n, slots, actions):
    """Replay the action list on a counter; returns the number of forward steps."""
    cur, stored, steps, reversed_ = 0, {}, 0, []
    for op, a, b in actions:
        if op == 0:
            assert a == cur and b > a
            steps += b - a
            cur = b
        elif op == 1:
            assert b == cur and 0 <= a < slots
            stored[a] = b
        elif op == 2:
            if a == -1:
                assert b == 0
            else:
                assert stored.get(a) == b
            cur = b
        elif op == 3:
            assert a in (cur, cur - 1)   # the current state holds u^cur and u^(cur-1)
            reversed_.append(a)
    assert reversed_ == list(range(n, 0, -1))
    return steps


@pytest.mark.parametrize("n,s", [(1, 1), (2, 1), (10, 2), (37, 3), (60, 1), (60, 5), (25, 30),
                                 (80, 0)])
def test_checkpoint_schedule_is_valid_and_optimal(n, s):
    acts = A.checkpoint_schedule(n, s)
    steps = _simulate(n, s, acts)
    # the paired problem's optimum for an even n, at most one step more for an odd n; never
    # more than the classic optimum
    assert steps == _dp2(n, s) if n % 2 == 0 else _dp2(n, s) <= steps <= _dp2(n, s) + 1
    assert steps <= _dp(n, s)
    # the first sweep advances 0 -> n once, before any reversal
    first_rev = next(i for i, a in enumerate(acts) if a[0] == 3)
    adv = [a for a in acts[:first_rev] if a[0] == 0]
    assert adv[0][1] == 0 and adv[-1][2] == n
    assert all(adv[i][2] == adv[i + 1][1] for i in range(len(adv) - 1))


def test_checkpoint_schedule_large_counts_binomial_cost():
    # 16 slots and 5000 levels: the binomial law on the 2500 pairs, two steps each (the paired
    # problem's optimum is twice the classic one at half the length, checked on small cases)
    acts = A.checkpoint_schedule(5000, 16)
    steps = _simulate(5000, 16, acts)
    assert 3 * 5000 < steps < 4 * 5000
    for l in (4, 10, 36, 60):
        assert _dp2(l, 3) == 2 * _dp(l // 2, 3)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_patchy_argument_checks_raise_before_any_device_call():
    import torch
    a = torch.zeros(5)
    with pytest.raises(TypeError):
        A.patchy(a, a, a, torch.zeros(4))             # size mismatch
    with pytest.raises(TypeError):
        A.patchy_vjp(a, a, a, a, a.double())          # wrong dtype
    with pytest.raises(NotImplementedError):
        A.patchy_rock_physics(a, a.clone().requires_grad_(True), a, a)


def test_born_forward_refuses_gradients_of_the_background():
    import torch
    z = torch.zeros(3)
    with pytest.raises(NotImplementedError):
        A.born_forward(z, z.clone().requires_grad_(True), z, None)


def _bench_module():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(root, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_roofline_bookkeeping():
    """Launch shapes map to fusion modes; a class that runs two levels per launch is charged the
    algorithmic bytes of two point-updates per grid point (the per-step table), with the
    launch's own fused bytes reported beside; the dominant kernel is the one with the larger
    time share."""
    bench = _bench_module()
    assert bench.fusion_of(None) == 0
    assert bench.fusion_of({"tz": 16}) == 0
    assert bench.fusion_of({"tz": 16, "levels_per_launch": 2}) == 3
    assert bench.fusion_of({"tz": 16, "fusion": 2}) == 2
    prof = {"forward": (3637, 3637 * 0.018), "adjoint": (1819, 1819 * 0.051)}
    k = bench.kernel_table(prof, 1000, {"forward": "fp32", "adjoint": "fp32"}, fused=2)
    assert k["forward"]["bytes_per_launch"] == 20 * 1000
    assert k["adjoint"]["bytes_per_launch"] == 2 * 36 * 1000        # two point-updates per point
    assert k["adjoint"]["fused_bytes_per_launch"] == 44 * 1000
    assert "fused_bytes_per_launch" not in k["forward"]
    assert k["adjoint"]["levels_per_launch"] == 2 and k["forward"]["levels_per_launch"] == 1
    assert abs(k["adjoint"]["achieved_GBs"] - 72e3 / 51e-6 / 1e9) < 0.1
    roof = bench.roofline_of(k, {"forward": "f", "adjoint": "a"})
    assert roof["kernel"] == "a"                       # 1819 x 51 us > 3637 x 18 us
    assert abs(roof["frac"] - roof["achieved"] / bench.PEAK_HBM_GBS) < 1e-4
    assert roof["fused_bytes_achieved"] == k["adjoint"]["fused_GBs"]
    k1 = bench.kernel_table({"forward": (100, 100 * 0.02), "adjoint": (100, 100 * 0.03)}, 1000,
                            {"forward": "fp32", "adjoint": "fp32"}, fused=0)
    assert bench.roofline_of(k1, {"forward": "f", "adjoint": "a"})["kernel"] == "a"
    k1["adjoint"]["avg_us"] = 15.0
    bench.refresh_rates(k1["adjoint"])
    assert abs(k1["adjoint"]["achieved_GBs"] - 36e3 / 15e-6 / 1e9) < 0.1


def test_bench_picks_the_fastest_pass_shape(monkeypatch):
    """The benchmark's own tile choice for single-pass workloads times every (tile height,
    forward fusion) candidate, skips two levels with 64-row tiles (no such kernel), keeps the
    cheapest and leaves the plan set to it; --tiles bypasses the search."""
    bench = _bench_module()
    cost = {(8, 0): 5.0, (16, 0): 4.0, (24, 0): 3.8, (32, 0): 3.5, (64, 0): 3.2, (8, 1): 4.5, (16, 1): 3.0,
            (24, 1): 3.05, (32, 1): 3.1}
    clock = [0.0]

    class FakePlan:
        tz = fu = None
        seen = []

        def set_tiles(self, tz, ty=8, bz=0, dirs=3):
            self.tz = tz

        def set_fusion(self, fu):
            self.fu = int(fu)

        def get_tiles(self):
            return {"tz": self.tz, "fusion": self.fu}

    plan = FakePlan()

    def run():
        plan.seen.append((plan.tz, plan.fu))
        clock[0] += cost[(plan.tz, plan.fu)]

    monkeypatch.setattr(bench, "sync", lambda: None)
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock[0])
    args = argparse.Namespace(tiles=None, no_autotune=False)
    tiles = bench.choose_pass_tiles(plan, args, run, fusions=(0, 1))
    assert tiles == {"tz": 16, "ty": 8, "bz": 0, "fusion": 1}
    assert (plan.tz, plan.fu) == (16, 1)
    assert (64, 1) not in plan.seen and len(set(plan.seen)) == 9
    fixed = argparse.Namespace(tiles={"tz": 32, "fusion": 0}, no_autotune=False)
    assert bench.choose_pass_tiles(plan, fixed, run) == {"tz": 32, "fusion": 0}
