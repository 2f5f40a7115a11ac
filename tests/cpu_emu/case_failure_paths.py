"""CPU build: a plan's failure paths.

1. AUTO storage with the device's free memory (EMU_FREE_BYTES) below the FULL workspace resolves
   to CHECKPOINT storage, and its gradient equals the FULL-storage gradient bit for bit.
2. Input screening: a NaN in m or dd gives NONFINITE, a velocity above the plan's vmax gives CFL,
   and no compute kernel runs.
3. Output screening: with the velocity ten times the bound the leapfrog blows up, and the
   traces are reported not finite.
4. Autotuner cache (AWE_TUNE_CACHE): the first call adds an entry; an entry found in the file is
   applied without running any kernel.
"""
import json
import os
import tempfile

import numpy as np

import driver as D
from paper_2304_05592_amd import binding as B
import workloads as W


def expect(status, fn):
    try:
        fn()
    except B.AweError as e:
        assert e.status == status, (e.status, str(e))
        return str(e)
    raise AssertionError(f"expected status {status}")


def main():
    lib = D.EmuLib(os.environ["AWE_EMU_SO"])
    wl = W.small_2d(nshot=2, T=60.0)
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 3 + i) for i, s in enumerate(wl.shots)]

    # 1. AUTO storage under a small free-memory figure
    full = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_FULL))
    m = full.pack([wl.m(w) for w in range(wl.nwindow)])
    q = full.pack([wl.q(s) for s in range(wl.nshot)])
    dd = full.pack(dds)
    g_full = full.gradient(m, q, dd)[0]
    os.environ["EMU_FREE_BYTES"] = str(int(full.ws_bytes() * 0.5 / 0.9))
    auto = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_AUTO))
    eff = auto.get_storage()
    assert eff.mode == B.STORE_CHECKPOINT and eff.nslots >= 1, eff
    assert auto.ws_bytes() <= full.ws_bytes() * 0.5
    g_auto = auto.gradient(m, q, dd)[0]
    assert np.array_equal(g_auto, g_full)
    del os.environ["EMU_FREE_BYTES"]
    print(f"AUTO -> CHECKPOINT {eff.nslots} slots: gradient bitwise equal to FULL", flush=True)

    # 2. input screening
    full.set_checks(B.CHECK_INPUTS)
    n0 = lib.L.emu_launch_count()
    bad = m.copy()
    bad[len(bad) // 3] = np.nan
    print(expect(B.AWE_ERR_NONFINITE, lambda: full.gradient(bad, q, dd)), flush=True)
    bad_dd = dd.copy()
    bad_dd[-1] = np.inf
    print(expect(B.AWE_ERR_NONFINITE, lambda: full.gradient(m, q, bad_dd)), flush=True)
    fast = (m / np.float32(100.0)).astype(np.float32)   # ten times the velocity bound
    print(expect(B.AWE_ERR_CFL, lambda: full.forward(fast, q)), flush=True)
    screens = lib.L.emu_launch_count() - n0
    assert screens <= 3 * 8, screens      # screening and counter clears only
    ok = full.gradient(m, q, dd)[0]
    assert np.array_equal(ok, g_full)

    # 3. output screening catches the blow-up
    full.set_checks(B.CHECK_OUTPUTS)
    print(expect(B.AWE_ERR_NONFINITE, lambda: full.forward(fast, q)), flush=True)
    full.set_checks(0)
    d = full.forward(fast, q)
    assert not np.isfinite(d).all()

    # 4. autotuner cache
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.json")
        os.environ["AWE_TUNE_CACHE"] = path
        p1 = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_FULL))
        tiles1, _ = p1.autotune(m, q, dd, probe_steps=2)
        entries = json.load(open(path))
        assert len(entries) == 1, entries
        key, e = next(iter(entries.items()))
        assert (tuple(e["fw"]), tuple(e["rv"]), e["fusion"]) == tiles1, (e, tiles1)
        with open(path, "w") as f:
            f.write('{\n  "%s": {"fw": [8, 8, 0], "rv": [64, 8, 0], "fusion": 1, "ms": 42.500000}\n}\n' % key)
        p2 = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_FULL))
        n0 = lib.L.emu_launch_count()
        tiles2, ms = p2.autotune(m, q, dd, probe_steps=2)
        assert lib.L.emu_launch_count() == n0, "a cached result must not run the probes"
        assert tiles2 == ((8, 8, 0), (64, 8, 0), 1) and ms == 42.5, (tiles2, ms)
        assert np.array_equal(p2.gradient(m, q, dd)[0], g_full)
        # another probe length is another key: timed again and added
        p2.autotune(m, q, dd, probe_steps=3)
        assert len(json.load(open(path))) == 2
        del os.environ["AWE_TUNE_CACHE"]
    print("CASE OK", flush=True)


if __name__ == "__main__":
    main()
