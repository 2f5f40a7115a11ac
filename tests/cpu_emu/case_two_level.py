"""CPU build: the 2D gradient with FULL FP32 storage on an uneven batch (three windows, per-shot
nt), with two levels per launch in both sweeps at every two-level tile height (8, 16, 24, 32
rows) and with one level per launch, under AddressSanitizer with poisoned gaps between the
workspace's sub-buffers; every result is bitwise the one-level result, which is compared with
the oracle.  Prints one JSON line."""
import json
import os

import numpy as np

import driver as D
from paper_2304_05592_amd import binding as B
import oracle as O
import workloads as W


def main():
    lib = D.EmuLib(os.environ["AWE_EMU_SO"])
    wl = W.small_2d(windows=[90, 70, 113], T_per_shot=[120.0, 80.0, 101.0])
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 3 + i) for i, s in enumerate(wl.shots)]
    out = {"nt": [s.nt for s in wl.shots]}
    res = {}
    for tz, fusion in ((16, 0), (8, 3), (16, 3), (24, 3), (32, 3)):
        plan = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_FULL))
        plan.set_checks(4)   # host-side launch checks
        plan.set_tiles(tz, 8, 0)
        plan.set_fusion(fusion)
        m = plan.pack([wl.m(w) for w in range(wl.nwindow)])
        q = plan.pack([wl.q(i) for i in range(wl.nshot)])
        res[(tz, fusion)] = plan.gradient(m, q, plan.pack(dds), v=True, d=True)
        assert plan.get_tiles()[0][0] == tz and plan.get_tiles()[2] == fusion
        del plan
    # Born modelling with two levels per launch at every height: bitwise the one-level traces
    dms = [W.random_field(wl.comp_shape(w), 17 + w, 2.0) * np.float32(0.01) for w in range(wl.nwindow)]
    born = {}
    for tz, fusion in ((16, 0), (8, 1), (16, 1), (24, 1), (32, 1)):
        plan = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_NONE))
        plan.set_checks(4)
        plan.set_tiles(tz, 8, 0)
        plan.set_fusion(fusion)
        m = plan.pack([wl.m(w) for w in range(wl.nwindow)])
        q = plan.pack([wl.q(i) for i in range(wl.nshot)])
        born[(tz, fusion)] = plan.born(m, q, plan.pack(dms))
        del plan
    out["born_bitwise"] = {f"{tz}_{fu}": bool(np.array_equal(r, born[(16, 0)])) for (tz, fu), r in born.items()}
    base = res[(16, 0)]
    out["bitwise"] = {f"{tz}_{fu}": all(np.array_equal(a, b) for a, b in zip(r, base)) for (tz, fu), r in res.items()}
    gs = [np.zeros(wl.comp_shape(w)) for w in range(wl.nwindow)]
    for i, sh in enumerate(wl.shots):
        gs[sh.window] += O.gradient(wl.m(sh.window), wl.q(i), dds[i], src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt,
                                    nbl=wl.nbl, vref=wl.vmax)
    g = base[0]
    plan = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_FULL))
    got = np.concatenate([g[o:o + int(np.prod(sh))] for o, sh in zip(plan.layout.m_offset, plan.layout.windows)])
    ref = np.concatenate([x.ravel() for x in gs])
    out["grad_rel"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
