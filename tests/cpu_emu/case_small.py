"""CPU build: 3D gradient with CHECKPOINT storage (FP32 and BF16 slots) on a small survey,
against FULL storage (bitwise for FP32 slots) and against the oracle; prints one JSON line."""
import json
import os

import numpy as np

import driver as D
from paper_2304_05592_amd import binding as B
import oracle as O
import workloads as W


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main():
    lib = D.EmuLib(os.environ["AWE_EMU_SO"])
    wl = W.small_3d(n=(26, 20, 70), nbl=8, T=float(os.environ.get("CASE_T", "20")), nrec_side=6)
    sh = wl.shots[0]
    dd = W.synthetic_residual(sh.nt, len(sh.rec), wl.dt, wl.f0, 3)
    out = {"nt": sh.nt, "poisoned_gaps": lib.asan is not None}
    gs = {}
    for tag, st in (("full", B.Storage(B.STORE_FULL)), ("ckpt_fp32", B.Storage(B.STORE_CHECKPOINT, 3)),
                    ("ckpt_bf16", B.Storage(B.STORE_CHECKPOINT, 3, B.PREC_BF16))):
        plan = D.EmuPlan(lib, wl, storage=st)
        plan.set_checks(int(os.environ.get("CASE_CHECKS", "0")))   # 4: host-side launch checks
        g, v, d = plan.gradient(plan.pack([wl.m(0)]), plan.pack([wl.q(0)]), plan.pack([dd]), v=True, d=True)
        gs[tag] = (g, v, d)
        del plan
    kw = dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    g_ref = O.gradient(wl.m(0), wl.q(0), dd, **kw)
    d_ref = O.forward(wl.m(0), wl.q(0), **kw)
    out["fp32_slots_bitwise_full"] = all(np.array_equal(a, b) for a, b in zip(gs["full"], gs["ckpt_fp32"]))
    out["grad_rel_full"] = rel(gs["full"][0], g_ref)
    out["grad_rel_ckpt_fp32"] = rel(gs["ckpt_fp32"][0], g_ref)
    out["grad_rel_ckpt_bf16"] = rel(gs["ckpt_bf16"][0], g_ref)
    out["traces_rel"] = rel(gs["ckpt_fp32"][2], d_ref)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
