"""CPU build: the 2D checkpointed gradient of an uneven batch (three windows, per-shot nt, 3
slots) whose paired reversals run as two-level adjoint launches imaging from the recomputed
forward levels, under AddressSanitizer with the host launch checks on.  With FP32 slots
(restores by reference) the gradient, F^T dd and traces are bitwise the FULL-storage one-level
result; with BF16 slots bitwise the one-level BF16 result.  Prints one JSON line."""
import json
import os

import numpy as np

import driver as D
from paper_2304_05592_amd import binding as B
import workloads as W


def main():
    lib = D.EmuLib(os.environ["AWE_EMU_SO"])
    wl = W.small_2d(nz=30, windows=[40, 33, 51], T_per_shot=[32.0, 21.0, 26.0])
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 3 + i) for i, s in enumerate(wl.shots)]

    def grad(storage, tz, fusion, groups):
        plan = D.EmuPlan(lib, wl, storage=storage)
        plan.set_checks(4)   # host-side launch checks
        plan.set_groups(groups)
        plan.set_tiles(tz, 8, 0)
        plan.set_fusion(fusion)
        assert plan.get_tiles()[2] == fusion
        m = plan.pack([wl.m(w) for w in range(wl.nwindow)])
        q = plan.pack([wl.q(i) for i in range(wl.nshot)])
        return plan.gradient(m, q, plan.pack(dds), v=True, d=True)

    ref32 = grad(B.Storage(B.STORE_FULL), 16, 0, 1)
    ref16 = grad(B.Storage(B.STORE_CHECKPOINT, 3, B.PREC_BF16), 16, 0, 1)
    out = {"nt": [s.nt for s in wl.shots], "bitwise": {}}
    for name, st, ref, tz, groups in (("fp32_8_2", B.Storage(B.STORE_CHECKPOINT, 3), ref32, 8, 2),
                                      ("fp32_24_1", B.Storage(B.STORE_CHECKPOINT, 3), ref32, 24, 1),
                                      ("bf16_16_2", B.Storage(B.STORE_CHECKPOINT, 3, B.PREC_BF16), ref16, 16, 2)):
        r = grad(st, tz, 2, groups)   # 2: two levels per launch in the reversals
        out["bitwise"][name] = all(np.array_equal(a, b) for a, b in zip(r, ref))
    out["nonzero"] = bool(np.abs(ref32[0]).max() > 0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
