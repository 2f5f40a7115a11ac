"""CPU build: the launch sequence of the 3D checkpointed-gradient GPU test (FULL FP32, then
CHECKPOINT with 4 FP32 slots, 26 x 20 x 70 physical grid + 8-cell border, default launch
shape), checked by AddressSanitizer with poisoned gaps between workspace sub-buffers; the
two gradients must agree bit for bit."""
import os
import sys
import time

import numpy as np

import driver as D
from paper_2304_05592_amd import binding as B
import workloads as W


def main():
    lib = D.EmuLib(os.environ["AWE_EMU_SO"])
    print("asan poisoning:", lib.asan is not None, flush=True)
    wl = W.small_3d(n=(26, 20, 70), nbl=8, T=float(os.environ.get("CASE_T", "260")), nrec_side=6)
    dds = [W.synthetic_residual(wl.shots[s].nt, len(wl.shots[s].rec), wl.dt, wl.f0, 3 + s)
           for s in range(wl.nshot)]
    print("grid", wl.comp_shape(0), "nt", wl.shots[0].nt, flush=True)
    res = []
    for st in (B.Storage(B.STORE_FULL), B.Storage(B.STORE_CHECKPOINT, int(os.environ.get("CASE_SLOTS", "4")))):
        t0 = time.time()
        plan = D.EmuPlan(lib, wl, storage=st)
        if int(os.environ.get("CASE_CHECKS", "0")):
            plan.set_checks(int(os.environ["CASE_CHECKS"]))   # 4: host-side launch checks
        m = plan.pack([wl.m(0)])
        q = plan.pack([wl.q(s) for s in range(wl.nshot)])
        dd = plan.pack(dds)
        # CASE_VD=0: no F^T dd and no trace outputs (null pointers), as the GPU test calls it
        vd = os.environ.get("CASE_VD", "1") == "1"
        g, v, d = plan.gradient(m, q, dd, v=vd, d=vd)
        res.append((g, v, d) if vd else (g,))
        print(f"storage mode {st.mode}: |g| {np.abs(g).max():.6e} launches {lib.L.emu_launch_count()} "
              f"{time.time() - t0:.1f} s", flush=True)
        del plan
    for name, a, b in zip("gvd", res[0], res[1]):
        same = np.array_equal(a, b)
        print(f"{name}: bitwise equal {same}; max diff {np.max(np.abs(a - b)):.3e}", flush=True)
        assert same, name
    print("CASE OK", flush=True)


if __name__ == "__main__":
    main()
