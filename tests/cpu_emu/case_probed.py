"""CPU build: the probed gradient (PROBED storage, awe_gradient_probed) against the oracle's
gradient_probed on an uneven 2D batch (three shots, two windows, different nt), with
Rademacher probes and with the identity table (which gives the exact gradient), under
AddressSanitizer with poisoned gaps between the workspace's sub-buffers; the probed gradient
does not depend on the launch shape, the number of levels per launch or the shot grouping."""
import json
import os

import numpy as np

import driver as D
from paper_2304_05592_amd import binding as B
import oracle as O
import workloads as W


def shot_kwargs(wl, i):
    sh = wl.shots[i]
    return dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)


def oracle_probed(wl, dds, C, s):
    """Sum over shots of the oracle's probed gradient, per window; column k = local level k."""
    gs = [np.zeros(wl.comp_shape(w)) for w in range(wl.nwindow)]
    for i, sh in enumerate(wl.shots):
        gs[sh.window] += O.gradient_probed(wl.m(sh.window), wl.q(i), dds[i], C=C[:, :sh.nt], s=s,
                                           **shot_kwargs(wl, i))
    return gs


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main():
    lib = D.EmuLib(os.environ["AWE_EMU_SO"])
    wl = W.small_2d(windows=[70, 130, 96], T_per_shot=[60.0, 36.0, 48.0])
    dds = [W.synthetic_residual(s.nt, len(s.rec), wl.dt, wl.f0, 3 + i) for i, s in enumerate(wl.shots)]
    max_nt = max(s.nt for s in wl.shots)
    out = {}
    for name, (C, s) in (("rademacher", W.probe_table("rademacher", max_nt, r=4, seed=11)),
                         ("identity", W.probe_table("identity", max_nt))):
        r = C.shape[0]
        plan = D.EmuPlan(lib, wl, storage=B.Storage(B.STORE_PROBED, r))
        plan.set_checks(4)   # host-side launch checks
        m = plan.pack([wl.m(w) for w in range(wl.nwindow)])
        q = plan.pack([wl.q(i) for i in range(wl.nshot)])
        dd = plan.pack(dds)
        g, v, d = plan.gradient_probed(m, q, dd, C, s, v=True, d=True)
        ref = oracle_probed(wl, dds, C.astype(np.float64), s)
        got = [g[o:o + int(np.prod(sh))].reshape(sh) for o, sh in zip(plan.layout.m_offset, plan.layout.windows)]
        out[name] = max(rel(a, b) for a, b in zip(got, ref))
        if name == "identity":
            exact = [np.zeros(wl.comp_shape(w)) for w in range(wl.nwindow)]
            for i, sh in enumerate(wl.shots):
                exact[sh.window] += O.gradient(wl.m(sh.window), wl.q(i), dds[i], **shot_kwargs(wl, i))
            out["identity_vs_exact"] = max(rel(a, b) for a, b in zip(got, exact))
        else:
            plan.set_tiles(8, 8, 0)
            plan.set_groups(3)
            g2 = plan.gradient_probed(m, q, dd, C, s)[0]
            # two levels per launch in both sweeps (uneven nt: odd and even level counts)
            plan.set_tiles(16, 8, 0)
            plan.set_fusion(3)
            plan.set_groups(1)
            g3 = plan.gradient_probed(m, q, dd, C, s)[0]
            # the autotuner runs the probe kernels (coefficients read from the sums the probed
            # direction does not write); whatever it picks gives the same bits
            plan.set_groups(1)
            plan.autotune(m, q, dd, probe_steps=4)
            g4 = plan.gradient_probed(m, q, dd, C, s)[0]
            out["shape_invariant"] = bool(np.array_equal(g, g2) and np.array_equal(g, g3) and np.array_equal(g, g4))
        print(name, out, flush=True)
    # 3D: one shot with receivers injected by the post-step pass (its part of A_j is added there)
    w3 = W.small_3d(n=(26, 20, 30), nbl=8, T=40.0, nrec_side=6)
    sh = w3.shots[0]
    dd3 = W.synthetic_residual(sh.nt, len(sh.rec), w3.dt, w3.f0, 5)
    for name, (C, s) in (("rademacher3d", W.probe_table("rademacher", sh.nt, r=4, seed=12)),):
        plan = D.EmuPlan(lib, w3, storage=B.Storage(B.STORE_PROBED, C.shape[0]))
        plan.set_checks(4)
        g = plan.gradient_probed(plan.pack([w3.m(0)]), plan.pack([w3.q(0)]), plan.pack([dd3]), C, s)[0]
        ref = O.gradient_probed(w3.m(0), w3.q(0), dd3, C=C.astype(np.float64), s=s, **shot_kwargs(w3, 0))
        out[name] = rel(g.reshape(ref.shape), ref)
        plan.set_tiles(32, 4, 7)
        g2 = plan.gradient_probed(plan.pack([w3.m(0)]), plan.pack([w3.q(0)]), plan.pack([dd3]), C, s)[0]
        plan.autotune(plan.pack([w3.m(0)]), plan.pack([w3.q(0)]), plan.pack([dd3]), probe_steps=2)
        g3 = plan.gradient_probed(plan.pack([w3.m(0)]), plan.pack([w3.q(0)]), plan.pack([dd3]), C, s)[0]
        out["shape_invariant3d"] = bool(np.array_equal(g, g2) and np.array_equal(g, g3))
        print(name, out, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
