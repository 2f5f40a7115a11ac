"""Measure the float32 rounding floor of the oracle (writes tests/golden/fp32_floor.json).

The oracle is dtype-generic; run in float32 it takes the same steps with float32 rounding,
which bounds what an FP32 implementation of the paper's operators can be expected to reach
against the FP64 result.  Calls only the oracle and the seeded input generators:

  * Born traces J(m0) dm of two c2_grad shots (0 and 8), float32 oracle vs the FP64 samples
    of tests/golden/c2_born_full.npz, and their forward traces F(m0) q vs
    tests/golden/c2_grad_full.npz;
  * the F and J dot tests of the 2-shot small 2D survey with the GPU test's seeded vectors:
    float32 operators, FP64 inner products, |a - b| / max(|a|, |b|);
  * the probed gradient of c2_grad shots 0 and 8 with 8 Rademacher probes (float32 oracle vs
    the FP64 samples of tests/golden/c9_probed_full.npz);
  * the probed gradient of the 3D crop's shot with the same probes (vs
    tests/golden/c9_probed_crop_full.npz; asked for by name only, about half an hour).

Run from the repository root:  python tests/golden/measure_fp32_floor.py [c2_grad] [dots] [c9_probed] [c9_probed_crop]
(no argument: all; a subset updates only its entries of the record).
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLD = os.path.join(ROOT, "tests", "golden")
SHOTS = (0, 8)


def _born_and_forward(s):
    import oracle as O
    import workloads as W
    wl = W.make_config("c2_grad")
    sh = wl.shots[s]
    kw = dict(h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax, dtype=np.float32)
    m0 = wl.m(sh.window, background=True)
    dm = wl.m(sh.window) - m0
    t0 = time.perf_counter()
    jb = O.born(m0, wl.q(s), dm, sh.src, sh.rec, **kw)
    d = O.forward(m0, wl.q(s), sh.src, sh.rec, **kw)
    print(f"  shot {s}: {time.perf_counter() - t0:.1f} s", flush=True)
    return s, jb, d


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def c2_floor():
    born_gold = np.load(os.path.join(GOLD, "c2_born_full.npz"))
    fwd_gold = np.load(os.path.join(GOLD, "c2_grad_full.npz"))
    with mp.get_context("spawn").Pool(len(SHOTS)) as pool:
        res = pool.map(_born_and_forward, SHOTS)
    got_b, ref_b, got_d, ref_d = [], [], [], []
    for s, jb, d in res:
        ix = np.ix_(born_gold[f"trace_t_{s}"], born_gold[f"trace_r_{s}"])
        got_b.append(jb[ix].ravel())
        ref_b.append(born_gold[f"trace_value_{s}"].ravel())
        ix = np.ix_(fwd_gold[f"trace_t_{s}"], fwd_gold[f"trace_r_{s}"])
        got_d.append(d[ix].ravel())
        ref_d.append(fwd_gold[f"trace_value_{s}"].ravel())
    return {"shots": list(SHOTS),
            "born_traces_rel_l2": _rel(np.concatenate(got_b), np.concatenate(ref_b)),
            "forward_traces_rel_l2": _rel(np.concatenate(got_d), np.concatenate(ref_d))}


def dot_floor():
    """The GPU dot tests' operators and vectors, in the float32 oracle."""
    import oracle as O
    import workloads as W
    wl = W.small_2d(nshot=2)
    rng = np.random.default_rng(0)
    xs = [rng.standard_normal(s.nt).astype(np.float32) for s in wl.shots]
    ys = [rng.standard_normal((s.nt, len(s.rec))).astype(np.float32) for s in wl.shots]
    dm = W.random_field(wl.comp_shape(0), 1).astype(np.float32)
    m = wl.m(0)
    out = {}
    for dtype, tag in ((np.float32, "fp32"), (np.float64, "fp64")):
        kws = [dict(src=s.src, rec=s.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax, dtype=dtype)
               for s in wl.shots]
        fx = [O.forward(m, xs[i], **kws[i]) for i in range(2)]
        fty = [O.adjoint(m, ys[i], **kws[i]) for i in range(2)]
        a = sum(float(np.sum(fx[i].astype(np.float64) * ys[i])) for i in range(2))
        b = sum(float(np.sum(xs[i].astype(np.float64) * fty[i])) for i in range(2))
        out[f"F_dot_rel_{tag}"] = abs(a - b) / max(abs(a), abs(b))
        jdm = [O.born(m, wl.q(i), dm, **kws[i]) for i in range(2)]
        g = sum(O.gradient(m, wl.q(i), ys[i], **kws[i]).astype(np.float64) for i in range(2))
        a = sum(float(np.sum(jdm[i].astype(np.float64) * ys[i])) for i in range(2))
        b = float(np.sum(dm.astype(np.float64) * g))
        out[f"J_dot_rel_{tag}"] = abs(a - b) / max(abs(a), abs(b))
    return out


def _probed(s):
    import oracle as O
    import workloads as W
    spec = __import__("importlib.util").util.spec_from_file_location("mfs", os.path.join(GOLD, "make_full_size.py"))
    G = __import__("importlib.util").util.module_from_spec(spec)
    spec.loader.exec_module(G)
    wl = W.make_config("c2_grad")
    sh = wl.shots[s]
    C, sw = G.probe_table(max(x.nt for x in wl.shots))
    t0 = time.perf_counter()
    g = O.gradient_probed(wl.m(sh.window, background=True), wl.q(s), G.residual(wl, s),
                          C=C[:, :sh.nt].astype(np.float64), s=sw, src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt,
                          nbl=wl.nbl, vref=wl.vmax, dtype=np.float32)
    print(f"  probed shot {s}: {time.perf_counter() - t0:.1f} s", flush=True)
    return s, g


def probed_floor():
    gold = np.load(os.path.join(GOLD, "c9_probed_full.npz"))
    shots = tuple(int(s) for s in gold["shots"])
    with mp.get_context("spawn").Pool(len(shots)) as pool:
        res = sorted(pool.map(_probed, shots), key=lambda r: r[0])
    g = sum(r[1].astype(np.float64) for r in res)
    return {"shots": list(shots), "probes": int(gold["probes"]),
            "gradient_rel_l2": _rel(g.ravel()[gold["grad_index_0"]], gold["grad_value_0"])}


def probed_crop_floor():
    import oracle as O
    import workloads as W
    spec = __import__("importlib.util").util.spec_from_file_location("mfs", os.path.join(GOLD, "make_full_size.py"))
    G = __import__("importlib.util").util.module_from_spec(spec)
    spec.loader.exec_module(G)
    gold = np.load(os.path.join(GOLD, "c9_probed_crop_full.npz"))
    wl = W.make_config("c5_crop")
    sh = wl.shots[0]
    C, sw = G.probe_table(sh.nt)
    t0 = time.perf_counter()
    g = O.gradient_probed(wl.m(0, background=True), wl.q(0), G.residual(wl, 0), C=C.astype(np.float64), s=sw,
                          src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax, dtype=np.float32)
    print(f"  probed crop: {time.perf_counter() - t0:.1f} s", flush=True)
    return {"probes": int(gold["probes"]),
            "gradient_rel_l2": _rel(g.astype(np.float64).ravel()[gold["grad_index_0"]], gold["grad_value_0"])}


def main():
    parts = sys.argv[1:] or ["c2_grad", "dots", "c9_probed"]
    path = os.path.join(GOLD, "fp32_floor.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec["what"] = "float32-emulated oracle against the FP64 oracle (rel-L2) and its own dot tests"
    t0 = time.perf_counter()
    if "c2_grad" in parts:
        rec["c2_grad"] = c2_floor()
    if "dots" in parts:
        rec["small_2d_dot_tests"] = dot_floor()
    if "c9_probed" in parts:
        rec["c9_probed"] = probed_floor()
    if "c9_probed_crop" in parts:
        rec["c9_probed_crop"] = probed_crop_floor()
    rec["seconds_last_run"] = round(time.perf_counter() - t0, 1)
    rec.pop("seconds", None)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
