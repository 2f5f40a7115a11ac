"""Write the full-size parity fixtures (sampled oracle outputs) under tests/golden/.

Calls only the oracle and the seeded input generators.  For each workload the
oracle runs at full size in FP64 (the forward at the background model, the
adjoint-state gradient for a seeded synthetic residual per shot, summed over
shots in ascending order) and a seeded sample of the outputs is stored:

  c2_grad_full.npz    16 shots on the 421 x 730 grid, 3638 samples per shot
  c4_uneven_full.npz  64 shots, each on its own window (widths 256..1024, 1.0..2.5 s)
  c5_crop_full.npz    the 64^3 crop of the 3D model (144^3 with the sponge)
  c2_born_full.npz    Born traces J(m0) dm of the 16 c2_grad shots, dm = m - m0 (the
                      model minus its smoothed background, float32)
  c3_autograd_full.npz  shots 0 and 31 of the 32 c3_autograd shots on the 592 x 1104 grid,
                      5191 samples per shot (a stated subset: the oracle takes minutes per
                      shot at this size)
  c9_probed_full.npz  the probed gradient of shots 0 and 8 of the c2_grad survey with
                      PROBES Rademacher probes (table seed PROBE_SEED, columns = local levels)
  c9_probed_crop_full.npz  the probed gradient of the 3D crop's shot (144^3 with the sponge,
                      nt 2308) with the same probes
  c6_timelapse_full.npz  all 60 shots of the 15-vintage time-lapse iteration (336 x 592 grid,
                      nt 2505): the gradient with respect to each vintage's wavespeed v at the
                      starting model (chain rule of m = 1/v^2 applied to J^T dd)
  c7_timelapse_rock_full.npz  all 60 shots of the reservoir-rock time-lapse iteration: the
                      gradient with respect to each vintage's CO2 saturation at zero
                      saturation (rock physics R, m = 1/v^2, J^T dd)

Gradient samples are flat indices into each window's computational grid (the
same number per window); trace samples are every TIME_STRIDE-th time sample of
every REC_STRIDE-th receiver.

Run from the repository root:
    python tests/golden/make_full_size.py [c2_grad] [c4_uneven] [c5_crop] [c2_born] [c3_autograd] [c9_probed]
                                          [c9_probed_crop] [c6_timelapse] [c7_timelapse_rock]
The 2D sets take minutes on 8 cores, each 3D crop set about half an hour.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RESIDUAL_SEED = 1000      # synthetic residual of shot s uses seed RESIDUAL_SEED + s
SAMPLE_SEED = 20230411
N_GRAD_SAMPLES = 4096
REC_STRIDE = {"c2_grad": 40, "c4_uneven": 64, "c5_crop": 64, "c3_autograd": 64, "c6_timelapse": 64,
              "c7_timelapse_rock": 64}
SHOT_SUBSET = {"c3_autograd": (0, 31), "c9_probed": (0, 8)}   # shots whose full-size oracle results are stored
PROBES, PROBE_SEED = 8, 1
TIME_STRIDE = 32
SEGMENT = 64              # oracle recomputation segment (result does not depend on it)


def residual(wl, s):
    import workloads as W
    sh = wl.shots[s]
    return W.synthetic_residual(sh.nt, len(sh.rec), wl.dt, wl.f0, RESIDUAL_SEED + s)


def _shot(args):
    name, s = args
    import oracle as O
    import workloads as W
    wl = W.make_config(name)
    sh = wl.shots[s]
    kw = dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    t0 = time.perf_counter()
    g, d = O.gradient(wl.m(sh.window, background=True), wl.q(s), residual(wl, s), segment=SEGMENT,
                      return_traces=True, **kw)
    print(f"  {name} shot {s}: {time.perf_counter() - t0:.1f} s", flush=True)
    return s, g, d


def probe_table(nt):
    import workloads as W
    return W.probe_table("rademacher", nt, r=PROBES, seed=PROBE_SEED)


def _probed_shot(s):
    import oracle as O
    import workloads as W
    wl = W.make_config("c2_grad")
    sh = wl.shots[s]
    C, sw = probe_table(max(x.nt for x in wl.shots))
    t0 = time.perf_counter()
    g = O.gradient_probed(wl.m(sh.window, background=True), wl.q(s), residual(wl, s),
                          C=C[:, :sh.nt].astype(np.float64), s=sw, src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt,
                          nbl=wl.nbl, vref=wl.vmax)
    print(f"  c9_probed shot {s}: {time.perf_counter() - t0:.1f} s", flush=True)
    return s, g


def make_probed(workers):
    import workloads as W
    wl = W.make_config("c2_grad")
    shots = SHOT_SUBSET["c9_probed"]
    with mp.get_context("spawn").Pool(min(workers, len(shots))) as pool:
        res = sorted(pool.map(_probed_shot, shots), key=lambda r: r[0])
    g = np.zeros(wl.comp_shape(0))
    for _, g_s in res:
        g = g + g_s
    rng = np.random.default_rng(SAMPLE_SEED)
    gidx = np.sort(rng.choice(g.size, size=N_GRAD_SAMPLES, replace=False))
    path = os.path.join(ROOT, "tests", "golden", "c9_probed_full.npz")
    np.savez_compressed(path, shots=np.asarray(shots, dtype=np.int64), probes=PROBES, probe_seed=PROBE_SEED,
                        grad_index_0=gidx.astype(np.int64), grad_value_0=g.ravel()[gidx],
                        grad_norm=np.linalg.norm(g))
    print(f"wrote {path}", flush=True)


def make_probed_crop():
    import oracle as O
    import workloads as W
    wl = W.make_config("c5_crop")
    sh = wl.shots[0]
    C, sw = probe_table(sh.nt)
    t0 = time.perf_counter()
    g = O.gradient_probed(wl.m(0, background=True), wl.q(0), residual(wl, 0), C=C.astype(np.float64), s=sw,
                          src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    print(f"  c9_probed_crop: {time.perf_counter() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    gidx = np.sort(rng.choice(g.size, size=N_GRAD_SAMPLES, replace=False))
    path = os.path.join(ROOT, "tests", "golden", "c9_probed_crop_full.npz")
    np.savez_compressed(path, probes=PROBES, probe_seed=PROBE_SEED, grad_index_0=gidx.astype(np.int64),
                        grad_value_0=g.ravel()[gidx], grad_norm=np.linalg.norm(g))
    print(f"wrote {path}", flush=True)


def born_perturbation(wl, w=0):
    """dm = m - m0 of window w in float32 (the true model minus the smoothed background)."""
    return wl.m(w) - wl.m(w, background=True)


def _born_shot(s):
    import oracle as O
    import workloads as W
    wl = W.make_config("c2_grad")
    sh = wl.shots[s]
    t0 = time.perf_counter()
    d = O.born(wl.m(sh.window, background=True), wl.q(s), born_perturbation(wl, sh.window), sh.src,
               sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    print(f"  c2_born shot {s}: {time.perf_counter() - t0:.1f} s", flush=True)
    return s, d


def make_born(workers):
    import workloads as W
    wl = W.make_config("c2_grad")
    with mp.get_context("spawn").Pool(min(workers, wl.nshot)) as pool:
        res = sorted(pool.map(_born_shot, range(wl.nshot)), key=lambda r: r[0])
    out = {}
    for s, d in res:
        nt, nrec = d.shape
        ti = np.arange(0, nt, TIME_STRIDE)
        ri = np.arange(0, nrec, REC_STRIDE["c2_grad"])
        out[f"trace_t_{s}"] = ti.astype(np.int64)
        out[f"trace_r_{s}"] = ri.astype(np.int64)
        out[f"trace_value_{s}"] = d[np.ix_(ti, ri)]
    path = os.path.join(ROOT, "tests", "golden", "c2_born_full.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}", flush=True)


def timelapse_models(wl):
    """The float32 inputs of a time-lapse gradient on each vintage's computational grid, as the
    consumer builds them: (parameter, wavespeed) per window.  c6: the starting wavespeed v0
    (parameter = wavespeed); c7: zero CO2 saturation (parameter) of the reservoir rock, whose
    wavespeed is R(0, vp, rho, phi), plus the rock arrays."""
    import oracle as O
    import workloads as W
    ext = lambda a: W.extend_edge(np.asarray(a, dtype=np.float32), wl.nbl)
    if "vp" not in wl.extra:
        v = [ext(wl.v0[w]) for w in range(wl.nwindow)]
        return v, v, None
    rock = tuple(ext(wl.extra[k]) for k in ("vp", "rho", "phi"))
    sw = [np.zeros(wl.comp_shape(w), dtype=np.float32) for w in range(wl.nwindow)]
    return sw, [O.patchy(sw[w], *rock)[0] for w in range(wl.nwindow)], rock


def _timelapse_shot(args):
    name, s = args
    import oracle as O
    import workloads as W
    wl = W.make_config(name)
    sh = wl.shots[s]
    _, v, _ = timelapse_models(wl)
    kw = dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    t0 = time.perf_counter()
    g, d = O.gradient(O.slowness2(v[sh.window]), wl.q(s), residual(wl, s), segment=SEGMENT,
                      return_traces=True, **kw)
    print(f"  {name} shot {s}: {time.perf_counter() - t0:.1f} s", flush=True)
    return s, g, d


def make_timelapse(name, workers):
    """J^T dd per shot at each vintage's starting model (FP64), summed over the vintage's shots
    in ascending order, then the chain rules: g_v = -2 g_m / v^3, and for the rock workload
    g_sw = (dR/dsw) g_v (the oracle's complex-step pullback of R)."""
    import oracle as O
    import workloads as W
    wl = W.make_config(name)
    par, v, rock = timelapse_models(wl)
    jobs = [(name, s) for s in range(wl.nshot)]
    with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
        res = pool.map(_timelapse_shot, jobs)
    res.sort(key=lambda r: r[0])
    gm = [np.zeros(wl.comp_shape(w)) for w in range(wl.nwindow)]
    for s, g_s, _ in res:
        w = wl.shots[s].window
        gm[w] = gm[w] + g_s
    gs = [O.velocity_gradient(v[w], gm[w]) for w in range(wl.nwindow)]
    if rock is not None:
        gs = [O.patchy_vjp(par[w], *rock, gs[w]) for w in range(wl.nwindow)]
    rng = np.random.default_rng(SAMPLE_SEED)
    per = max(64, N_GRAD_SAMPLES // wl.nwindow)
    out = {"shots": np.arange(wl.nshot, dtype=np.int64)}
    for w, g in enumerate(gs):
        gidx = np.sort(rng.choice(g.size, size=min(per, g.size), replace=False))
        out[f"grad_index_{w}"] = gidx.astype(np.int64)
        out[f"grad_value_{w}"] = g.ravel()[gidx]
    for s, _, d in res:
        ti = np.arange(0, d.shape[0], TIME_STRIDE)
        ri = np.arange(0, d.shape[1], REC_STRIDE[name])
        out[f"trace_t_{s}"] = ti.astype(np.int64)
        out[f"trace_r_{s}"] = ri.astype(np.int64)
        out[f"trace_value_{s}"] = d[np.ix_(ti, ri)]
    path = os.path.join(ROOT, "tests", "golden", f"{name}_full.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}", flush=True)


def make(name, workers):
    import workloads as W
    wl = W.make_config(name)
    shots = SHOT_SUBSET.get(name, tuple(range(wl.nshot)))
    jobs = [(name, s) for s in shots]
    if workers > 1 and len(jobs) > 1:
        with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
            res = pool.map(_shot, jobs)
    else:
        res = [_shot(j) for j in jobs]
    res.sort(key=lambda r: r[0])
    gs = [np.zeros(wl.comp_shape(w)) for w in range(wl.nwindow)]
    for s, g_s, _ in res:         # ascending shot order within each window
        w = wl.shots[s].window
        gs[w] = gs[w] + g_s
    rng = np.random.default_rng(SAMPLE_SEED)
    per = max(64, N_GRAD_SAMPLES // wl.nwindow)
    out = {"shots": np.asarray(shots, dtype=np.int64)}
    for w, g in enumerate(gs):
        gidx = np.sort(rng.choice(g.size, size=min(per, g.size), replace=False))
        out[f"grad_index_{w}"] = gidx.astype(np.int64)
        out[f"grad_value_{w}"] = g.ravel()[gidx]
    for s, _, d in res:
        nt, nrec = d.shape
        ti = np.arange(0, nt, TIME_STRIDE)
        ri = np.arange(0, nrec, REC_STRIDE[name])
        out[f"trace_t_{s}"] = ti.astype(np.int64)
        out[f"trace_r_{s}"] = ri.astype(np.int64)
        out[f"trace_value_{s}"] = d[np.ix_(ti, ri)]
    path = os.path.join(ROOT, "tests", "golden", f"{name}_full.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}", flush=True)


def main():
    names = sys.argv[1:] or ["c2_grad", "c4_uneven", "c5_crop"]
    workers = min(8, len(os.sched_getaffinity(0)))
    for name in names:
        t0 = time.perf_counter()
        if name == "c2_born":
            make_born(workers)
        elif name == "c9_probed":
            make_probed(workers)
        elif name == "c9_probed_crop":
            make_probed_crop()
        elif name in ("c6_timelapse", "c7_timelapse_rock"):
            make_timelapse(name, workers)
        else:
            make(name, workers)
        print(f"{name}: {time.perf_counter() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
