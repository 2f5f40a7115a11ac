"""Benchmark of the acoustic forward / adjoint-state gradient path on one MI355X.

Default (the headline line): the batched 2D gradient workload c2_grad — 650 x 341 physical
grid at 6.25 m (+40-cell damping border), layered 1.5-4.5 km/s with a 5 % smoothed random
perturbation, 16 shots, 650 receivers, T = 1.8 s, full FP32 wavefield storage.  One step =
the whole hot path over the 16 shots: forward solve keeping the wavefield in HBM, residual
r = d - d_obs with the misfit 1/2 ||r||^2 in FP64, and the reverse sweep g = J^T r (adjoint
solve + imaging condition, FP64 accumulation), all in the library's HIP kernels, captured
once into a HIP graph and replayed.  Inputs are resident in HBM before the timed region.

Other workloads (--config): c1_fwd (single-shot 2D forward, 201 x 101, graph vs eager),
c3_autograd (torch.autograd through the wave operator with 16
checkpoint slots per shot, 32 shots), c6_timelapse (15-vintage crosswell time-lapse gradient
with respect to wavespeed, 4 sampled shots per vintage), c7_timelapse_rock (the same iteration
with respect to CO2 saturation through the patchy rock physics), c8_born (batched Born
modelling of the c2_grad survey), c4_uneven (64 uneven windows, forward, batched vs 64
sequential single-shot runs), c5_3d (256^3, FULL BF16 / FP16 storage gradient).

Prints one JSON line.  Gpts/s = sum over shots of N_s (nt_s - 1) per step / step time
(N_s = computational-grid points of the shot).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "Gpts/s (fwd+adjoint gradient) batched vs single-shot; % HBM roofline"
# Algorithmic HBM bytes per point-update of each step (FP32 fields, FP64 accumulator): the
# per-step table of the design notes.  A launch that advances two time levels performs two
# point-updates per grid point, so its algorithmic bytes are twice these.
BYTES = {
    ("forward", "none"): 16,   # read u^{k-1}, u^{k-2}, coef; write u^k
    ("forward", "fp32"): 20,   # + stored copy of u^k
    ("forward", "16bit"): 18,  # + 16-bit stored copy
    ("adjoint", "none"): 16,   # read w^{j+1}, w^{j+2}, coef; write w^j
    ("adjoint", "fp32"): 36,   # + stored u^j (4) + accumulator read and write (16)
    ("adjoint", "16bit"): 34,  # + 16-bit stored u^j (2) + accumulator (16)
    ("adjoint", "buffers"): 36,  # u^j from the recomputed forward buffer (4) + accumulator
    ("born", "none"): 32,       # read u^{k-1}, u^{k-2}, du^{k-1}, du^{k-2}, coef, dm; write u^k, du^k
}
# What a two-level launch itself moves per grid point (inputs read once, both new levels
# written): reported beside the algorithmic figure, not used for the roofline fraction.
FUSED_BYTES = {
    ("forward", "none"): 20,   # read u^{k-1}, u^{k-2}, coef; write u^k, u^{k+1}
    ("forward", "fp32"): 28,   # + stored copies of u^k and u^{k+1}
    ("adjoint", "none"): 20,   # read w^{j+1}, w^{j+2}, coef; write w^j, w^{j-1}
    ("adjoint", "fp32"): 44,   # read w^{j+1}, w^{j+2}, coef, stored u^j, u^{j-1}, acc; write w^j, w^{j-1}, acc
    ("adjoint", "buffers"): 44,  # the same with u^j, u^{j-1} from the recomputed forward levels
    ("born", "none"): 40,      # read u^{k-1}, u^{k-2}, du^{k-1}, du^{k-2}, coef, dm; write u, du at k and k+1
}
# Per-launch event timing records two HIP events around a launch; a profiler's counter pass over
# tens of thousands of such records once ended in a host fault inside the runtime, so the eager
# timing samples at most this many launches (evenly strided) and counter passes run the
# event-free --counter-step program.
MAX_TIMED_LAUNCHES = 4096
TRAFFIC_NOTE = ("rocprofv3 FETCH_SIZE + WRITE_SIZE per launch (TCC-to-fabric bytes: L2 misses served by "
                "the Infinity Cache are counted too), each scaled by the counter's reading for a 1 GiB "
                "device copy")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2_grad",
                    choices=["c1_fwd", "c2_grad", "c3_autograd", "c4_uneven", "c5_3d", "c6_timelapse", "c9_probed", "c9_probed_3d",
                             "c7_timelapse_rock", "c8_born"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probes", type=int, default=8, help="c9_probed: time-axis probes (1..64)")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of a graph")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=600, help="time steps of the oracle sample")
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp16", "fp32"],
                    help="stored-wavefield precision of the 3D workload")
    ap.add_argument("--tiles", default=None,
                    help="fixed launch shape instead of the autotuner, e.g. tz=32 or tz=32,atz=16,fusion=3 "
                         "(tz/ty/bz both directions, atz/aty/abz adjoint steps only; two levels per "
                         "launch: fusion 1 forward, 2 reverse sweep, 3 both)")
    ap.add_argument("--groups", type=int, default=0,
                    help="shot groups per plan (0: automatic, sized to the last-level cache)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the plain device-to-device copy probe (PMC calibration)")
    ap.add_argument("--counter-step", action="store_true",
                    help="only run one eager gradient step of c2_grad (or c5_3d with --config), "
                         "without timing events (for profiler counter passes)")
    args = ap.parse_args()
    if args.tiles:
        args.tiles = {k: int(v) for k, v in (kv.split("=") for kv in args.tiles.split(","))}
    return args


def copy_probe(nbytes=1 << 30, reps=5):
    """Bandwidth of a plain device-to-device copy (torch) of nbytes: read + write bytes / time."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    sync()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_copied": nbytes, "GBs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4)}


def traffic_record(workload, kernel_file, kernel_name, launch_points, shape=None):
    """HBM bytes per launch measured by rocprofv3 PMC counters (profiles/traffic_<workload>.json),
    or None when the record is missing, was taken for another kernel, size or launch shape, or the
    kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    src = os.path.join(ROOT, "paper_2304_05592_amd", "csrc", kernel_file)
    if not os.path.exists(path) or not os.path.exists(src):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    if rec.get("kernel") != kernel_name or rec.get("launch_points") != launch_points:
        return None
    if shape is not None and rec.get("shape") != shape:
        return None
    return rec.get("hbm_bytes_per_launch")


def sync():
    import torch
    torch.cuda.synchronize()


def fusion_of(tiles):
    """Two-levels-per-launch mode of a launch shape (bit 0 forward, bit 1 reverse sweep); the
    older key levels_per_launch=2 means both."""
    if not tiles:
        return 0
    if "fusion" in tiles:
        return int(tiles["fusion"])
    return 3 if tiles.get("levels_per_launch", 1) == 2 else 0


def apply_tiles(plan, t):
    """Set a fixed launch shape: tz / ty / bz for both directions, atz / aty / abz (optional) for
    the adjoint steps only, and the fusion mode; returns the shapes in effect."""
    plan.set_tiles(t.get("tz", 32), t.get("ty", 8), t.get("bz", 0))
    if any(k in t for k in ("atz", "aty", "abz")):
        plan.set_tiles(t.get("atz", t.get("tz", 32)), t.get("aty", t.get("ty", 8)), t.get("abz", t.get("bz", 0)),
                       dirs=2)
    plan.set_fusion(fusion_of(t))
    return plan.get_tiles()


def adjoint_tz(tiles):
    """Row count of the adjoint steps' tiles in a launch-shape record."""
    return tiles.get("adjoint", {}).get("tz", tiles.get("atz", tiles.get("tz")))


def choose_tiles(plan, args, m, q, dd, ws=None):
    """Fixed launch shape from --tiles, else the autotuner's choice (None with --no-autotune)."""
    if args.tiles:
        return apply_tiles(plan, args.tiles)
    if args.no_autotune:
        return None
    return plan.autotune(m, q, dd, probe_steps=32, ws=ws)[0]


def choose_pass_tiles(plan, args, run, fusions=(0,)):
    """Launch shape of a benchmark that times one kind of pass (forward only, Born): fixed by
    --tiles, else one timed eager pass per 2D tile height and forward fusion mode (the
    library's autotuner scores forward and adjoint levels together, and no Born levels)."""
    if args.tiles or args.no_autotune:
        return choose_tiles(plan, args, None, None, None)
    best = None
    for tz in (8, 16, 24, 32, 64):
        for fu in fusions:
            if fu and tz == 64:                # two-level kernels exist for 8, 16, 24, 32 rows
                continue
            plan.set_tiles(tz)
            plan.set_fusion(fu)
            run()
            sync()
            t0 = time.perf_counter()
            run()
            sync()
            t = time.perf_counter() - t0
            if best is None or t < best[0]:
                best = (t, tz, fu)
    plan.set_tiles(best[1])
    plan.set_fusion(best[2])
    return {"tz": best[1], "ty": 8, "bz": 0, "fusion": best[2]}


def make_plan(wl, storage, shots):
    import paper_2304_05592_amd as A
    geoms = [A.ShotGeometry(wl.shots[s].window, wl.shots[s].nt, wl.shots[s].src, wl.shots[s].rec)
             for s in shots]
    windows = [wl.comp_shape(w) for w in range(wl.nwindow)]
    return A.Plan(wl.ndim, wl.h, wl.dt, wl.nbl, wl.vmax, windows, geoms, storage=storage,
                  damp_vref=wl.vmax)


def points_of(wl, shots):
    per_step = sum(int(np.prod(wl.comp_shape(wl.shots[s].window))) * (wl.shots[s].nt - 1) for s in shots)
    per_launch = sum(int(np.prod(wl.comp_shape(wl.shots[s].window))) for s in shots)
    return per_step, per_launch


def kernel_table(prof, launch_points, kinds, fused=0, mixed=None):
    """Per kernel class: launches, average event time and achieved algorithmic GB/s.  A class
    that runs two levels per launch (fused: bit 0 forward, bit 1 adjoint) performs two
    point-updates per grid point and launch; its own (fused) bytes are reported beside."""
    out = {}
    for name, kind in kinds.items():
        cnt, ms = prof[name]
        if cnt == 0:
            continue
        avg_ms = ms / cnt
        if mixed and name in mixed:
            # launches of one or two levels: (two-level launches, one-level launches) per run,
            # from the schedule; priced by the levels they advance
            pairs, singles = mixed[name]
            lv = (2 * pairs + singles) / (pairs + singles)
            b = round(BYTES[(name, kind)] * lv * launch_points)
            fb = round((FUSED_BYTES[(name, kind)] * pairs + BYTES[(name, kind)] * singles) / (pairs + singles)
                       * launch_points)
            out[name] = {"launches_timed": cnt, "avg_us": round(avg_ms * 1e3, 3),
                         "bytes_per_point_update": BYTES[(name, kind)], "levels_per_launch": round(lv, 4),
                         "bytes_per_launch": b, "achieved_GBs": round(b / (avg_ms * 1e-3) / 1e9, 1),
                         "fused_bytes_per_point": FUSED_BYTES[(name, kind)], "fused_bytes_per_launch": fb,
                         "fused_GBs": round(fb / (avg_ms * 1e-3) / 1e9, 1)}
            continue
        # Born runs two levels per launch with the forward solves
        two = bool(fused & (1 if name in ("forward", "born") else 2 if name == "adjoint" else 0)) and \
            (name, kind) in FUSED_BYTES
        levels = 2 if two else 1
        b = BYTES[(name, kind)] * levels * launch_points
        k = {"launches_timed": cnt, "avg_us": round(avg_ms * 1e3, 3), "bytes_per_point_update": BYTES[(name, kind)],
             "levels_per_launch": levels, "bytes_per_launch": b,
             "achieved_GBs": round(b / (avg_ms * 1e-3) / 1e9, 1)}
        if two:
            fb = FUSED_BYTES[(name, kind)] * launch_points
            k["fused_bytes_per_point"] = FUSED_BYTES[(name, kind)]
            k["fused_bytes_per_launch"] = fb
            k["fused_GBs"] = round(fb / (avg_ms * 1e-3) / 1e9, 1)
        out[name] = k
    return out


def refresh_rates(k):
    """Recompute a kernel entry's rates after its avg_us changed."""
    s = k["avg_us"] * 1e-6
    k["achieved_GBs"] = round(k["bytes_per_launch"] / s / 1e9, 1)
    if "fused_bytes_per_launch" in k:
        k["fused_GBs"] = round(k["fused_bytes_per_launch"] / s / 1e9, 1)


def roofline_of(kernels, names, fused_bytes=False):
    # the dominant kernel is the one with the larger share of the step's time (launches can
    # differ when one direction runs two levels per launch); fused_bytes: a two-level launch is
    # priced at the bytes it must move itself (where twice the per-step figure is no lower bound)
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches_timed"])
    ach = kernels[dom]["fused_GBs" if fused_bytes and "fused_GBs" in kernels[dom] else "achieved_GBs"]
    out = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None, "kernel": names[dom]}
    if "fused_GBs" in kernels[dom]:
        out["fused_bytes_achieved"] = kernels[dom]["fused_GBs"]
        out["fused_bytes_frac"] = round(kernels[dom]["fused_GBs"] / PEAK_HBM_GBS, 4)
        if not fused_bytes:
            out["accounting"] = ("achieved counts the per-step table's bytes of every level the launch "
                                 "advances; a two-level launch moves fewer (fused_bytes_achieved: inputs "
                                 "read once, the first level kept on chip), so achieved can exceed the peak")
    return out


def timed_gradient(run, args, kind):
    """Time the gradient step of a GradientRunner.  Region 1: one to three eager steps with HIP
    events around each sweep's step loop (the library's kernel timing: interval / launches, no
    event between launches).  Region 2 (headline, unless --no-graph): the step as two HIP graphs,
    forward sweep + residual and reverse sweep, replayed back to back for args.steps steps with
    HIP events between the segments; a kernel's average is its segment's time divided by its
    launches.  Returns (seconds per step, eager seconds per step, kernel table, timing note)."""
    n_eager = max(1, min(args.steps, 3))
    eager_sec, prof = run.run(n_eager, args.warmup, use_graph=False, profile=True)
    kernels = kernel_table(prof, run.launch_points, {"forward": kind, "adjoint": kind},
                           fused=fusion_of(run.tiles))
    if args.no_graph:
        return eager_sec, eager_sec, kernels, "HIP events around each sweep's step loop of the eager timed steps"
    run.capture()
    sec, seg = run.run(args.steps, args.warmup, use_graph=True, profile=True)
    nsteps = max(run.wl.shots[i].nt for i in run.shots) - 1
    for name, key in (("forward", "forward_ms"), ("adjoint", "backward_ms")):
        # launches of this class per step: one per time level, or per pair of levels
        n_l = run.groups * -(-nsteps // kernels[name]["levels_per_launch"])
        avg_ms = sum(seg[key]) / len(seg[key]) / n_l
        k = kernels[name]
        k["eager_event_us"] = k["avg_us"]
        k["avg_us"] = round(avg_ms * 1e3, 3)
        refresh_rates(k)
        k["segment_ms"] = round(sum(seg[key]) / len(seg[key]), 3)
    timing = ("HIP events on the launch stream between two graph segments (forward sweep + residual; "
              "reverse sweep) of every timed step: segment time / launches of its step kernel (the "
              "segment's auxiliary kernels included); eager_event_us = events around each sweep's step "
              "loop of an eager step, interval / launches")
    return sec, eager_sec, kernels, timing


class GradientRunner:
    """Forward (kept wavefield) + residual + reverse sweep on resident inputs."""

    def __init__(self, wl, shots, storage, autotune=True, tiles=None, groups=0):
        import torch
        import paper_2304_05592_amd as A
        self.A, self.torch = A, torch
        self.wl, self.shots = wl, list(shots)
        self.plan = make_plan(wl, storage, self.shots)
        p = self.plan
        self.m_true = p.pack([wl.m(w) for w in range(wl.nwindow)], "m")
        self.m0 = p.pack([wl.m(w, background=True) for w in range(wl.nwindow)], "m")
        self.q = p.pack([wl.q(s) for s in self.shots], "q")
        self.ws = p.workspace()
        self.d_obs = p.forward(self.m_true, self.q, ws=self.ws)
        self.d = torch.empty_like(self.d_obs)
        self.r = torch.empty_like(self.d_obs)
        self.g = torch.empty(p.layout.m_size, dtype=torch.float64, device="cuda")
        self.points, self.launch_points = points_of(wl, self.shots)
        self.tiles = None
        if tiles:
            self.tiles = apply_tiles(p, tiles)
        elif autotune:
            self.tiles, _ = p.autotune(self.m0, self.q, self.d_obs, probe_steps=32, ws=self.ws)
        self.groups = p.set_groups(groups)   # shot groups in effect (0: automatic)
        self.launch_points //= self.groups
        self.graph = None
        sync()

    def forward_part(self):
        p = self.plan
        p.forward(self.m0, self.q, d=self.d, keep=True, ws=self.ws)
        _, self.loss = self.A.residual(self.d, self.d_obs, r=self.r)

    def backward_part(self):
        self.plan.backward(self.m0, self.q, self.r, g=self.g, v=None, ws=self.ws)

    def step(self):
        self.forward_part()
        self.backward_part()

    def capture(self):
        """Capture the step as two HIP graphs: forward sweep + residual, and the reverse sweep."""
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.step()
        torch.cuda.current_stream().wait_stream(s)
        sync()
        self.graph = (torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph())
        with torch.cuda.graph(self.graph[0], stream=s):
            self.forward_part()
        with torch.cuda.graph(self.graph[1], stream=s):
            self.backward_part()
        sync()

    def replay(self, ev=None):
        if ev is not None:
            ev[0].record()
        self.graph[0].replay()
        if ev is not None:
            ev[1].record()
        self.graph[1].replay()
        if ev is not None:
            ev[2].record()

    def run(self, steps, warmup, use_graph, profile):
        """Seconds per step and, with profile: eager = kernel-timing summary; graph = event
        time of the two graph segments per step ({'forward_ms': [...], 'backward_ms': [...]})."""
        torch = self.torch
        for _ in range(warmup):
            self.replay() if use_graph else self.step()
        sync()
        if profile and not use_graph:
            # one timed interval per sweep (forward, reverse) of each shot group and step
            self.plan.profile_enable(2 * steps * self.groups + 64, 1)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)] \
            if profile and use_graph else None
        sync()
        t0 = time.perf_counter()
        for i in range(steps):
            if use_graph:
                self.replay(evs[i] if evs else None)
            else:
                self.step()
        sync()
        sec = (time.perf_counter() - t0) / steps
        prof = None
        if profile and not use_graph:
            prof = self.plan.profile_read()
            self.plan.profile_disable()
        if evs:
            prof = {"forward_ms": [e[0].elapsed_time(e[1]) for e in evs],
                    "backward_ms": [e[1].elapsed_time(e[2]) for e in evs]}
        return sec, prof

    def release(self):
        self.graph = None
        self.ws = None
        self.plan = None
        self.torch.cuda.empty_cache()


# ------------------------------------------------------------------------------ CPU baseline
def _oracle_worker(args):
    """Oracle gradient of one shot over its first n samples (runs in a worker process)."""
    name, s, n, dtype = args
    import workloads as W
    import oracle as O
    wl = W.make_config(name)
    sh = wl.shots[s]
    kw = dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax, dtype=dtype)
    m_true, m0 = wl.m(sh.window), wl.m(sh.window, background=True)
    q = wl.q(s)[:n]
    d_obs = O.forward(m_true, q, **kw)
    t1 = time.perf_counter()
    g = O.gradient(m0, q, O.forward(m0, q, **kw) - d_obs, **kw)
    t2 = time.perf_counter()
    npts = int(np.prod(wl.comp_shape(sh.window)))
    return npts * (n - 1), (t2 - t1), float(np.abs(g).max())


def _oracle_sample(name, wl, n, workers, dtype):
    import multiprocessing as mp
    jobs = [(name, s, min(n, wl.shots[s].nt), dtype) for s in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    return sum(r[0] for r in res), max(r[1] for r in res), wall, jobs[0][2]


def cpu_baseline(name, wl, n):
    """The oracle (as written) on the host cores: one process per shot, bounded sample, in FP64
    (the reference) and float32 (the oracle's float32 emulation); the whole workload's time at
    the measured rate is stated beside."""
    ncpu = len(os.sched_getaffinity(0))
    workers = max(1, min(8, ncpu, wl.nshot))
    work, busy, wall, nsamp = _oracle_sample(name, wl, n, workers, np.float64)
    work32, busy32, _, _ = _oracle_sample(name, wl, n, workers, np.float32)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    full_work = sum(int(np.prod(wl.comp_shape(sh.window))) * (sh.nt - 1) for sh in wl.shots)
    rate = work / busy
    return {"value": round(rate / 1e9, 6), "unit": "Gpts/s", "cores": workers,
            "kind": "oracle", "cpu": cpu_model,
            "sample": f"{workers} shots of {name} in parallel processes (one NumPy thread each), "
                      f"first {nsamp} of {wl.shots[0].nt} time samples; timed: forward at the "
                      f"starting model + gradient call (forward with stored wavefield, adjoint, "
                      f"imaging) in FP64; wall {wall:.1f} s including process start",
            "fp32_value": round(work32 / busy32 / 1e9, 6),
            "full_workload_seconds_at_this_rate": round(full_work / rate, 1),
            "full_workload_note": f"all {wl.nshot} shots x all time steps on the same {workers} cores "
                                  f"({full_work / 1e9:.2f} G point-updates), extrapolated from the sample's "
                                  f"measured rate"}


def base_line(args, wl, value, sec, extra):
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}
    out.update(extra)
    return out


# ------------------------------------------------------------------------------ workloads
def bench_c2(args):
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c2_grad")
    run = GradientRunner(wl, range(wl.nshot), A.Storage(A.STORE_FULL), autotune=not args.no_autotune,
                         tiles=args.tiles, groups=args.groups)
    sec, eager_sec, kernels, timing = timed_gradient(run, args, "fp32")
    value = run.points / sec / 1e9
    mode = fusion_of(run.tiles)
    ff, fa = bool(mode & 1), bool(mode & 2)
    use_graph = not args.no_graph
    names = {"forward": ("fwd2d2 (two forward levels + stored FP32 copies per launch; 20 B per point-update, "
                         "the launch itself moves 28 B per point)" if ff else
                         "fwd2d step (forward + stored FP32 copy, 20 B per point-update)"),
             "adjoint": ("adj2d2 (two adjoint levels + imaging from stored FP32 per launch; 36 B per "
                         "point-update, the launch itself moves 44 B per point)" if fa
                         else "adj2d step (adjoint + imaging from stored FP32, 36 B per point-update)")}
    roof = roofline_of(kernels, names)
    dom_name = (f"adj2d2_kernel<{adjoint_tz(run.tiles)}, 1>" if fa else f"adj2d_kernel<{adjoint_tz(run.tiles)}, 1>") \
        if run.tiles else None
    roof["traffic"] = traffic_record("c2_grad", "kernels2d.hip", dom_name, run.launch_points)
    roof["traffic_counter"] = TRAFFIC_NOTE
    # the whole step against the per-step table: 20 B forward + 36 B adjoint per point-update
    path_bytes = (BYTES[("forward", "fp32")] + BYTES[("adjoint", "fp32")]) * run.points
    loss = float(run.loss.item())
    tiles, points, groups = run.tiles, run.points, run.groups
    run.release()
    single = None
    if not args.no_single:
        r1 = GradientRunner(wl, [0], A.Storage(A.STORE_FULL), autotune=False)
        s1, _ = r1.run(max(1, min(args.steps, 2)), 1, use_graph=False, profile=False)
        single = {"value": round(r1.points / s1 / 1e9, 3), "ms_per_step": round(s1 * 1e3, 2), "shots": 1,
                  "form": "one shot, one launch per time step, no graph"}
        r1.release()
    cpu = None if args.no_cpu_baseline else cpu_baseline("c2_grad", wl, args.cpu_steps)
    copy = copy_probe()
    return base_line(args, wl, value, sec, {
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)),
                   "shots": wl.nshot, "nt": int(wl.shots[0].nt), "storage": "FULL FP32",
                   "batched": True, "graph": use_graph, "tiles": tiles, "shot_groups": groups},
        "roofline": roof, "cpu_baseline": cpu, "kernels": kernels, "kernel_timing": timing,
        "path_hbm_fraction": round(path_bytes / sec / 1e9 / PEAK_HBM_GBS, 4),
        "eager": {"value": round(points / eager_sec / 1e9, 3), "ms_per_step": round(eager_sec * 1e3, 3)},
        "physical_grid_value": round(value * float(np.prod(wl.v[0].shape)) / float(np.prod(wl.comp_shape(0))), 3),
        "single_shot": single, "copy_probe": copy, "loss": loss})


def bench_c3(args):
    """Autograd through WaveOp with 16 FP32 checkpoint slots per shot (32 shots)."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c3_autograd")
    plan = make_plan(wl, A.Storage(A.STORE_CHECKPOINT, 16, A.PREC_FP32), range(wl.nshot))
    m_true = plan.pack([wl.m(0)], "m")
    m0 = plan.pack([wl.m(0, background=True)], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    d_obs = plan.forward(m_true, q)
    tiles = choose_tiles(plan, args, m0, q, d_obs)
    groups = plan.set_groups(args.groups)   # shot groups in effect; the 32 shots split evenly
    points, launch_points = points_of(wl, range(wl.nshot))
    launch_points //= groups

    def step():
        m = m0.clone().requires_grad_(True)
        loss = A.misfit(A.wave_forward(m, q, plan), d_obs)
        loss.backward()
        return loss, m.grad

    for _ in range(args.warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, g = step()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    # kernel timing in one more step: every checkpoint advance is one timed interval (its forward
    # steps back to back, no event between them), every adjoint step another; sampled evenly
    sched = A.checkpoint_schedule(wl.shots[0].nt - 1, 16)
    fwd_steps = int(sum(b - a for op, a, b in sched if op == 0))   # forward steps per gradient
    intervals = groups * (sum(1 for op, _, _ in sched if op == 0) + wl.shots[0].nt)
    plan.profile_enable(min(intervals, MAX_TIMED_LAUNCHES), -(-intervals // MAX_TIMED_LAUNCHES))
    step()
    sync()
    prof = plan.profile_read()
    plan.profile_disable()
    # paired reversals (x, x-1) run as one two-level launch when the adjoint fusion is on
    two = bool(plan.get_tiles()["fusion"] & A.FUSE_ADJOINT)
    pairs = singles = 0
    i = 0
    while i < len(sched):
        if sched[i][0] == 3:
            if two and i + 1 < len(sched) and sched[i + 1][0] == 3 and sched[i + 1][1] == sched[i][1] - 1 \
                    and sched[i][1] >= 2:
                pairs += 1
                i += 2
                continue
            singles += 1
        i += 1
    kernels = kernel_table(prof, launch_points, {"forward": "none", "adjoint": "buffers"},
                           mixed={"adjoint": (pairs, singles)} if two else None)
    names = {"forward": "fwd2d step (forward / recompute, 16 B/point)",
             "adjoint": ("adj2d2 / adj2d steps (paired reversals two levels per launch, imaging from the "
                         "recomputed forward levels, 36 B/point-update)" if two else
                         "adj2d step (adjoint + imaging from recomputed buffers, 36 B/point)")}
    return base_line(args, wl, points / sec / 1e9, sec, {
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)),
                   "shots": wl.nshot, "nt": int(wl.shots[0].nt), "storage": "CHECKPOINT 16 FP32 slots",
                   "batched": True, "graph": False, "tiles": tiles, "shot_groups": groups},
        "roofline": roofline_of(kernels, names), "cpu_baseline": None, "kernels": kernels,
        "forward_steps_per_gradient": fwd_steps,
        "adjoint_launches_per_gradient": pairs + singles, "adjoint_two_level_launches": pairs,
        "recompute_factor": round(fwd_steps / (wl.shots[0].nt - 1), 3), "loss": float(loss.item()),
        "kernel_timing": "value from eager steps without events; kernels from one more eager step, "
                         "HIP events around each checkpoint advance (its forward launches back to back) "
                         "and around each adjoint launch, sampled evenly"})


def counter_step(args):
    """One eager gradient step of c2_grad (FULL FP32) or c5_3d (FULL, --prec) at the given launch
    shape (else the autotuner's), with no HIP events between launches: the program a profiler's
    counter pass runs."""
    import paper_2304_05592_amd as A
    import workloads as W
    name = args.config if args.config in ("c2_grad", "c5_3d") else "c2_grad"
    wl = W.make_config(name)
    prec = {"bf16": A.PREC_BF16, "fp16": A.PREC_FP16, "fp32": A.PREC_FP32}[args.prec] if name == "c5_3d" \
        else A.PREC_FP32
    run = GradientRunner(wl, range(wl.nshot), A.Storage(A.STORE_FULL, 0, prec), autotune=not args.no_autotune,
                         tiles=args.tiles, groups=args.groups)
    run.step()
    sync()
    print(json.dumps({"counter_step": name, "tiles": run.tiles, "points_per_launch": run.launch_points}),
          flush=True)


def bench_c1(args):
    """Single-shot 2D forward (201x101 two-layer model, T = 1 s): graph-replayed time loop vs
    eager launches, and the oracle's forward on the host (the whole shot)."""
    import torch
    import oracle as O
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c1_fwd")
    plan = make_plan(wl, A.Storage(A.STORE_NONE), [0])
    m = plan.pack([wl.m(0)], "m")
    q = plan.pack([wl.q(0)], "q")
    ws = plan.workspace()
    d = torch.empty(plan.layout.d_size, dtype=torch.float32, device="cuda")
    tiles = choose_pass_tiles(plan, args, lambda: plan.forward(m, q, d=d, ws=ws),
                              fusions=(A.FUSE_NONE, A.FUSE_FORWARD))
    points, _ = points_of(wl, [0])
    for _ in range(max(1, args.warmup)):
        plan.forward(m, q, d=d, ws=ws)
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(m, q, d=d, ws=ws)
    sync()
    eager = (time.perf_counter() - t0) / args.steps
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.forward(m, q, d=d, ws=ws)
    for _ in range(max(1, args.warmup)):
        graph.replay()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    cpu = None
    if not args.no_cpu_baseline:
        sh = wl.shots[0]
        t0 = time.perf_counter()
        O.forward(wl.m(0), wl.q(0), sh.src, sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
        tc = time.perf_counter() - t0
        cpu = {"value": round(points / tc / 1e9, 6), "unit": "Gpts/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole shot ({sh.nt} samples) in FP64 NumPy, one process; {tc:.1f} s"}
    return base_line(args, wl, points / sec / 1e9, sec, {
        "metric": "Gpts/s forward, single shot (launch-bound: 0.03 G point-updates per pass)",
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)), "shots": 1,
                   "nt": int(wl.shots[0].nt), "storage": "none (forward)", "graph": True, "tiles": tiles},
        "roofline": None, "cpu_baseline": cpu,
        "eager": {"value": round(points / eager / 1e9, 3), "ms_per_step": round(eager * 1e3, 3)}})


def bench_c6(args):
    """Time-lapse inversion iteration: 15 vintages (model windows) x 4 shots drawn with
    replacement, gradient of 1/2 ||F(m(v)) q - d_obs||^2 with respect to each vintage's
    wavespeed v through WaveOp and the m = 1/v^2 parameterisation, FULL FP32 storage."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c6_timelapse")
    plan = make_plan(wl, A.Storage(A.STORE_FULL), range(wl.nshot))
    v_true = plan.pack([W.extend_edge(wl.v[w].astype(np.float32), wl.nbl) for w in range(wl.nwindow)], "m")
    v0 = plan.pack([W.extend_edge(wl.v0[w].astype(np.float32), wl.nbl) for w in range(wl.nwindow)], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    d_obs = plan.forward(A.slowness2(v_true), q)
    tiles = choose_tiles(plan, args, A.slowness2(v0), q, d_obs)
    groups = plan.set_groups(args.groups)
    points, _ = points_of(wl, range(wl.nshot))

    def step():
        v = v0.clone().requires_grad_(True)
        loss = A.misfit(A.wave_forward(A.slowness2_from_velocity(v), q, plan), d_obs)
        loss.backward()
        return loss, v.grad

    for _ in range(args.warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, g = step()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    return base_line(args, wl, points / sec / 1e9, sec, {
        "metric": "Gpts/s time-lapse gradient (wavespeed), 15 vintages x 4 sampled shots",
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)),
                   "vintages": wl.nwindow, "shots": wl.nshot, "nt": int(wl.shots[0].nt),
                   "storage": "FULL FP32", "graph": False, "tiles": tiles, "shot_groups": groups},
        "roofline": None, "cpu_baseline": None, "loss": float(loss.item()),
        "grad_norm": float(g.norm().item())})


def _time_launches(fn, reps):
    """Mean duration (s) of `fn` (library kernels on torch's current stream) over reps calls,
    bracketed by events on that stream."""
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def rock_kernel_rates(n_cells):
    """Achieved bandwidth of the rock-physics kernels on n_cells synthetic reservoir cells:
    forward reads sw, vp, rho, phi and writes vp_new, rho_new (24 B/cell); the pullback reads
    sw, vp, rho, phi, g_vp and writes g_sw (24 B/cell)."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    side = 4096
    vp, rho, phi = (torch.from_numpy(a.ravel()).cuda() for a in W.reservoir_rock((side,), 7))
    sw = torch.from_numpy(W.saturation_field((side,), 8).ravel()).cuda()
    reps = -(-n_cells // side)
    sw, vp, rho, phi = (t.repeat(reps)[:n_cells].contiguous() for t in (sw, vp, rho, phi))
    g_vp = torch.ones_like(vp)
    out = {}
    for name, fn in (("forward", lambda: A.patchy(sw, vp, rho, phi)),
                     ("pullback", lambda: A.patchy_vjp(sw, vp, rho, phi, g_vp))):
        t = _time_launches(fn, 20)
        out[name] = {"us": round(t * 1e6, 2), "GB/s": round(24.0 * n_cells / t / 1e9, 1),
                     "frac": round(24.0 * n_cells / t / 1e9 / PEAK_HBM_GBS, 4)}
    del sw, vp, rho, phi, g_vp
    torch.cuda.empty_cache()
    return {"cells": int(n_cells), "bytes_per_cell": 24, **out}


def bench_c7(args):
    """Time-lapse iteration through the rock physics: gradient of 1/2 ||F(m(R(sw))) q - d_obs||^2
    with respect to every vintage's CO2 saturation sw, with R the patchy-saturation map of the
    reservoir rock, m = 1/v^2 and WaveOp (15 vintages x 4 sampled shots, FULL FP32 storage).
    The observed data come from the vintages' true saturations; the gradient is taken at zero
    saturation (the brine rock)."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c7_timelapse_rock")
    plan = make_plan(wl, A.Storage(A.STORE_FULL), range(wl.nshot))
    ext = lambda a: W.extend_edge(np.asarray(a, dtype=np.float32), wl.nbl)
    vp, rho, phi = (plan.pack([ext(wl.extra[k])] * wl.nwindow, "m") for k in ("vp", "rho", "phi"))
    sw_true = plan.pack([ext(a) for a in wl.extra["sat"]], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    v_true, _ = A.patchy(sw_true, vp, rho, phi)
    if float(v_true.max()) > wl.vmax:
        raise RuntimeError("rock physics raised the wavespeed above the plan's vmax")
    d_obs = plan.forward(A.slowness2(v_true), q)
    tiles = choose_tiles(plan, args, A.slowness2(vp), q, d_obs)
    groups = plan.set_groups(args.groups)
    points, _ = points_of(wl, range(wl.nshot))
    sw0 = torch.zeros_like(sw_true)

    def step():
        sw = sw0.clone().requires_grad_(True)
        v, _ = A.patchy_rock_physics(sw, vp, rho, phi)
        loss = A.misfit(A.wave_forward(A.slowness2_from_velocity(v), q, plan), d_obs)
        loss.backward()
        return loss, sw.grad

    for _ in range(args.warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, g = step()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    rock = {"workload_size": rock_kernel_rates(sw0.numel()), "large": rock_kernel_rates(1 << 28)}
    return base_line(args, wl, points / sec / 1e9, sec, {
        "metric": "Gpts/s time-lapse gradient (CO2 saturation through rock physics), 15 vintages x 4 sampled shots",
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)),
                   "vintages": wl.nwindow, "shots": wl.nshot, "nt": int(wl.shots[0].nt),
                   "storage": "FULL FP32", "graph": False, "tiles": tiles, "shot_groups": groups},
        "roofline": None, "cpu_baseline": None, "loss": float(loss.item()),
        "grad_norm": float(g.norm().item()), "rock_physics_kernels": rock})


def bench_c8(args):
    """Batched Born modelling dd = J(m0, q) dm of the c2_grad survey (16 shots, dm = m - m0):
    background and scattered wavefields advanced together by one fused kernel per time step,
    the whole pass captured into a HIP graph and replayed."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c2_grad")
    plan = make_plan(wl, A.Storage(A.STORE_NONE), range(wl.nshot))
    m0 = plan.pack([wl.m(0, background=True)], "m")
    dm = plan.pack([wl.m(0) - wl.m(0, background=True)], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    ws = plan.workspace()
    dd = torch.empty(plan.layout.d_size, dtype=torch.float32, device="cuda")
    tiles = choose_pass_tiles(plan, args, lambda: plan.born(m0, q, dm, dd=dd, ws=ws),
                              fusions=(A.FUSE_NONE, A.FUSE_FORWARD))
    groups = plan.set_groups(args.groups)
    points, launch_points = points_of(wl, range(wl.nshot))
    launch_points //= groups
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.born(m0, q, dm, dd=dd, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    sync()
    graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            plan.born(m0, q, dm, dd=dd, ws=ws)
        sync()
    run = (lambda: graph.replay()) if graph is not None else (lambda: plan.born(m0, q, dm, dd=dd, ws=ws))
    for _ in range(args.warmup):
        run()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    nt = wl.shots[0].nt
    plan.profile_enable(groups * nt + 64, 1)
    plan.born(m0, q, dm, dd=dd, ws=ws)
    prof = plan.profile_read()
    plan.profile_disable()
    fused = fusion_of(tiles) & 1
    kernels = kernel_table(prof, launch_points, {"born": "none"}, fused=fused)
    k = kernels["born"]
    k["eager_event_us"] = k["avg_us"]
    timing = "HIP events around each shot group's step loop of one eager pass"
    if graph is not None:
        # graph replay: the pass's time over its step launches (fills and the last gather included)
        avg_s = sec / (k["launches_timed"] // groups * groups)
        k["avg_us"] = round(avg_s * 1e6, 3)
        refresh_rates(k)
        timing = ("graph replay time per pass / step launches of the pass (auxiliary kernels included); "
                  "eager_event_us = HIP events around each shot group's step loop of one eager pass")
    names = {"born": ("born2d2 (two levels of background + scattered field per launch; 32 B per point-update, "
                      "the launch itself moves 40 B per point)") if fused else
             "born2d step (background + scattered field, 32 B/point)"}
    return base_line(args, wl, points / sec / 1e9, sec, {
        "metric": "Gpts/s Born modelling J dm (batched, 16 shots)",
        "config": {"workload": "c8_born: Born modelling of the c2_grad survey (650x341 @ 6.25 m + 40-cell "
                               "border, 16 shots, 650 receivers, T = 1.8 s), dm = true model - smoothed "
                               "background, no wavefield storage",
                   "grid": list(wl.comp_shape(0)), "shots": wl.nshot, "nt": int(nt), "storage": "none",
                   "batched": True, "graph": graph is not None, "tiles": tiles, "shot_groups": groups},
        "roofline": roofline_of(kernels, names), "cpu_baseline": None, "kernels": kernels,
        "kernel_timing": timing, "dd_norm": float(dd.norm().item())})


def bench_c9(args, base="c2_grad"):
    """Probed gradient of the c2_grad survey (16 shots) or of the 3D c5_3d shot: no stored
    wavefield, r Rademacher probes of the time axis accumulated in FP64 by the forward and adjoint
    step kernels, the estimate formed per point at the end.  One call captured into a HIP graph
    and replayed."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config(base)
    r = args.probes
    shots = range(wl.nshot)
    plan = make_plan(wl, A.Storage(A.STORE_PROBED, r), shots)
    m = plan.pack([wl.m(0, background=True)], "m")
    q = plan.pack([wl.q(i) for i in shots], "q")
    dd = plan.pack([W.synthetic_residual(wl.shots[i].nt, len(wl.shots[i].rec), wl.dt, wl.f0, 100 + i)
                    for i in shots], "d")
    max_nt = max(wl.shots[i].nt for i in shots)
    C, sw = W.probe_table("rademacher", max_nt, r=r, seed=1)
    Cd = torch.from_numpy(C).cuda()
    ws = plan.workspace()
    call = lambda: plan.gradient_probed(m, q, dd, Cd, sw, ws=ws)    # noqa: E731
    tiles = (choose_pass_tiles(plan, args, call, fusions=(A.FUSE_NONE, A.FUSE_BOTH)) if wl.ndim == 2
             else choose_tiles(plan, args, m, q, dd, ws))
    groups = plan.set_groups(args.groups)
    points, launch_points = points_of(wl, shots)
    launch_points //= groups
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        g = call()[0]
    torch.cuda.current_stream().wait_stream(st)
    sync()
    graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=st):
            g = call()[0]
        sync()
    run = (lambda: graph.replay()) if graph is not None else call
    for _ in range(args.warmup):
        run()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    kind = f"probe{r}"
    BYTES[("forward", kind)] = BYTES[("forward", "none")] + 16 * r   # + FP64 read and write of B_1..B_r
    BYTES[("adjoint", kind)] = BYTES[("adjoint", "none")] + 16 * r   # + FP64 read and write of A_1..A_r
    # two levels per launch: inputs and both new levels once, and one read and write of the r
    # sums for both levels' terms
    FUSED_BYTES[("forward", kind)] = FUSED_BYTES[("forward", "none")] + 16 * r
    FUSED_BYTES[("adjoint", kind)] = FUSED_BYTES[("adjoint", "none")] + 16 * r
    fused = fusion_of(tiles)
    plan.profile_enable(2 * groups + 64, 1)   # one interval per sweep of each shot group
    call()
    prof = plan.profile_read()
    plan.profile_disable()
    kernels = kernel_table(prof, launch_points, {"forward": kind, "adjoint": kind}, fused=fused)
    for k in kernels.values():
        if "fused_bytes_per_launch" in k:
            # twice the per-step figure is no lower bound here (one read-modify-write of the sums
            # serves both levels): a two-level launch is priced at the bytes it moves
            k["per_step_table_bytes_per_launch"] = k["bytes_per_launch"]
            k["bytes_per_launch"] = k["fused_bytes_per_launch"]
            refresh_rates(k)
    dim = f"{wl.ndim}d"
    names = {d: (f"{d[:3]}{dim}2 two steps + {r} FP64 probe sums ({FUSED_BYTES[(d, kind)]} B/point per launch)"
                 if fused & (1 if d == "forward" else 2) else
                 f"{d[:3]}{dim} step + {r} FP64 probe sums ({BYTES[(d, kind)]} B/point)")
             for d in ("forward", "adjoint")}
    _, full_ws = A.select_storage(wl.ndim, wl.h, wl.dt, wl.nbl, wl.vmax, [wl.comp_shape(0)],
                                  [A.ShotGeometry(wl.shots[i].window, wl.shots[i].nt, wl.shots[i].src,
                                                  wl.shots[i].rec) for i in shots],
                                  A.Storage(A.STORE_FULL, 0, A.PREC_FP32 if wl.ndim == 2 else A.PREC_BF16),
                                  damp_vref=wl.vmax)
    return base_line(args, wl, points / sec / 1e9, sec, {
        "metric": f"Gpts/s probed gradient ({wl.nshot} shots)",
        "config": {"workload": f"{args.config}: the {base} gradient from {r} Rademacher probes of the "
                               "time axis (no stored wavefield)",
                   "grid": list(wl.comp_shape(0)), "shots": wl.nshot, "nt": int(max_nt),
                   "storage": f"PROBED {r}", "batched": True, "graph": graph is not None, "tiles": tiles,
                   "shot_groups": groups},
        "workspace_bytes": plan.ws_bytes, "full_storage_workspace_bytes": full_ws,
        "full_storage_precision": "fp32" if wl.ndim == 2 else "bf16",
        "roofline": roofline_of(kernels, names, fused_bytes=True), "cpu_baseline": None, "kernels": kernels,
        "kernel_timing": "HIP events around each sweep's step loop of one eager call (interval / "
                         "launches); value from graph replays",
        "g_norm": float(g.norm().item())})


def bench_c4(args):
    """64 uneven windows, forward: one batched graph-captured run vs 64 sequential runs."""
    import torch
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c4_uneven")
    plan = make_plan(wl, A.Storage(A.STORE_NONE), range(wl.nshot))
    m = plan.pack([wl.m(w) for w in range(wl.nwindow)], "m")
    q = plan.pack([wl.q(s) for s in range(wl.nshot)], "q")
    ws = plan.workspace()
    d = torch.empty(plan.layout.d_size, dtype=torch.float32, device="cuda")
    tiles = choose_pass_tiles(plan, args, lambda: plan.forward(m, q, d=d, ws=ws),
                              fusions=(A.FUSE_NONE, A.FUSE_FORWARD))
    groups = plan.set_groups(args.groups)
    points, launch_points = points_of(wl, range(wl.nshot))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(m, q, d=d, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    sync()
    nt_max = max(sh.nt for sh in wl.shots)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.forward(m, q, d=d, ws=ws)
    sync()
    for _ in range(args.warmup):
        graph.replay()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    # kernel durations: one eager pass with HIP events around each shot group's step loop
    plan.profile_enable(groups * nt_max + 64, 1)   # one launch per step and shot group
    plan.forward(m, q, d=d, ws=ws)
    prof = plan.profile_read()
    plan.profile_disable()
    # sequential single-shot runs (plain form: one plan per shot, one launch per step)
    seq = 0.0
    for sidx in range(wl.nshot):
        p1 = make_plan(wl, A.Storage(A.STORE_NONE), [sidx])
        m1 = p1.pack([wl.m(w) for w in range(wl.nwindow)], "m")
        q1 = p1.pack([wl.q(sidx)], "q")
        ws1 = p1.workspace()
        d1 = torch.empty(p1.layout.d_size, dtype=torch.float32, device="cuda")
        p1.forward(m1, q1, d=d1, ws=ws1)
        sync()
        t0 = time.perf_counter()
        p1.forward(m1, q1, d=d1, ws=ws1)
        sync()
        seq += time.perf_counter() - t0
        del p1, m1, q1, ws1, d1
    # launches cover different numbers of active shots: use the pass's summed kernel time
    cnt, ms = prof["forward"]
    est_kernel_s = ms * 1e-3
    fused = bool(fusion_of(tiles) & 1)
    ach = BYTES[("forward", "none")] * points / est_kernel_s / 1e9 if cnt else None
    return base_line(args, wl, points / sec / 1e9, sec, {
        "metric": "Gpts/s forward, uneven batching (64 windows) batched vs sequential single-shot",
        "config": {"workload": f"{wl.name}: {wl.description}", "shots": wl.nshot,
                   "points_per_pass": points, "storage": "none (forward)", "batched": True,
                   "graph": True, "tiles": tiles, "shot_groups": groups},
        "roofline": {"bound": "hbm", "achieved": None if ach is None else round(ach, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": None if ach is None else round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": ("fwd2d2 (two levels per launch, 16 B per point-update; the launch itself "
                                "moves 20 B per point)" if fused else "fwd2d step (16 B per point-update)")
                               + "; event time of each shot group's step loop in one eager pass"},
        "sequential_single_shot": {"value": round(points / seq / 1e9, 3), "seconds": round(seq, 4)},
        "cpu_baseline": None})


def bench_c5(args):
    """3D 256^3 single shot: forward + gradient with FULL 16-bit (or FP32) storage."""
    import paper_2304_05592_amd as A
    import workloads as W
    wl = W.make_config("c5_3d")
    prec = {"bf16": A.PREC_BF16, "fp16": A.PREC_FP16, "fp32": A.PREC_FP32}[args.prec]
    run = GradientRunner(wl, [0], A.Storage(A.STORE_FULL, 0, prec), autotune=not args.no_autotune,
                         tiles=args.tiles)
    kind = "fp32" if prec == A.PREC_FP32 else "16bit"
    sec, eager_sec, kernels, timing = timed_gradient(run, args, kind)
    names = {"forward": f"fwd3d step (forward + stored {args.prec} copy, {BYTES[('forward', kind)]} B/point)",
             "adjoint": f"adj3d step (adjoint + imaging, {BYTES[('adjoint', kind)]} B/point)"}
    roof = roofline_of(kernels, names)
    if run.tiles and roof.get("kernel") == names["adjoint"]:
        adj = run.tiles["adjoint"]
        img = {A.PREC_FP32: 1, A.PREC_BF16: 3, A.PREC_FP16: 4}[prec]
        roof["traffic"] = traffic_record("c5_3d", "kernels3d.hip", f"adj3d_kernel<{adj['ty']}, {img}>",
                                         run.launch_points, {"ty": adj["ty"], "bz": adj["bz"]})
        roof["traffic_counter"] = TRAFFIC_NOTE
    out = base_line(args, wl, run.points / sec / 1e9, sec, {
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)),
                   "shots": 1, "nt": int(wl.shots[0].nt), "storage": f"FULL {args.prec}",
                   "batched": False, "graph": not args.no_graph, "tiles": run.tiles},
        "roofline": roof, "cpu_baseline": None, "kernels": kernels,
        "kernel_timing": timing,
        "eager": {"value": round(run.points / eager_sec / 1e9, 3), "ms_per_step": round(eager_sec * 1e3, 3)},
        "loss": float(run.loss.item())})
    run.release()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X; sharding "
              "shots over several GPUs (with an FP64 all-reduce of the gradient) is not "
              "implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_probe()}), flush=True)
        return
    if args.counter_step:
        counter_step(args)
        return
    fn = {"c1_fwd": bench_c1, "c2_grad": bench_c2, "c3_autograd": bench_c3, "c4_uneven": bench_c4,
          "c5_3d": bench_c5, "c6_timelapse": bench_c6,
          "c7_timelapse_rock": bench_c7, "c8_born": bench_c8, "c9_probed": bench_c9,
          "c9_probed_3d": lambda a: bench_c9(a, "c5_3d")}[args.config]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
