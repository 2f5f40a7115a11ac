"""Benchmark: batched 2D forward + adjoint-state gradient on one MI355X.

One step = the whole hot path over one batch of shots: forward solve with the wavefield
kept in HBM (traces d = F(m0) q), residual r = d - d_obs with the misfit 1/2 ||r||^2 in
FP64, and the reverse sweep g = J^T r (adjoint solve + imaging condition, FP64
accumulation), all in the library's HIP kernels.  Inputs are resident in HBM before the
timed region.  Default workload: 650 x 341 physical grid at 6.25 m (+40-cell damping
border), layered 1.5-4.5 km/s with a 5 % smoothed random perturbation, 16 shots, 650
receivers, T = 1.8 s, full FP32 wavefield storage.

Prints one JSON line.  Gpts/s = sum over shots of N_s (nt_s - 1) per step, divided by the
step time (N_s = computational-grid points of the shot).
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
# algorithmic bytes per grid point per launch of each step kernel (FP32 fields, FP64 accumulator)
BYTES_FWD_FULL = 20   # read u^{k-1}, u^{k-2}, coef; write u^k and its stored copy
BYTES_ADJ_FULL = 36   # read w^{j+1}, w^{j+2}, coef, stored u^j, acc (8); write w^j, acc (8)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2_grad")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=120, help="time steps of the oracle sample")
    return ap.parse_args()


def make_plan(wl, storage, shots):
    import paper_2304_05592_amd as A
    geoms = [A.ShotGeometry(wl.shots[s].window, wl.shots[s].nt, wl.shots[s].src, wl.shots[s].rec)
             for s in shots]
    windows = [wl.comp_shape(w) for w in range(wl.nwindow)]
    return A.Plan(wl.ndim, wl.h, wl.dt, wl.nbl, wl.vmax, windows, geoms, storage=storage,
                  damp_vref=wl.vmax)


class Runner:
    """Inputs resident on the GPU and one step of the hot path."""

    def __init__(self, wl, shots):
        import torch
        import paper_2304_05592_amd as A
        self.A, self.torch = A, torch
        self.wl, self.shots = wl, list(shots)
        self.plan = make_plan(wl, A.Storage(A.STORE_FULL), self.shots)
        p = self.plan
        self.m_true = p.pack([wl.m(w) for w in range(wl.nwindow)], "m")
        self.m0 = p.pack([wl.m(w, background=True) for w in range(wl.nwindow)], "m")
        self.q = p.pack([wl.q(s) for s in self.shots], "q")
        self.ws = p.workspace()
        self.d_obs = p.forward(self.m_true, self.q, ws=self.ws)
        self.d = torch.empty_like(self.d_obs)
        self.r = torch.empty_like(self.d_obs)
        self.g = torch.empty(p.layout.m_size, dtype=torch.float64, device="cuda")
        self.points = sum(int(np.prod(wl.comp_shape(wl.shots[s].window))) * (wl.shots[s].nt - 1)
                          for s in self.shots)
        self.launch_points = sum(int(np.prod(wl.comp_shape(wl.shots[s].window))) for s in self.shots)
        torch.cuda.synchronize()

    def step(self):
        p = self.plan
        p.forward(self.m0, self.q, d=self.d, keep=True, ws=self.ws)
        _, self.loss = self.A.residual(self.d, self.d_obs, r=self.r)
        p.backward(self.m0, self.q, self.r, g=self.g, v=None, ws=self.ws)

    def timed(self, steps, warmup, profile=False):
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        if profile:
            nt = max(self.wl.shots[s].nt for s in self.shots)
            self.plan.profile_enable(2 * nt * steps + 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = self.plan.profile_read() if profile else None
        if profile:
            self.plan.profile_disable()
        return (t1 - t0) / steps, prof

    def release(self):
        self.ws = None
        self.plan = None
        self.torch.cuda.empty_cache()


def _oracle_worker(args):
    """Oracle gradient of one shot over its first n samples (runs in a worker process)."""
    name, s, n = args
    import workloads as W
    import oracle as O
    wl = W.make_config(name)
    sh = wl.shots[s]
    kw = dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)
    m_true, m0 = wl.m(sh.window), wl.m(sh.window, background=True)
    q = wl.q(s)[:n]
    t0 = time.perf_counter()
    d_obs = O.forward(m_true, q, **kw)
    t1 = time.perf_counter()
    g = O.gradient(m0, q, O.forward(m0, q, **kw) - d_obs, **kw)
    t2 = time.perf_counter()
    npts = int(np.prod(wl.comp_shape(sh.window)))
    # work of one step of the path for this sample: N (n - 1) point-updates; the oracle's
    # gradient call repeats the forward, so time the forward-with-residual + gradient part
    return npts * (n - 1), (t2 - t1), float(np.abs(g).max())


def cpu_baseline(name, wl, n):
    """The oracle (as written) on the host cores: one process per shot, bounded sample."""
    import multiprocessing as mp
    ncpu = len(os.sched_getaffinity(0))
    workers = max(1, min(8, ncpu, wl.nshot))
    jobs = [(name, s, min(n, wl.shots[s].nt)) for s in range(workers)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": round(work / busy / 1e9, 6), "unit": "Gpts/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{workers} shots of {name} in parallel processes (one NumPy thread each), "
                      f"first {jobs[0][2]} of {wl.shots[0].nt} time samples, gradient "
                      f"(forward with stored wavefield + adjoint + imaging) in FP64; "
                      f"wall {wall:.1f} s including process start"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this path is built and measured on a single MI355X; "
              "multi-GPU runs (shots sharded over GPUs, FP64 gradient all-reduce) are not part "
              "of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    wl = W.make_config(args.config)
    run = Runner(wl, range(wl.nshot))
    sec, prof = run.timed(args.steps, args.warmup, profile=True)
    value = run.points / sec / 1e9
    loss = float(run.loss.item())
    kernels = {}
    for name, bpp in (("forward", BYTES_FWD_FULL), ("adjoint", BYTES_ADJ_FULL)):
        cnt, ms = prof[name]
        avg_ms = ms / max(cnt, 1)
        bytes_per_launch = bpp * run.launch_points
        kernels[name] = {"launches": cnt, "avg_us": round(avg_ms * 1e3, 3),
                         "bytes_per_launch": bytes_per_launch,
                         "achieved_GBs": round(bytes_per_launch / (avg_ms * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    ach = kernels[dom]["achieved_GBs"]
    roofline = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                "kernel": f"adj2d step (adjoint + imaging, {BYTES_ADJ_FULL} B/point)" if dom == "adjoint"
                else f"fwd2d step (forward + stored copy, {BYTES_FWD_FULL} B/point)"}
    path_bytes = (BYTES_FWD_FULL + BYTES_ADJ_FULL) * run.points
    run.release()

    single = None
    if not args.no_single:
        r1 = Runner(wl, [0])
        sec1, _ = r1.timed(max(1, min(args.steps, 2)), 1)
        single = {"value": round(r1.points / sec1 / 1e9, 3), "ms_per_step": round(sec1 * 1e3, 2),
                  "shots": 1}
        r1.release()

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.config, wl, args.cpu_steps)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}", "grid": list(wl.comp_shape(0)),
                   "shots": wl.nshot, "nt": int(wl.shots[0].nt), "storage": "FULL FP32",
                   "batched": True},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "path_hbm_fraction": round(path_bytes / sec / 1e9 / PEAK_HBM_GBS, 4),
        "single_shot": single,
        "loss": loss,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
