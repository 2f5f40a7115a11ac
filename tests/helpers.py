"""Test-side glue: run the oracle over the shots of a seeded workload."""
from __future__ import annotations

import numpy as np

import oracle as O


def shot_kwargs(wl, s):
    sh = wl.shots[s]
    return dict(src=sh.src, rec=sh.rec, h=wl.h, dt=wl.dt, nbl=wl.nbl, vref=wl.vmax)


def oracle_forward(wl, ms=None, shots=None, dtype=None):
    """Traces of every shot (list of [nt][nrec] float64 arrays)."""
    ms = [wl.m(w) for w in range(wl.nwindow)] if ms is None else ms
    shots = range(wl.nshot) if shots is None else shots
    return [O.forward(ms[wl.shots[s].window], wl.q(s), dtype=dtype, **shot_kwargs(wl, s)) for s in shots]


def oracle_gradient(wl, dds, ms=None, shots=None, segment=None):
    """Per-window gradients: shots on one window summed in ascending shot order."""
    ms = [wl.m(w) for w in range(wl.nwindow)] if ms is None else ms
    shots = range(wl.nshot) if shots is None else list(shots)
    gs = [np.zeros(m.shape) for m in ms]
    for i, s in enumerate(shots):
        w = wl.shots[s].window
        gs[w] = gs[w] + O.gradient(ms[w], wl.q(s), dds[i], segment=segment, **shot_kwargs(wl, s))
    return gs


def oracle_adjoint(wl, dds, ms=None, shots=None):
    ms = [wl.m(w) for w in range(wl.nwindow)] if ms is None else ms
    shots = range(wl.nshot) if shots is None else list(shots)
    return [O.adjoint(ms[wl.shots[s].window], dds[i], **shot_kwargs(wl, s)) for i, s in enumerate(shots)]


def oracle_born(wl, dms, ms=None, shots=None):
    ms = [wl.m(w) for w in range(wl.nwindow)] if ms is None else ms
    shots = range(wl.nshot) if shots is None else list(shots)
    return [O.born(ms[wl.shots[s].window], wl.q(s), dms[wl.shots[s].window], **shot_kwargs(wl, s))
            for s in shots]


def rel_l2(a, b):
    a = np.concatenate([np.ravel(x) for x in a]) if isinstance(a, (list, tuple)) else np.ravel(a)
    b = np.concatenate([np.ravel(x) for x in b]) if isinstance(b, (list, tuple)) else np.ravel(b)
    return float(np.linalg.norm(a.astype(np.float64) - b.astype(np.float64)) /
                 np.linalg.norm(b.astype(np.float64)))


# ------------------------------------------------------------------------------ GPU side
def make_plan(wl, storage=None, shots=None, **kw):
    """Plan for the workload's shots (all, or the given indices) on its windows."""
    import paper_2304_05592_amd as A
    shots = range(wl.nshot) if shots is None else list(shots)
    geoms = [A.ShotGeometry(wl.shots[s].window, wl.shots[s].nt, wl.shots[s].src, wl.shots[s].rec)
             for s in shots]
    windows = [wl.comp_shape(w) for w in range(wl.nwindow)]
    return A.Plan(wl.ndim, wl.h, wl.dt, wl.nbl, wl.vmax, windows, geoms, storage=storage,
                  damp_vref=wl.vmax, **kw)


def gpu_inputs(wl, plan, shots=None, background=False):
    """Packed float32 device tensors m (all windows) and q (the plan's shots)."""
    shots = range(wl.nshot) if shots is None else list(shots)
    m = plan.pack([wl.m(w, background=background) for w in range(wl.nwindow)], "m")
    q = plan.pack([wl.q(s) for s in shots], "q")
    return m, q
