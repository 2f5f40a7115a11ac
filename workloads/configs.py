"""Workload definitions and seeded generators (inputs only, no wave-equation arithmetic).

Every generator is deterministic for a given seed (numpy ``default_rng`` and
``scipy.ndimage.gaussian_filter``), so the oracle side and the GPU side rebuild
bit-identical float32 inputs on any machine with the same numpy/scipy.

Readings of the paper fixed here (the paper gives no discretisation, see the
section "Wave-equation-based inversion"):
  * layered model: 8 equal-thickness flat layers over the physical depth with
    v_l = vmin + (vmax - vmin) * l / 7;
  * perturbation: a unit-variance Gaussian-smoothed N(0,1) field, kernel std =
    (correlation length / 2) in cells, ``mode='reflect'``; v = v_layer (1 + 0.05 p);
  * time grid: dt = CFL h / vmax with vmax the maximum of the true model,
    nt = ceil(T / dt) + 1, t_n = n dt;
  * Ricker wavelet with delay t0 = 1.5 / f0 and unit amplitude;
  * sources and receivers at depth 2h, receivers on every physical column.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np
from scipy.ndimage import gaussian_filter

__all__ = ["Shot", "Workload", "ricker", "layered_velocity", "two_layer_velocity",
           "smooth_perturbation", "smooth_background", "extend_edge", "cfl_time_grid",
           "make_config", "config_names", "small_2d", "small_3d", "synthetic_residual",
           "random_field"]


# --------------------------------------------------------------------------------------
# basic generators
# --------------------------------------------------------------------------------------
def ricker(nt: int, dt: float, f0: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet r(t) = (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2) at t_n = n dt.

    f0 in kHz, dt in ms; default delay t0 = 1.5 / f0.  Returned as float32 (the
    precision both the oracle and the GPU path read).
    """
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f0 * (t - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def two_layer_velocity(nz: int, nx: int, h: float, z_interface: float,
                       v_top: float, v_bottom: float) -> np.ndarray:
    """Two flat layers: v_top for depth z = k h < z_interface, v_bottom below."""
    z = np.arange(nz, dtype=np.float64) * h
    col = np.where(z < z_interface, v_top, v_bottom)
    return np.repeat(col[:, None], nx, axis=1)


def layered_velocity(shape, nlayers: int = 8, vmin: float = 1.5, vmax: float = 4.5) -> np.ndarray:
    """Flat layers of equal thickness over the depth axis (axis 0), velocity rising linearly."""
    nz = shape[0]
    k = np.arange(nz)
    layer = (k * nlayers) // nz
    col = vmin + (vmax - vmin) * layer / (nlayers - 1)
    out = np.empty(shape, dtype=np.float64)
    out[...] = col.reshape((nz,) + (1,) * (len(shape) - 1))
    return out


def smooth_perturbation(shape, h: float, corr_length: float, seed: int) -> np.ndarray:
    """Unit-variance Gaussian-smoothed white noise (kernel std corr_length / 2 in metres)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    p = gaussian_filter(white, sigma=0.5 * corr_length / h, mode="reflect")
    p -= p.mean()
    return p / p.std()


def smooth_background(v: np.ndarray, h: float, length: float = 100.0) -> np.ndarray:
    """Smoothed starting model v0 = gaussian_filter(v, length / h cells, mode='nearest')."""
    return gaussian_filter(v, sigma=length / h, mode="nearest")


def extend_edge(a: np.ndarray, nbl: int) -> np.ndarray:
    """Replicate the edge values of a physical-grid array nbl cells outward on every axis."""
    return np.pad(a, nbl, mode="edge")


def cfl_time_grid(T: float, h: float, vmax: float, cfl: float = 0.4):
    """dt = cfl h / vmax (ms) and nt = ceil(T / dt) + 1 samples (last sample at or past T)."""
    dt = cfl * h / vmax
    nt = int(math.ceil(T / dt - 1e-9)) + 1
    return dt, nt


def random_field(shape, seed: int, smooth_cells: float = 0.0, dtype=np.float32) -> np.ndarray:
    """Seeded N(0,1) field, optionally Gaussian-smoothed (std in cells) and renormalised."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape)
    if smooth_cells > 0:
        a = gaussian_filter(a, sigma=smooth_cells, mode="reflect")
        a /= a.std()
    return a.astype(dtype)


def synthetic_residual(nt: int, nrec: int, dt: float, f0: float, seed: int) -> np.ndarray:
    """Band-limited random traces [nt][nrec]: white noise convolved in time with a Ricker.

    Used as a data residual when only the linear adjoint / gradient operators are
    being compared (any residual exercises them; this one has the data's band).
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((nt, nrec))
    half = int(math.ceil(1.5 / f0 / dt))
    t = (np.arange(-half, half + 1) * dt)
    a = (math.pi * f0 * t) ** 2
    w = (1.0 - 2.0 * a) * np.exp(-a)
    out = np.empty_like(white)
    for r in range(nrec):
        out[:, r] = np.convolve(white[:, r], w, mode="full")[half:half + nt]
    out /= np.abs(out).max()
    return out.astype(np.float32)


# --------------------------------------------------------------------------------------
# workload container
# --------------------------------------------------------------------------------------
@dataclass
class Shot:
    """One shot: which model window it runs on, its length and its acquisition.

    Positions are (x, y, z) in metres in the physical coordinates of the shot's
    window (x = i h for physical column i; y = 0 in 2D).
    """
    window: int
    nt: int
    src: np.ndarray
    rec: np.ndarray


@dataclass
class Workload:
    name: str
    ndim: int
    h: float
    nbl: int
    dt: float
    f0: float
    vmax: float
    cfl: float
    v: List[np.ndarray]                # physical velocity per window (float64)
    shots: List[Shot]
    description: str = ""
    v0: Optional[List[np.ndarray]] = None   # smooth starting model (gradient configs)
    extra: dict = field(default_factory=dict)

    # ---- sizes -------------------------------------------------------------------
    @property
    def nshot(self) -> int:
        return len(self.shots)

    @property
    def nwindow(self) -> int:
        return len(self.v)

    def comp_shape(self, w: int):
        """Computational-grid shape (nz, [ny,] nx) of window w: physical + 2 nbl per axis."""
        return tuple(n + 2 * self.nbl for n in self.v[w].shape)

    def point_updates(self) -> int:
        """Sum over shots of N_s (nt_s - 1): the work unit of the Gpts/s metric."""
        return int(sum(int(np.prod(self.comp_shape(s.window))) * (s.nt - 1) for s in self.shots))

    # ---- arrays ------------------------------------------------------------------
    def m(self, w: int, background: bool = False) -> np.ndarray:
        """Squared slowness on the computational grid of window w (float32, edge-extended)."""
        vv = (self.v0 if background else self.v)[w]
        m_phys = (1.0 / vv.astype(np.float64) ** 2).astype(np.float32)
        return extend_edge(m_phys, self.nbl)

    def q(self, s: int) -> np.ndarray:
        """Source wavelet samples of shot s (float32, length nt_s)."""
        return ricker(self.shots[s].nt, self.dt, self.f0)

    def with_shots(self, idx) -> "Workload":
        """A copy restricted to the given shot indices (window list unchanged)."""
        return replace(self, shots=[self.shots[i] for i in idx])


# --------------------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------------------
def _surface_receivers(nx: int, h: float, depth: float) -> np.ndarray:
    rec = np.zeros((nx, 3))
    rec[:, 0] = np.arange(nx) * h
    rec[:, 2] = depth
    return rec


def _c1() -> Workload:
    nx, nz, h = 201, 101, 10.0
    v = two_layer_velocity(nz, nx, h, 500.0, 1.5, 2.5)
    vmax = float(v.max())
    dt, nt = cfl_time_grid(1000.0, h, vmax)
    rec = np.zeros((101, 3))
    rec[:, 0] = np.arange(101) * 20.0
    rec[:, 2] = 20.0
    shots = [Shot(0, nt, np.array([1000.0, 0.0, 20.0]), rec)]
    return Workload("c1_fwd", 2, h, 40, dt, 0.015, vmax, 0.4, [v], shots,
                    "2D forward, 201x101 @ 10 m, two layers 1.5/2.5 km/s, 1 shot, 101 receivers")


def _layered_perturbed(shape, h, seed):
    return layered_velocity(shape) * (1.0 + 0.05 * smooth_perturbation(shape, h, 200.0, seed))


def _surface_survey(name, nx, nz, h, T, nshot, seed, desc):
    v = _layered_perturbed((nz, nx), h, seed)
    vmax = float(v.max())
    dt, nt = cfl_time_grid(T, h, vmax)
    rec = _surface_receivers(nx, h, 2 * h)
    shots = []
    for s in range(nshot):
        xs = (s + 0.5) * (nx - 1) * h / nshot
        shots.append(Shot(0, nt, np.array([xs, 0.0, 2 * h]), rec))
    v0 = [smooth_background(v, h)]
    return Workload(name, 2, h, 40, dt, 0.015, vmax, 0.4, [v], shots, desc, v0=v0)


def _c2() -> Workload:
    return _surface_survey("c2_grad", 650, 341, 6.25, 1800.0, 16, 0,
                           "2D forward + gradient, 650x341 @ 6.25 m, layered 1.5-4.5 + 5% "
                           "perturbation, 16 shots, 650 receivers, full FP32 wavefield storage")


def _c3() -> Workload:
    return _surface_survey("c3_autograd", 1024, 512, 6.25, 2500.0, 32, 0,
                           "2D autograd gradient, 1024x512 @ 6.25 m, 32 shots, 1024 receivers, "
                           "16 FP32 checkpoint slots per shot")


def _c4() -> Workload:
    h, nz, nx_big = 6.25, 341, 4096
    vbig = _layered_perturbed((nz, nx_big), h, 1)
    vmax = float(vbig.max())
    rng = np.random.default_rng(101)
    widths = rng.integers(256, 1025, size=64)
    Ts = rng.uniform(1000.0, 2500.0, size=64)
    starts = [int(rng.integers(0, nx_big - w + 1)) for w in widths]
    dt = 0.4 * h / vmax
    windows, shots = [], []
    for i, (w, T, x0) in enumerate(zip(widths, Ts, starts)):
        windows.append(np.ascontiguousarray(vbig[:, x0:x0 + int(w)]))
        nt = int(math.ceil(T / dt - 1e-9)) + 1
        src = np.array([0.5 * (int(w) - 1) * h, 0.0, 2 * h])
        shots.append(Shot(i, nt, src, _surface_receivers(int(w), h, 2 * h)))
    v0 = [smooth_background(v, h) for v in windows]
    return Workload("c4_uneven", 2, h, 40, dt, 0.015, vmax, 0.4, windows, shots,
                    "2D uneven batching: 64 windows, widths U{256..1024} x 341 @ 6.25 m, "
                    "T ~ U[1.0, 2.5] s", v0=v0)


def _volume_survey(name, n, h, T, src, rec_step_cells, rec_n, seed, desc, crop=None):
    shape = (n, n, n)
    v = _layered_perturbed(shape, h, seed)
    vmax = float(v.max())
    dt, nt = cfl_time_grid(T, h, vmax)
    if crop is not None:
        (z0, z1), (y0, y1), (x0, x1) = crop
        v = np.ascontiguousarray(v[z0:z1, y0:y1, x0:x1])
        src = src - np.array([x0 * h, y0 * h, z0 * h])
    g = np.arange(rec_n) * rec_step_cells * h
    X, Y = np.meshgrid(g, g, indexing="xy")
    rec = np.zeros((rec_n * rec_n, 3))
    rec[:, 0] = X.ravel()
    rec[:, 1] = Y.ravel()
    rec[:, 2] = 2 * h
    shots = [Shot(0, nt, src, rec)]
    v0 = [smooth_background(v, h)]
    return Workload(name, 3, h, 40, dt, 0.015, vmax, 0.4, [v], shots, desc, v0=v0)


def _c5() -> Workload:
    return _volume_survey("c5_3d", 256, 12.5, 2000.0, np.array([1600.0, 1600.0, 25.0]), 2, 128, 0,
                          "3D forward + gradient, 256^3 @ 12.5 m, 1 shot, 128x128 receivers")


def _c5_crop() -> Workload:
    return _volume_survey("c5_crop", 256, 12.5, 2000.0, np.array([1600.0, 1600.0, 25.0]), 2, 32, 0,
                          "64^3 crop (x, y in [96,160), z in [0,64)) of the 3D model, 32x32 receivers",
                          crop=((0, 64), (96, 160), (96, 160)))


def plume_mask(shape, h: float, vintage: int, nvint: int) -> np.ndarray:
    """Synthetic stand-in for a CO2 plume at vintage i of n (0 outside, up to 1 inside): an
    inverted cone above a reservoir layer whose width grows as sqrt(i/n), smoothed over ~2 cells.
    It only provides time-lapse wavespeed changes of a plausible shape (no flow physics)."""
    nz, nx = shape
    z = (np.arange(nz) + 0.5)[:, None] / nz
    x = (np.arange(nx) + 0.5)[None, :] / nx
    frac = np.sqrt(max(vintage, 0) / float(nvint))
    top, bottom = 0.45, 0.70                        # reservoir band (fraction of depth)
    half = 0.30 * frac * (0.4 + 0.6 * (z - top) / (bottom - top))   # cone: wider at the bottom
    inside = (z >= top) & (z <= bottom) & (np.abs(x - 0.5) <= half)
    out = gaussian_filter(inside.astype(np.float64), 2.0, mode="nearest")
    return np.clip(out, 0.0, 1.0)


def reservoir_rock(shape, seed: int = 7):
    """Seeded brine-saturated reservoir rock for the patchy-saturation map: wavespeed vp
    3.1-3.8 km/s, density 2250-2450 kg/m^3 and porosity 0.20-0.30, each a smooth random field
    (correlation ~8 cells) mapped into its range.  Within these ranges the dry frame implied by
    the brine-saturated moduli (vs = vp / sqrt 3) is positive, as for a physical sandstone.
    Returns float32 arrays (vp, rho, phi)."""
    out = []
    for k, (lo, hi) in enumerate(((3.1, 3.8), (2250.0, 2450.0), (0.20, 0.30))):
        f = random_field(shape, seed * 10 + k, smooth_cells=4.0, dtype=np.float64)
        u = 0.5 * (1.0 + np.tanh(0.8 * f))                      # smooth, in (0, 1)
        out.append((lo + (hi - lo) * u).astype(np.float32))
    return tuple(out)


def saturation_field(shape, seed: int = 8, zero_frac: float = 0.3, one_frac: float = 0.1):
    """Seeded CO2 saturation in [0, 1]: a smooth random field whose lowest `zero_frac` of cells
    are exactly 0 (no CO2) and highest `one_frac` exactly 1 (fully saturated), the rest in
    between.  float32."""
    f = random_field(shape, seed, smooth_cells=3.0, dtype=np.float64)
    lo, hi = np.quantile(f, [zero_frac, 1.0 - one_frac])
    return np.clip((f - lo) / (hi - lo), 0.0, 1.0).astype(np.float32)


def timelapse_survey(name="c6_timelapse", nx=512, nz=256, h=6.25, T=1200.0, nvint=15, nsrc=32, nrec=960,
                     shots_per_vintage=4, iteration=0, seed=6, drop=0.05, nbl=40,
                     rock_seed=None, saturation=0.9) -> Workload:
    """Time-lapse crosswell survey: vintages i = 1..nvint share a layered baseline and differ by
    a growing low-wavespeed plume (v^i = v_base (1 - drop * plume_i)); sources in the left well,
    receivers in the right well.  One inversion iteration draws `shots_per_vintage` of the nsrc
    sources per vintage with replacement (seeded by `iteration`); shot s runs on window = its
    vintage.  The starting model of every vintage is the smoothed baseline.

    With `rock_seed`, the medium is instead the brine-saturated reservoir rock of
    `reservoir_rock` (vp, rho, phi) and vintage i is described by its CO2 saturation
    `saturation * plume_i` (extra["sat"], physical grid); its wavespeed is the rock physics
    map of that saturation, which the consumer evaluates.  v and v0 then hold the brine rock
    (zero saturation), which bounds every vintage's wavespeed for this soft rock."""
    rock = None
    if rock_seed is not None:
        rock = [a.astype(np.float64) for a in reservoir_rock((nz, nx), rock_seed)]
        vs = [rock[0]] * nvint
    else:
        v_base = _layered_perturbed((nz, nx), h, seed)
        vs = [v_base * (1.0 - drop * plume_mask((nz, nx), h, i + 1, nvint)) for i in range(nvint)]
    vmax = float(max(v.max() for v in vs))
    dt, nt = cfl_time_grid(T, h, vmax)
    xs, xr = 0.1 * (nx - 1) * h, 0.9 * (nx - 1) * h
    src_z = np.linspace(0.1, 0.9, nsrc) * (nz - 1) * h
    rec = np.zeros((nrec, 3))
    rec[:, 0] = xr
    rec[:, 2] = np.linspace(0.05, 0.95, nrec) * (nz - 1) * h
    rng = np.random.default_rng(1000 * seed + iteration)
    shots = []
    for i in range(nvint):
        for k in rng.integers(0, nsrc, size=shots_per_vintage):
            shots.append(Shot(i, nt, np.array([xs, 0.0, src_z[k]]), rec))
    extra = {"src_z": src_z, "iteration": iteration}
    desc = (f"2D time-lapse crosswell, {nx}x{nz} @ {h} m, {nvint} vintages x {shots_per_vintage} "
            f"of {nsrc} shots (with replacement), {nrec} receivers, T = {T / 1000:g} s")
    if rock is not None:
        extra.update(vp=rock[0], rho=rock[1], phi=rock[2],
                     sat=[saturation * plume_mask((nz, nx), h, i + 1, nvint) for i in range(nvint)])
        return Workload(name, 2, h, nbl, dt, 0.015, vmax, 0.4, vs, shots,
                        desc + f", reservoir rock, CO2 saturation up to {saturation:g}",
                        v0=list(vs), extra=extra)
    v0 = smooth_background(v_base, h)
    return Workload(name, 2, h, nbl, dt, 0.015, vmax, 0.4, vs, shots, desc, v0=[v0] * nvint,
                    extra=extra)


def _c6() -> Workload:
    return timelapse_survey()


def _c7() -> Workload:
    return timelapse_survey("c7_timelapse_rock", rock_seed=7)


_CONFIGS = {"c1_fwd": _c1, "c2_grad": _c2, "c3_autograd": _c3, "c4_uneven": _c4,
            "c5_3d": _c5, "c5_crop": _c5_crop, "c6_timelapse": _c6,
            "c7_timelapse_rock": _c7}


def probe_table(kind: str, nt: int, r: int = 0, seed: int = 0, freqs=None, dtype=np.float32):
    """Coefficients C [r][nt] (dtype) and weights s [r] (float64) of a probed gradient:
    'identity' (r = nt, s = 1), 'rademacher' (seeded +-1 rows, s = 1/r) or 'dft' (the real DFT
    of length N = nt - 1 over the levels k = 1..nt-1 at the integer frequencies `freqs`: a cos
    row, and a sin row unless f is 0 or N/2, with weights 1/N for f = 0 and N/2, 2/N otherwise;
    all frequencies 0..N/2 give a complete orthogonal basis).  Column 0 is zero."""
    if kind == "identity":
        C = np.eye(nt, dtype=dtype)
        C[0, 0] = 0.0
        return C, np.ones(nt)
    if kind == "rademacher":
        rng = np.random.default_rng(seed)
        C = np.where(rng.random((r, nt)) < 0.5, -1.0, 1.0).astype(dtype)
        C[:, 0] = 0.0
        return C, np.full(r, 1.0 / r)
    if kind == "dft":
        N = nt - 1
        k = np.arange(1, nt)
        rows, wts = [], []
        for f in freqs:
            edge = f == 0 or 2 * f == N
            rows.append(np.cos(2 * np.pi * f * (k - 1) / N))
            wts.append((1.0 if edge else 2.0) / N)
            if not edge:
                rows.append(np.sin(2 * np.pi * f * (k - 1) / N))
                wts.append(2.0 / N)
        C = np.zeros((len(rows), nt), dtype=np.float64)
        C[:, 1:] = np.array(rows)
        return C.astype(dtype), np.array(wts)
    raise ValueError(kind)


def config_names():
    return list(_CONFIGS)


def make_config(name: str) -> Workload:
    """Build one of the named workloads (c1_fwd, c2_grad, c3_autograd, c4_uneven, c5_3d, c5_crop,
    c6_timelapse, c7_timelapse_rock)."""
    return _CONFIGS[name]()


# --------------------------------------------------------------------------------------
# small workloads for tests (sizes the oracle finishes in seconds)
# --------------------------------------------------------------------------------------
def small_2d(nx: int = 90, nz: int = 60, h: float = 10.0, nbl: int = 12, T: float = 400.0,
             nshot: int = 3, seed: int = 5, nrec: Optional[int] = None, windows: Optional[list] = None,
             T_per_shot: Optional[list] = None, perturb: float = 0.05) -> Workload:
    """A small layered/perturbed 2D survey: off-grid sources, receivers near the top.

    ``windows`` (list of widths) gives one model window per shot (uneven batching);
    ``T_per_shot`` gives each shot its own duration.
    """
    if windows is None:
        widths = [nx]
    else:
        widths = list(windows)
    vbig = layered_velocity((nz, max(widths)), vmin=1.5, vmax=3.0) * \
        (1.0 + perturb * smooth_perturbation((nz, max(widths)), h, 80.0, seed))
    vmax = float(vbig.max())
    dt = 0.4 * h / vmax
    vs = [np.ascontiguousarray(vbig[:, :w]) for w in widths]
    shots = []
    n = nshot if windows is None else len(widths)
    for s in range(n):
        wi = 0 if windows is None else s
        w = widths[wi]
        T_s = T if T_per_shot is None else T_per_shot[s]
        nt = int(math.ceil(T_s / dt - 1e-9)) + 1
        xs = (s + 0.5) * (w - 1) * h / n if windows is None else 0.37 * (w - 1) * h
        src = np.array([xs + 0.3 * h, 0.0, 2.4 * h])
        k = w if nrec is None else nrec
        rec = np.zeros((k, 3))
        rec[:, 0] = np.linspace(0.5 * h, (w - 1.6) * h, k)
        rec[:, 2] = 3.3 * h
        shots.append(Shot(wi, nt, src, rec))
    v0 = [smooth_background(v, h, 3 * h) for v in vs]
    return Workload("small_2d", 2, h, nbl, dt, 0.015, vmax, 0.4, vs, shots,
                    "small 2D test survey", v0=v0)


def small_3d(n=(24, 20, 22), h: float = 12.5, nbl: int = 8, T: float = 300.0, seed: int = 7,
             nrec_side: int = 5, nshot: int = 1) -> Workload:
    """A small layered/perturbed 3D survey with off-grid source and a receiver patch."""
    nz, ny, nx = n
    v = layered_velocity((nz, ny, nx), vmin=1.5, vmax=3.0) * \
        (1.0 + 0.05 * smooth_perturbation((nz, ny, nx), h, 80.0, seed))
    vmax = float(v.max())
    dt, nt = cfl_time_grid(T, h, vmax)
    gx = np.linspace(0.7 * h, (nx - 1.8) * h, nrec_side)
    gy = np.linspace(0.4 * h, (ny - 1.3) * h, nrec_side)
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    rec = np.zeros((nrec_side * nrec_side, 3))
    rec[:, 0] = X.ravel()
    rec[:, 1] = Y.ravel()
    rec[:, 2] = 2.6 * h
    shots = []
    for s in range(nshot):
        src = np.array([(0.45 + 0.1 * s) * (nx - 1) * h + 0.21 * h,
                        0.52 * (ny - 1) * h - 0.33 * h, 2.2 * h])
        shots.append(Shot(0, nt, src, rec))
    v0 = [smooth_background(v, h, 3 * h)]
    return Workload("small_3d", 3, h, nbl, dt, 0.015, vmax, 0.4, [v], shots,
                    "small 3D test survey", v0=v0)
