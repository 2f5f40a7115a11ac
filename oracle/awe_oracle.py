"""FP64 CPU oracle of the acoustic forward solve and its adjoint-state gradient.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It shares no code with the HIP library
(no kernels, headers, tables or pre/post-processing); both read the same seeded
float32 inputs and nothing else.

What is computed (paper, section "Wave-equation-based inversion", equation
eq-fwi and the two Julia listings that follow it):

    F(m) = P_r A(m)^{-1} P_s^T,   phi(m) = 1/2 || F(m) q - d ||^2,
    pullback of y = F q:  (J^T dy, F^T dy),   gradient g = J^T (F(m) q - d),

with m the squared slowness.  The paper does not give a discretisation; this
module fixes one (the readings are listed in the design notes of the repository)
and then computes its *exact* discrete operators:

  * grid: computational grid = physical grid + nbl cells on both ends of every
    axis, arrays indexed (z, x) or (z, y, x); fields are zero outside the grid;
  * L_h: 8th-order central Laplacian, coefficients STENCIL below, per axis;
  * damping eta = sum over axes of eta1(d), eta1(d) = 3 ln(1/R) / (2 L vref) (d/nbl)^2,
    d = cells past the inner edge of the border, L = nbl h; eta does not depend on m;
  * time stepping, row k = 1 .. nt-1 of A u = s (u^{-1} = u^0 = 0):
        B u^k + C u^{k-1} + E u^{k-2} = s^{k-1},
        B = m/dt^2 + eta/(2dt),  C = -(2m/dt^2 + L_h),  E = m/dt^2 - eta/(2dt);
  * P_r: bilinear / trilinear interpolation weights R(x_r), d^n = R u^n, n = 0..nt-1;
    P_s^T = R(x_s)^T / h^ndim, so s^n = R(x_s)^T q^n / h^ndim;
  * adjoint: A^T w = P_r^T dd solved backward from w^{nt} = w^{nt+1} = 0;
    (F^T dd)^n = R(x_s) w^{n+1} / h^ndim, n = 0..nt-2, and 0 at n = nt-1;
  * Jacobian: dA/dm_p acts on u as (u^k - 2u^{k-1} + u^{k-2})_p / dt^2 on row k, so
        J dm = P_r du,   A du = -dm (u^k - 2u^{k-1} + u^{k-2}) / dt^2,
        J^T r = -sum_k w^k (u^k - 2u^{k-1} + u^{k-2}) / dt^2  with  A^T w = P_r^T r.

Every routine is dtype-generic: float64 is the reference, complex128 serves the
complex-step checks and float32 estimates the rounding floor of a float32
implementation.  Units: h in m, t in ms, m in ms^2/m^2, velocities in km/s.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

__all__ = ["STENCIL", "STENCIL_EXACT", "laplacian", "damping_profile", "interp_nodes",
           "restriction", "Propagator", "forward", "adjoint", "born", "gradient", "gradient_probed",
           "objective", "fold_edge", "stability_limit", "slowness2", "velocity_gradient",
           "PATCHY_CONSTANTS", "patchy", "patchy_vjp"]

# 8th-order central second-derivative weights c0, c1..c4 (standard Taylor-series weights).
STENCIL_EXACT = (Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315),
                 Fraction(-1, 560))
STENCIL = tuple(float(c) for c in STENCIL_EXACT)


def stability_limit(ndim: int) -> float:
    """Largest v dt / h for which undamped leapfrog with this stencil is stable: 2/sqrt(ndim * S),
    S = |c0| + 2 sum |c_r| = the stencil symbol's magnitude at the Nyquist wavenumber."""
    S = abs(STENCIL[0]) + 2.0 * sum(abs(c) for c in STENCIL[1:])
    return 2.0 / math.sqrt(ndim * S)


# --------------------------------------------------------------------------------------
# spatial operators
# --------------------------------------------------------------------------------------
def laplacian(u: np.ndarray, h: float) -> np.ndarray:
    """(L_h u)_p = h^-2 sum_axes [c0 u_p + sum_r c_r (u_{p+r e} + u_{p-r e})], zero outside."""
    nd = u.ndim
    up = np.pad(u, 4)
    out = (nd * STENCIL[0]) * u
    for ax in range(nd):
        for r in range(1, 5):
            lo = [slice(4, 4 + n) for n in u.shape]
            hi = list(lo)
            lo[ax] = slice(4 - r, 4 - r + u.shape[ax])
            hi[ax] = slice(4 + r, 4 + r + u.shape[ax])
            out = out + STENCIL[r] * (up[tuple(lo)] + up[tuple(hi)])
    return out / (h * h)


def damping_profile(shape, nbl: int, h: float, vref: float, R: float = 1e-3) -> np.ndarray:
    """eta = sum over axes of eta1(d_axis) on the computational grid (units ms/m^2)."""
    eta = np.zeros(shape)
    if nbl == 0:
        return eta
    amp = 3.0 * math.log(1.0 / R) / (2.0 * nbl * h * vref)
    for ax, n in enumerate(shape):
        i = np.arange(n)
        d = np.maximum(np.maximum(nbl - i, i - (n - 1 - nbl)), 0)
        prof = amp * (d / nbl) ** 2
        eta = eta + prof.reshape([n if a == ax else 1 for a in range(len(shape))])
    return eta


def interp_nodes(pos, shape, h: float, nbl: int):
    """Grid nodes and bilinear/trilinear weights of a point at physical (x, y, z) metres.

    Returns a list of (index tuple, weight).  The node index along an axis is
    floor(c / h + nbl), the fractional part f gives weights (1 - f, f).
    """
    nd = len(shape)
    coords = (pos[2], pos[0]) if nd == 2 else (pos[2], pos[1], pos[0])
    base, frac = [], []
    for c, n in zip(coords, shape):
        g = c / h + nbl
        i0 = int(math.floor(g))
        if i0 < 0 or i0 > n - 2:
            raise ValueError(f"position {pos} is outside the computational grid")
        base.append(i0)
        frac.append(g - i0)
    nodes = []
    for corner in range(1 << nd):
        idx, w = [], 1.0
        for a in range(nd):
            bit = (corner >> a) & 1
            idx.append(base[a] + bit)
            w *= frac[a] if bit else 1.0 - frac[a]
        nodes.append((tuple(idx), w))
    return nodes


def restriction(positions, shape, h: float, nbl: int) -> sp.csr_matrix:
    """Sparse interpolation matrix (npos x N): row r holds the weights of position r."""
    N = int(np.prod(shape))
    rows, cols, vals = [], [], []
    for r, pos in enumerate(np.atleast_2d(positions)):
        for idx, w in interp_nodes(pos, shape, h, nbl):
            rows.append(r)
            cols.append(np.ravel_multi_index(idx, shape))
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(np.atleast_2d(positions)), N))


def fold_edge(g_comp: np.ndarray, nbl: int) -> np.ndarray:
    """Adjoint of edge replication: every border cell is added onto the physical edge cell it copies.

    Along one axis replication is E[j, i] = 1 when clip(j - nbl, 0, n - 1) == i; the fold
    applies E^T axis by axis.
    """
    out = np.asarray(g_comp)
    for ax in range(out.ndim):
        nc = out.shape[ax]
        n = nc - 2 * nbl
        E = np.zeros((nc, n))
        E[np.arange(nc), np.clip(np.arange(nc) - nbl, 0, n - 1)] = 1.0
        out = np.moveaxis(np.tensordot(E.T, np.moveaxis(out, ax, 0), axes=1), 0, ax)
    return out


# --------------------------------------------------------------------------------------
# time stepping
# --------------------------------------------------------------------------------------
class Propagator:
    """One shot's discrete system: m, eta, dt, h, source and receiver interpolation."""

    def __init__(self, m, src, rec, *, h, dt, nbl, vref, R=1e-3, dtype=None):
        self.dtype = np.result_type(m, np.float64) if dtype is None else np.dtype(dtype)
        self.m = np.asarray(m).astype(self.dtype)
        self.shape = self.m.shape
        self.nd = self.m.ndim
        self.h = self.dtype.type(h) if self.dtype.kind == "f" else h
        self.dt = dt
        self.eta = damping_profile(self.shape, nbl, h, vref, R).astype(self.dtype)
        self.Ps = restriction(np.asarray(src, dtype=np.float64).reshape(1, 3), self.shape, h, nbl)
        self.Pr = restriction(np.asarray(rec, dtype=np.float64).reshape(-1, 3), self.shape, h, nbl)
        if self.dtype == np.float32:
            self.Ps = self.Ps.astype(np.float32)
            self.Pr = self.Pr.astype(np.float32)
        self.hd = h ** self.nd
        dt_ = self.dtype.type(dt) if self.dtype.kind == "f" else dt
        self.dt2 = dt_ * dt_
        self.half_eta_dt = self.eta * (dt_ / 2)
        self.den = self.m + self.half_eta_dt

    def step(self, u1, u2, rhs):
        """Solve row k for u^k given u^{k-1} = u1, u^{k-2} = u2 and the right-hand side s^{k-1}:
        u^k = [dt^2 (L_h u1 + rhs) + m (2 u1 - u2) + (eta dt / 2) u2] / (m + eta dt / 2)."""
        return (self.dt2 * (laplacian(u1, self.h) + rhs) + self.m * (2 * u1 - u2)
                + self.half_eta_dt * u2) / self.den

    def inject_source(self, qk):
        return (self.Ps.T @ np.array([qk])).reshape(self.shape) / self.hd

    def record(self, u):
        return self.Pr @ u.ravel()

    def inject_receivers(self, ddk):
        return (self.Pr.T @ ddk).reshape(self.shape)

    def sample_source(self, w):
        return (self.Ps @ w.ravel())[0] / self.hd


def _zeros(P, dtype=None):
    return np.zeros(P.shape, dtype=P.dtype if dtype is None else dtype)


def _forward_fields(P: Propagator, q, nt, callback=None):
    """March u^1..u^{nt-1}; calls callback(k, u^k, u^{k-1}, u^{k-2}); returns traces [nt][nrec]."""
    dtype = np.result_type(P.dtype, np.asarray(q).dtype)
    u2 = _zeros(P, dtype)
    u1 = _zeros(P, dtype)
    d = np.zeros((nt, P.Pr.shape[0]), dtype=dtype)
    d[0] = P.record(u1)
    if callback is not None:
        callback(0, u1, u2, u2)
    for k in range(1, nt):
        u = P.step(u1, u2, P.inject_source(q[k - 1]))
        d[k] = P.record(u)
        if callback is not None:
            callback(k, u, u1, u2)
        u2, u1 = u1, u
    return d


def forward(m, q, src, rec, *, h, dt, nbl, vref, R=1e-3, dtype=None):
    """d = F(m) q: traces [nt][nrec] of one shot (nt = len(q))."""
    P = Propagator(m, src, rec, h=h, dt=dt, nbl=nbl, vref=vref, R=R, dtype=dtype)
    q = np.asarray(q).astype(np.result_type(P.dtype, np.asarray(q).dtype))
    return _forward_fields(P, q, len(q))


def adjoint(m, dd, src, rec, *, h, dt, nbl, vref, R=1e-3, dtype=None):
    """v = F(m)^T dd: one value per source sample (length nt = dd.shape[0])."""
    P = Propagator(m, src, rec, h=h, dt=dt, nbl=nbl, vref=vref, R=R, dtype=dtype)
    dd = np.asarray(dd)
    nt = dd.shape[0]
    dtype = np.result_type(P.dtype, dd.dtype)
    w1 = _zeros(P, dtype)   # w^{k+1}
    w2 = _zeros(P, dtype)   # w^{k+2}
    v = np.zeros(nt, dtype=dtype)
    for k in range(nt - 1, 0, -1):
        w = P.step(w1, w2, P.inject_receivers(dd[k]))
        v[k - 1] = P.sample_source(w)
        w2, w1 = w1, w
    return v


def born(m, q, dm, src, rec, *, h, dt, nbl, vref, R=1e-3, dtype=None):
    """J dm: linearised traces [nt][nrec]; du solves A du = -dm (u^k - 2u^{k-1} + u^{k-2}) / dt^2."""
    P = Propagator(m, src, rec, h=h, dt=dt, nbl=nbl, vref=vref, R=R, dtype=dtype)
    dm = np.asarray(dm).astype(np.result_type(P.dtype, np.asarray(dm).dtype))
    q = np.asarray(q)
    nt = len(q)
    dtype = np.result_type(P.dtype, q.dtype, dm.dtype)
    state = {"du1": _zeros(P, dtype), "du2": _zeros(P, dtype)}
    out = np.zeros((nt, P.Pr.shape[0]), dtype=dtype)

    def cb(k, u, u1, u2):
        if k == 0:
            return
        rhs = -dm * (u - 2 * u1 + u2) / P.dt2
        du = P.step(state["du1"], state["du2"], rhs)
        out[k] = P.record(du)
        state["du2"], state["du1"] = state["du1"], du

    _forward_fields(P, q.astype(dtype), nt, cb)
    return out


def gradient(m, q, dd, src, rec, *, h, dt, nbl, vref, R=1e-3, dtype=None, segment=None,
             return_traces=False):
    """g = J^T dd on the computational grid (shape of m).

    The forward wavefield is needed in reverse time order.  With ``segment=None``
    every u^k is kept; otherwise restart pairs (u^k, u^{k-1}) are kept every
    ``segment`` steps and each segment is recomputed into a buffer during the
    reverse sweep (the recomputation repeats the same arithmetic, so the result
    does not depend on ``segment``).
    """
    P = Propagator(m, src, rec, h=h, dt=dt, nbl=nbl, vref=vref, R=R, dtype=dtype)
    q = np.asarray(q)
    dd = np.asarray(dd)
    nt = len(q)
    dtype = np.result_type(P.dtype, q.dtype, dd.dtype)
    q = q.astype(dtype)
    K = nt if segment is None else max(1, int(segment))

    # forward sweep: keep restart pairs at k = 0, K, 2K, ... (pair = (u^k, u^{k-1}))
    restarts = {}
    full = {} if segment is None else None
    zero = _zeros(P, dtype)

    def keep(k, u, u1, u2):
        if full is not None:
            full[k] = u
        elif k % K == 0:
            restarts[k] = (u, u1)

    traces = _forward_fields(P, q, nt, keep)

    def fields_of_segment(k0):
        """u^j for j in [k0, min(k0 + K, nt)) recomputed from the restart pair at k0."""
        if full is not None:
            return {j: full[j] for j in range(k0, min(k0 + K, nt))}
        u1, u2 = restarts[k0]
        out = {k0: u1}
        for j in range(k0 + 1, min(k0 + K, nt)):
            u = P.step(u1, u2, P.inject_source(q[j - 1]))
            out[j] = u
            u2, u1 = u1, u
        return out

    g = np.zeros(P.shape, dtype=dtype)
    w1 = zero.copy()
    w2 = zero.copy()
    cache = {}
    for k in range(nt - 1, 0, -1):
        w = P.step(w1, w2, P.inject_receivers(dd[k]))
        for j in (k, k - 1, k - 2):
            if j >= 0 and j not in cache:
                cache.update(fields_of_segment((j // K) * K))
        uk, uk1 = cache[k], cache[k - 1]
        uk2 = cache[k - 2] if k >= 2 else zero
        g -= w * (uk - 2 * uk1 + uk2) / P.dt2
        for j in [j for j in cache if j > k]:
            del cache[j]
        w2, w1 = w1, w
    if return_traces:
        return g, traces
    return g


def gradient_probed(m, q, dd, src, rec, C, s, *, h, dt, nbl, vref, R=1e-3, dtype=None):
    """Estimate of J^T dd from r probes of the time axis instead of the stored wavefield.

    The section "Remaining challenges" names the memory of the adjoint-state gradient as a
    bottleneck and cites randomized trace estimation (Louboutin and Herrmann, 2022 and 2023);
    on-the-fly Fourier transforms (Witte et al., 2019, cited in "Wave-equation-based
    inversion") are the deterministic variant.  Both replace the nt stored fields by a few
    weighted sums over time.  Written out: the exact gradient (see `gradient`) is
        g = -(1/dt^2) sum_k w^k b^k,  b^k = u^k - 2u^{k-1} + u^{k-2},  k = 1..nt-1,
    i.e. at every point the inner product of the two time series w and b.  With a table
    C [r][nt] (column k weights level k) and weights s [r], the forward sweep keeps the r fields
    B_j = sum_k C[j,k] b^k, the adjoint sweep the r fields A_j = sum_k C[j,k] w^k, and
        g~ = -(1/dt^2) sum_j s_j A_j B_j = -(1/dt^2) sum_{k,l} w^k M_kl b^l,  M = C^T diag(s) C.
    g~ = g when M = I (C = I, or the rows of a complete orthogonal basis with the inverse
    squared norms as weights, e.g. the real DFT); with Rademacher rows and s = 1/r, E[M] = I
    and g~ is Hutchinson's unbiased estimate.  Column 0 of C is not used (w^0, b^0 do not
    enter).  Memory: 2 r fields instead of nt.
    """
    P = Propagator(m, src, rec, h=h, dt=dt, nbl=nbl, vref=vref, R=R, dtype=dtype)
    q = np.asarray(q)
    dd = np.asarray(dd)
    nt = len(q)
    dtype = np.result_type(P.dtype, q.dtype, dd.dtype)
    C = np.asarray(C, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    r = C.shape[0]
    assert C.shape[1] >= nt and s.shape == (r,)
    B = np.zeros((r,) + P.shape, dtype=dtype)
    A = np.zeros((r,) + P.shape, dtype=dtype)

    def probe_forward(k, u, u1, u2):
        if k >= 1:
            b = u - 2 * u1 + u2
            for j in range(r):
                B[j] += C[j, k] * b

    _forward_fields(P, q.astype(dtype), nt, probe_forward)
    w1 = _zeros(P, dtype)
    w2 = _zeros(P, dtype)
    for k in range(nt - 1, 0, -1):
        w = P.step(w1, w2, P.inject_receivers(dd[k]))
        for j in range(r):
            A[j] += C[j, k] * w
        w2, w1 = w1, w
    g = np.zeros(P.shape, dtype=dtype)
    for j in range(r):
        g -= s[j] * A[j] * B[j] / P.dt2
    return g


def objective(d_pred, d_obs):
    """phi = 1/2 sum (d_pred - d_obs)^2 (plain Euclidean sum; no conjugation for complex input)."""
    r = np.asarray(d_pred) - np.asarray(d_obs)
    return 0.5 * np.sum(r * r)


def slowness2(v):
    """m = 1/v^2: the squared slowness of a compressional wavespeed (the time-lapse operator of
    "Putting it all together" is parameterised by v, the wave operators by m)."""
    v = np.asarray(v, dtype=np.float64)
    return 1.0 / (v * v)


def velocity_gradient(v, g_m):
    """Chain rule of m = 1/v^2: dphi/dv = dphi/dm * dm/dv = -2 g_m / v^3 (elementwise)."""
    v = np.asarray(v, dtype=np.float64)
    return -2.0 * np.asarray(g_m, dtype=np.float64) / (v * v * v)


# Rock and fluid constants of the patchy-saturation model in "Putting it all together": bulk
# moduli of the mineral, the brine and the CO2 (Pa) and the densities of the CO2 and the brine
# (kg/m^3).
PATCHY_CONSTANTS = {"k_min": 36.6e9, "k_brine": 2.735e9, "k_co2": 0.125e9,
                    "rho_co2": 700.0, "rho_brine": 1000.0}


def patchy(sw, vp, rho, phi, consts=None):
    """Rock physics R of "Putting it all together": patchy CO2 saturation sw lowers the wavespeed.

    Inputs per cell: saturation sw in [0, 1], brine-saturated wavespeed vp (km/s), density rho
    (kg/m^3), porosity phi.  The shear wavespeed is taken as vp / sqrt(3).  Moduli of the
    brine-saturated rock: shear mu = rho vs^2, bulk K1 = rho vp^2 - 4 mu / 3.  Gassmann's
    relation, written with r(K) = K / (k_min - K), says r(K_sat) - r(K_fluid) / phi is the same
    for every pore fluid (it is r of the dry frame), which swaps brine for CO2:
        r(K2) = r(K1) - r(k_brine) / phi + r(k_co2) / phi,   K2 = k_min r / (1 + r).
    The patchy mixture's P-wave modulus is the saturation-weighted harmonic average of the two
    P-wave moduli K + 4 mu / 3; the density mixes the fluids linearly; vp_new follows from the
    P-wave modulus and density.  Returns (vp_new in km/s, rho_new).  dtype-generic (complex
    inputs give complex-step derivatives)."""
    c = dict(PATCHY_CONSTANTS if consts is None else consts)
    as_arr = lambda a: np.asarray(a) if np.iscomplexobj(a) else np.asarray(a, dtype=np.float64)
    sw, vp, rho, phi = (as_arr(a) for a in (sw, vp, rho, phi))
    vp_si = 1e3 * vp                                        # km/s -> m/s
    vs_si = vp_si / math.sqrt(3.0)
    mu = rho * vs_si ** 2
    k_brine_rock = rho * (vp_si ** 2 - 4.0 / 3.0 * vs_si ** 2)

    def r(k):
        return k / (c["k_min"] - k)

    r_co2_rock = r(k_brine_rock) - r(c["k_brine"]) / phi + r(c["k_co2"]) / phi
    k_co2_rock = c["k_min"] / (1.0 / r_co2_rock + 1.0)
    p_brine = k_brine_rock + 4.0 / 3.0 * mu                 # P-wave moduli
    p_co2 = k_co2_rock + 4.0 / 3.0 * mu
    p_mix = 1.0 / ((1.0 - sw) / p_brine + sw / p_co2)
    rho_new = rho + phi * sw * (c["rho_co2"] - c["rho_brine"])
    vp_new = np.sqrt(p_mix / rho_new) / 1e3
    return vp_new, rho_new


def patchy_vjp(sw, vp, rho, phi, g_vp, g_rho=None, consts=None, step=1e-30):
    """Pullback of R with respect to the saturation: g_sw = g_vp dvp_new/dsw + g_rho drho_new/dsw
    (R is elementwise, so its Jacobian in sw is diagonal).  The derivatives are complex-step
    derivatives Im R(sw + i step) / step, exact up to rounding for this analytic map."""
    sw = np.asarray(sw, dtype=np.float64)
    vp_c, rho_c = patchy(sw + 1j * step, vp, rho, phi, consts)
    g = np.asarray(g_vp, dtype=np.float64) * (vp_c.imag / step)
    if g_rho is not None:
        g = g + np.asarray(g_rho, dtype=np.float64) * (rho_c.imag / step)
    return g
