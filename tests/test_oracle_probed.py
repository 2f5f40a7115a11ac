"""Pins of the oracle's probed gradient (`gradient_probed`): the estimate of J^T dd from r sums
over the time axis that replaces the stored wavefield (randomized trace estimation, and the
on-the-fly Fourier variant).

* brute force: on a tiny grid the forward and adjoint histories come from a direct sparse
  space-time solve, and the estimate is the double sum -(1/dt^2) w^T (M x I) b with
  M = C^T diag(s) C, for a random table;
* identity table: the exact gradient;
* the complete real DFT basis with Parseval weights: the exact gradient (the identity
  sum_k a_k b_k = sum_f weighted Fourier products);
* Rademacher rows with s = 1/r: unbiased (the mean over independent draws approaches the exact
  gradient within its standard error);
* linear in dd and in s.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import shot_kwargs
from test_oracle_pins import _brute


def _tiny():
    rng = np.random.default_rng(5)
    shape, nbl, h, nt = (8, 10), 2, 10.0, 21
    src = np.array([27.0, 0.0, 13.0])
    rec = np.array([[3.0, 0.0, 9.0], [41.0, 0.0, 22.0]])
    m = 1.0 / (1.5 + rng.uniform(0, 1.5, shape)) ** 2
    vref, dt = 3.0, 0.4 * h / 3.0
    q = rng.standard_normal(nt)
    dd = rng.standard_normal((nt, len(rec)))
    return m, q, dd, dict(src=src, rec=rec, h=h, dt=dt, nbl=nbl, vref=vref)


def test_probed_gradient_matches_the_brute_force_double_sum():
    m, q, dd, kw = _tiny()
    nt = len(q)
    sysm = _brute(m, q, kw["src"], kw["rec"], kw["h"], kw["dt"], kw["nbl"], kw["vref"])
    K, N = sysm["K"], sysm["N"]
    u = sysm["lu"].solve(sysm["Sbig"] @ q[:-1]).reshape(K, N)           # u^1..u^{nt-1}
    U = np.vstack([np.zeros((2, N)), u])                                # u^{-1}, u^0, u^1, ...
    b = U[2:] - 2 * U[1:-1] + U[:-2]                                    # b^1..b^{nt-1}
    w = sysm["lu"].solve(sysm["Rbig"].T @ dd[1:].ravel(), trans="T").reshape(K, N)   # w^1..w^{nt-1}
    rng = np.random.default_rng(8)
    r = 5
    C = rng.standard_normal((r, nt))
    s = rng.uniform(0.5, 2.0, r)
    M = C[:, 1:].T @ np.diag(s) @ C[:, 1:]                              # levels 1..nt-1
    g_ref = -(np.einsum("kp,kl,lp->p", w, M, b) / kw["dt"] ** 2).reshape(m.shape)
    g = O.gradient_probed(m, q, dd, C=C, s=s, **kw)
    assert np.max(np.abs(g - g_ref)) <= 1e-12 * np.abs(g_ref).max()


@pytest.mark.parametrize("kind", ["identity", "dft"])
def test_complete_tables_give_the_exact_gradient(kind):
    wl = W.small_2d(nshot=1, T=120.0)
    kw, nt = shot_kwargs(wl, 0), wl.shots[0].nt
    q, m = wl.q(0), wl.m(0)
    dd = W.synthetic_residual(nt, len(wl.shots[0].rec), wl.dt, wl.f0, 4)
    C, s = W.probe_table(kind, nt, freqs=range((nt - 1) // 2 + 1), dtype=np.float64)
    assert C.shape[0] == nt - (0 if kind == "identity" else 1)
    g = O.gradient(m, q, dd, **kw)
    gp = O.gradient_probed(m, q, dd, C=C, s=s, **kw)
    assert np.max(np.abs(gp - g)) <= 1e-11 * np.abs(g).max()


def test_rademacher_probes_are_unbiased():
    m, q, dd, kw = _tiny()
    nt = len(q)
    g = O.gradient(m, q, dd, **kw)
    tables = [W.probe_table("rademacher", nt, r=2, seed=100 + i, dtype=np.float64) for i in range(400)]
    draws = np.array([O.gradient_probed(m, q, dd, C=C, s=s, **kw) for C, s in tables])
    mean, se = draws.mean(0), draws.std(0, ddof=1) / np.sqrt(len(draws))
    scale = np.abs(g).max()
    z = np.abs(mean - g) / np.maximum(se, 1e-6 * scale)
    assert np.median(z) < 1.5 and z.max() < 5.0
    # a single draw is far from exact (the estimate is noisy), the average much closer
    assert np.abs(draws[0] - g).max() > 10 * np.abs(mean - g).max()


def test_probed_gradient_is_linear_in_the_residual_and_the_weights():
    m, q, dd, kw = _tiny()
    C, s = W.probe_table("rademacher", len(q), r=4, seed=3, dtype=np.float64)
    g1 = O.gradient_probed(m, q, dd, C=C, s=s, **kw)
    assert np.allclose(O.gradient_probed(m, q, 2 * dd, C=C, s=s, **kw), 2 * g1, rtol=1e-13, atol=0)
    assert np.allclose(O.gradient_probed(m, q, dd, C=C, s=3 * s, **kw), 3 * g1, rtol=1e-13, atol=0)
