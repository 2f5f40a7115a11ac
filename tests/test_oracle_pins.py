"""Pins of the CPU oracle against what mathematics fixes, independent of the oracle's own code.

Each test compares the oracle with something it does not compute itself: closed forms
(stencil moments, polynomial exactness, analytic Green's functions), a brute-force sparse
assembly of the whole space-time system, exact identities of the discrete operators
(adjointness, reciprocity, complex-step derivatives, Taylor remainders) and invariances
(time shift, mirror symmetry, linearity).  No GPU is involved.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.integrate import quad

import oracle as O
import workloads as W
from helpers import shot_kwargs, rel_l2


def _ricker64(t, f0, t0=None):
    t0 = 1.5 / f0 if t0 is None else t0
    a = (math.pi * f0 * (np.asarray(t) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


# ------------------------------------------------------------------------------ stencil
def test_stencil_moments_fix_the_8th_order_weights():
    c = O.STENCIL_EXACT
    # a symmetric 9-point stencil is the 8th-order second derivative iff its even moments are
    # (0, 2, 0, 0, 0) for powers r^0, r^2, r^4, r^6, r^8: five equations, five unknowns
    assert c[0] + 2 * sum(c[1:]) == 0
    assert 2 * sum(c[r] * r ** 2 for r in range(1, 5)) == 2
    for j in (2, 3, 4):
        assert sum(c[r] * r ** (2 * j) for r in range(1, 5)) == 0
    assert O.STENCIL == tuple(float(x) for x in c)


def test_laplacian_exact_on_degree_9_polynomials_and_not_beyond():
    h = 0.5
    z = (np.arange(21) * h)[:, None]
    x = (np.arange(24) * h)[None, :]
    X, Z = x - 4.7, z - 3.1
    u = X ** 9 + 2 * Z ** 8 + X ** 3 * Z ** 4
    exact = 72 * X ** 7 + 112 * Z ** 6 + 6 * X * Z ** 4 + 12 * X ** 3 * Z ** 2
    L = O.laplacian(u, h)
    sl = (slice(4, -4), slice(4, -4))
    assert np.max(np.abs(L[sl] - exact[sl])) <= 1e-9 * np.abs(exact[sl]).max()
    # degree 10 is not reproduced: the leading error term h^8 u^(10) is visible
    u10 = X ** 10 * np.ones_like(Z)
    err = np.abs(O.laplacian(u10, h)[sl] - (90 * X ** 8 * np.ones_like(Z))[sl]).max()
    assert err > 1e-3
    # 3D: axis order (z, y, x) with the same per-axis weights
    y = (np.arange(20) * h)[None, :, None]
    z3, x3 = z[:, :, None][:, :, :], x[:, None, :]
    Y3, Z3, X3 = y - 2.2, z3 - 3.1, x3 - 4.7
    u3 = Y3 ** 7 * Z3 ** 2 + X3 ** 5
    ex3 = 42 * Y3 ** 5 * Z3 ** 2 + 2 * Y3 ** 7 + 20 * X3 ** 3
    L3 = O.laplacian(u3 * np.ones((21, 20, 24)), h)
    s3 = (slice(4, -4),) * 3
    ex3 = ex3 * np.ones((21, 20, 24))
    assert np.max(np.abs(L3[s3] - ex3[s3])) <= 1e-9 * np.abs(ex3[s3]).max()


def _lap_matrix(shape, h):
    """Kronecker-sum assembly of the Laplacian with the grid truncated (zero outside)."""
    mats = []
    for n in shape:
        diags = [np.full(n - abs(r), O.STENCIL[abs(r)]) for r in range(-4, 5)]
        mats.append(sp.diags(diags, list(range(-4, 5)), shape=(n, n)))
    L = None
    for ax, D in enumerate(mats):
        term = None
        for a, n in enumerate(shape):
            f = D if a == ax else sp.identity(n)
            term = f if term is None else sp.kron(term, f)
        L = term if L is None else L + term
    return (L / (h * h)).tocsr()


@pytest.mark.parametrize("shape", [(13, 17), (9, 11, 10)])
def test_laplacian_matches_kronecker_assembly(shape):
    rng = np.random.default_rng(3)
    u = rng.standard_normal(shape)
    h = 7.0
    ref = (_lap_matrix(shape, h) @ u.ravel()).reshape(shape)
    assert np.max(np.abs(O.laplacian(u, h) - ref)) <= 1e-14 * np.abs(ref).max()


def test_stability_limit_matches_stencil_spectrum_and_blows_up_above_it():
    # largest |eigenvalue| of the periodic 1D stencil is reached at the Nyquist wavenumber
    n = 64
    col = np.zeros(n)
    col[0] = O.STENCIL[0]
    for r in range(1, 5):
        col[r] = col[-r] = O.STENCIL[r]
    lam = np.fft.fft(col).real
    S = np.abs(lam).max()
    assert abs(O.stability_limit(2) - 2 / math.sqrt(2 * S)) < 1e-14
    assert abs(O.stability_limit(3) - 2 / math.sqrt(3 * S)) < 1e-14
    # run the undamped scheme driven by white noise just below / above the limit
    rng = np.random.default_rng(0)
    m = np.ones((40, 40))
    q = rng.standard_normal(600)
    kw = dict(src=(195.0, 0.0, 205.0), rec=np.array([[100.0, 0.0, 100.0]]), h=10.0, nbl=0, vref=1.0)
    lim = O.stability_limit(2)
    d_ok = O.forward(m, q, dt=0.98 * lim * 10.0, **kw)
    d_bad = O.forward(m, q, dt=1.05 * lim * 10.0, **kw)
    assert np.abs(d_ok).max() < 1e3 * np.abs(d_ok[:50]).max()
    assert np.abs(d_bad).max() > 1e6 * np.abs(d_ok).max()


# ------------------------------------------------------------------------------ interpolation
@pytest.mark.parametrize("nd", [2, 3])
def test_interpolation_partition_of_unity_and_linear_exactness(nd):
    rng = np.random.default_rng(11)
    shape = (30, 25) if nd == 2 else (20, 18, 22)
    h, nbl = 6.25, 5
    for _ in range(50):
        phys = [(n - 2 * nbl - 1) * h for n in shape]
        pos = np.zeros(3)
        if nd == 2:
            pos[2], pos[0] = rng.uniform(0, phys[0]), rng.uniform(0, phys[1])
        else:
            pos[2], pos[1], pos[0] = [rng.uniform(0, p) for p in phys]
        nodes = O.interp_nodes(pos, shape, h, nbl)
        assert len(nodes) == 2 ** nd
        assert abs(sum(w for _, w in nodes) - 1.0) < 1e-14
        coords = (pos[2], pos[0]) if nd == 2 else (pos[2], pos[1], pos[0])
        for a in range(nd):
            got = sum(w * (idx[a] - nbl) * h for idx, w in nodes)
            assert abs(got - coords[a]) < 1e-9
        assert all(w >= 0 for _, w in nodes)


def test_on_grid_position_is_one_node_with_unit_weight():
    nodes = O.interp_nodes((50.0, 0.0, 30.0), (40, 40), 10.0, 4)
    live = [(i, w) for i, w in nodes if w != 0.0]
    assert live == [((7, 9), 1.0)]


def test_fold_edge_is_the_adjoint_of_edge_replication():
    rng = np.random.default_rng(4)
    for shape, nbl in [((7, 9), 3), ((4, 5, 6), 2)]:
        x = rng.standard_normal(shape)
        y = rng.standard_normal(tuple(n + 2 * nbl for n in shape))
        a = np.sum(np.pad(x, nbl, mode="edge") * y)
        b = np.sum(x * O.fold_edge(y, nbl))
        assert abs(a - b) <= 1e-13 * abs(a)


# ------------------------------------------------------------------------------ analytic Green's functions
def _green2d(r, t, c, f0):
    if t <= r / c:
        return 0.0
    top = math.acosh(c * t / r)
    val, _ = quad(lambda th: _ricker64(t - (r / c) * math.cosh(th), f0), 0.0, top, limit=200)
    return val / (2 * math.pi)


def test_green_2d_homogeneous_second_order_convergence():
    """m u_tt - Lap u = delta(x) f(t):  u = (1/2pi) int_0^{acosh(ct/r)} f(t - (r/c) cosh th) dth.

    At fixed CFL the O(dt^2) time error dominates the O(h^8) space error, so halving h
    must divide the error by about 4.  The domain is large enough that no boundary wave
    reaches a receiver before T."""
    c, f0, half, T = 1.5, 0.015, 500.0, 400.0
    offs = [(300.0, 0.0), (0.0, 300.0), (-240.0, 180.0)]
    errs = []
    for h in (10.0, 5.0, 2.5):
        n = int(round(2 * half / h)) + 1
        dt = 0.4 * h / c
        nt = int(math.ceil(T / dt)) + 1
        t = np.arange(nt) * dt
        q = _ricker64(t, f0)
        rec = np.array([[half + ox, 0.0, half + oz] for ox, oz in offs])
        d = O.forward(np.full((n, n), 1.0 / c ** 2), q, (half, 0.0, half), rec, h=h, dt=dt, nbl=0, vref=c)
        ref = np.array([[_green2d(math.hypot(ox, oz), tk, c, f0) for (ox, oz) in offs] for tk in t])
        errs.append(rel_l2(d, ref))
    assert errs[2] < 0.01
    assert 3.0 <= errs[0] / errs[1] <= 5.0
    assert 3.0 <= errs[1] / errs[2] <= 5.0


def test_green_3d_homogeneous_second_order_convergence():
    """3D: u = f(t - r/c) / (4 pi r); single refinement h = 10 -> 5 m."""
    c, f0, half, T = 1.5, 0.015, 300.0, 280.0
    offs = [(150.0, 0.0, 0.0), (0.0, 0.0, 150.0), (90.0, 120.0, 0.0)]
    errs = []
    for h in (10.0, 5.0):
        n = int(round(2 * half / h)) + 1
        dt = 0.4 * h / c
        nt = int(math.ceil(T / dt)) + 1
        t = np.arange(nt) * dt
        q = _ricker64(t, f0)
        rec = np.array([[half + o[0], half + o[1], half + o[2]] for o in offs])
        d = O.forward(np.full((n, n, n), 1.0 / c ** 2), q, (half, half, half), rec, h=h, dt=dt,
                      nbl=0, vref=c)
        ref = np.stack([_ricker64(t - 150.0 / c, f0) / (4 * math.pi * 150.0) for _ in offs], axis=1)
        errs.append(rel_l2(d, ref))
    assert errs[1] < 0.02
    assert 3.0 <= errs[0] / errs[1] <= 5.0


# ------------------------------------------------------------------------------ sponge
def test_sponge_absorbs_what_a_hard_boundary_reflects():
    """Homogeneous medium: traces in a small domain with the damping border vs the same
    traces in a domain so large that nothing returns before T.  The quadratic sponge must
    keep the border reflection small; with R = 1 (no damping) the reflection is large."""
    c, h, f0, nbl, T = 2.0, 10.0, 0.015, 40, 900.0
    dt = 0.4 * h / c
    nt = int(math.ceil(T / dt)) + 1
    q = _ricker64(np.arange(nt) * dt, f0)
    n_small, pad = 81, 100
    src = np.array([400.0, 0.0, 400.0])
    rec = np.array([[100.0, 0.0, 400.0], [400.0, 0.0, 100.0], [700.0, 0.0, 700.0]])
    sh = np.array([pad * h, 0.0, pad * h])
    n_big = n_small + 2 * pad
    big = O.forward(np.full((n_big + 2 * nbl,) * 2, 1 / c ** 2), q, src + sh, rec + sh, h=h, dt=dt,
                    nbl=nbl, vref=c)
    small = O.forward(np.full((n_small + 2 * nbl,) * 2, 1 / c ** 2), q, src, rec, h=h, dt=dt,
                      nbl=nbl, vref=c)
    hard = O.forward(np.full((n_small + 2 * nbl,) * 2, 1 / c ** 2), q, src, rec, h=h, dt=dt,
                     nbl=nbl, vref=c, R=1.0)
    assert rel_l2(small, big) < 0.03
    assert rel_l2(hard, big) > 0.3


# ------------------------------------------------------------------------------ brute force
def _hat_restriction(positions, shape, h, nbl):
    """Interpolation as products of hat functions max(0, 1 - |g - p|), g = coordinate/h + nbl."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    rows = []
    for pos in positions:
        coords = (pos[2], pos[0]) if len(shape) == 2 else (pos[2], pos[1], pos[0])
        w = np.ones(shape)
        for a, c in enumerate(coords):
            w *= np.maximum(0.0, 1.0 - np.abs(c / h + nbl - grids[a]))
        rows.append(w.ravel())
    return sp.csr_matrix(np.array(rows))


def _eta(shape, nbl, h, vref, R=1e-3):
    amp = 3.0 * math.log(1.0 / R) / (2.0 * nbl * h * vref)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    eta = np.zeros(shape)
    for a, n in enumerate(shape):
        dist = np.maximum(0, np.maximum(nbl - grids[a], grids[a] - (n - 1 - nbl)))
        eta += amp * (dist / nbl) ** 2
    return eta


def _brute(m, q, src, rec, h, dt, nbl, vref):
    """Assemble the (nt-1) N space-time system A (rows k = 1..nt-1) and solve it directly."""
    shape, N, nt = m.shape, m.size, len(q)
    nd = m.ndim
    eta = _eta(shape, nbl, h, vref).ravel()
    mm = m.ravel()
    L = _lap_matrix(shape, h)
    B = sp.diags(mm / dt ** 2 + eta / (2 * dt))
    C = -(sp.diags(2 * mm / dt ** 2) + L)
    E = sp.diags(mm / dt ** 2 - eta / (2 * dt))
    K = nt - 1
    A = (sp.kron(sp.identity(K), B) + sp.kron(sp.eye(K, k=-1), C) + sp.kron(sp.eye(K, k=-2), E)).tocsc()
    S = _hat_restriction([src], shape, h, nbl).T / h ** nd          # N x 1
    R = _hat_restriction(rec, shape, h, nbl)                          # nrec x N
    Rbig = sp.kron(sp.identity(K), R).tocsr()
    Sbig = sp.kron(sp.identity(K), S).tocsr()                         # maps q^0..q^{nt-2}
    lu = spla.splu(A)
    return dict(A=A, lu=lu, R=R, Rbig=Rbig, Sbig=Sbig, S=S, K=K, N=N, shape=shape)


@pytest.mark.parametrize("nd", [2, 3])
def test_brute_force_space_time_solve(nd):
    rng = np.random.default_rng(21)
    if nd == 2:
        shape, nbl, h, nt = (8, 10), 2, 10.0, 25
        src = np.array([27.0, 0.0, 13.0])
        rec = np.array([[3.0, 0.0, 9.0], [41.0, 0.0, 22.0], [18.5, 0.0, 1.0]])
    else:
        shape, nbl, h, nt = (6, 5, 7), 1, 10.0, 15
        src = np.array([21.0, 13.0, 17.0])
        rec = np.array([[3.0, 4.0, 9.0], [33.0, 18.0, 22.0]])
    m = 1.0 / (1.5 + rng.uniform(0, 1.5, shape)) ** 2
    vref, dt = 3.0, 0.4 * h / 3.0
    q = rng.standard_normal(nt)
    kw = dict(src=src, rec=rec, h=h, dt=dt, nbl=nbl, vref=vref)
    sysm = _brute(m, q, src, rec, h, dt, nbl, vref)
    K, N = sysm["K"], sysm["N"]
    nrec = len(rec)

    # forward: A u = S q^{k-1}; d^0 = 0
    u = sysm["lu"].solve(sysm["Sbig"] @ q[:-1])
    d_ref = np.vstack([np.zeros(nrec), (sysm["Rbig"] @ u).reshape(K, nrec)])
    d = O.forward(m, q, **kw)
    assert np.max(np.abs(d - d_ref)) <= 1e-13 * np.abs(d_ref).max()

    # adjoint: F^T = S^T A^{-T} R^T, output v^{n} pairs with q^{n}; last entry 0
    dd = rng.standard_normal((nt, nrec))
    wv = sysm["lu"].solve(sysm["Rbig"].T @ dd[1:].ravel(), trans="T")
    v_ref = np.append(sysm["Sbig"].T @ wv, 0.0)
    v = O.adjoint(m, dd, **kw)
    assert np.max(np.abs(v - v_ref)) <= 1e-13 * np.abs(v_ref).max()

    # Jacobian as a dense matrix: column p = -R A^{-1} (dA/dm_p) u
    U = np.vstack([np.zeros(N), u.reshape(K, N)])                     # u^0..u^{nt-1}
    Uprev = np.vstack([np.zeros((2, N)), U[:-1]])                     # shifted copies
    D = (U - 2 * Uprev[1:] + Uprev[:-1])[1:] / dt ** 2                # rows k = 1..nt-1
    Gu = sp.csc_matrix((D.ravel(), (np.arange(K * N), np.tile(np.arange(N), K))), shape=(K * N, N))
    Jrows = -(sysm["Rbig"] @ sysm["lu"].solve(Gu.toarray()))
    J = np.vstack([np.zeros((nrec, N)), Jrows.reshape(K * nrec, N)])  # sample 0 rows are zero
    dm = rng.standard_normal(shape)
    jdm = O.born(m, q, dm, **kw)
    assert np.max(np.abs(jdm.ravel() - J @ dm.ravel())) <= 1e-12 * np.abs(J @ dm.ravel()).max()
    g = O.gradient(m, q, dd, **kw)
    g_ref = (J.T @ dd.ravel()).reshape(shape)
    assert np.max(np.abs(g - g_ref)) <= 1e-12 * np.abs(g_ref).max()


# ------------------------------------------------------------------------------ operator identities
def _setup(nd):
    wl = W.small_2d(nshot=1) if nd == 2 else W.small_3d(n=(16, 14, 15), nbl=6, T=200.0)
    return wl, wl.m(0), shot_kwargs(wl, 0), wl.shots[0].nt


@pytest.mark.parametrize("nd", [2, 3])
def test_dot_test_forward_adjoint(nd):
    wl, m, kw, nt = _setup(nd)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(nt)
    y = rng.standard_normal((nt, len(kw["rec"])))
    a = np.sum(O.forward(m, x, **kw) * y)
    b = np.sum(x * O.adjoint(m, y, **kw))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-12


@pytest.mark.parametrize("nd", [2, 3])
def test_dot_test_born_gradient(nd):
    wl, m, kw, nt = _setup(nd)
    rng = np.random.default_rng(2)
    dm = rng.standard_normal(m.shape)
    y = rng.standard_normal((nt, len(kw["rec"])))
    q = wl.q(0)
    a = np.sum(O.born(m, q, dm, **kw) * y)
    b = np.sum(dm * O.gradient(m, q, y, **kw))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-12


@pytest.mark.parametrize("nd", [2, 3])
def test_source_receiver_reciprocity(nd):
    wl, m, kw, nt = _setup(nd)
    q = wl.q(0)
    a = np.asarray(kw["src"], dtype=float)
    b = np.asarray(kw["rec"][len(kw["rec"]) // 2 + 1], dtype=float)
    base = {k: v for k, v in kw.items() if k not in ("src", "rec")}
    dab = O.forward(m, q, src=a, rec=b[None], **base)
    dba = O.forward(m, q, src=b, rec=a[None], **base)
    assert np.max(np.abs(dab - dba)) <= 1e-12 * np.abs(dab).max()


def test_complex_step_gradient_and_born():
    wl, m_true, kw, nt = _setup(2)
    m0 = wl.m(0, background=True).astype(np.float64)
    q = wl.q(0)
    d_obs = O.forward(m_true, q, **kw)
    rng = np.random.default_rng(8)
    dm = W.random_field(m0.shape, 9, smooth_cells=2.0).astype(np.float64)
    eps = 1e-20 * np.abs(m0).max() / np.abs(dm).max()
    dc = O.forward(m0 + 1j * eps * dm, q, **kw)
    dphi = O.objective(dc, d_obs).imag / eps
    g = O.gradient(m0, q, O.forward(m0, q, **kw) - d_obs, **kw)
    assert abs(dphi - np.sum(g * dm)) <= 1e-12 * abs(dphi)
    jdm_cs = dc.imag / eps
    jdm = O.born(m0, q, dm, **kw)
    assert np.max(np.abs(jdm - jdm_cs)) <= 1e-12 * np.abs(jdm_cs).max()
    del rng


def test_taylor_remainder_is_second_order():
    wl, m_true, kw, nt = _setup(2)
    m0 = wl.m(0, background=True).astype(np.float64)
    q = wl.q(0)
    d_obs = O.forward(m_true, q, **kw)
    phi = lambda mm: O.objective(O.forward(mm, q, **kw), d_obs)
    g = O.gradient(m0, q, O.forward(m0, q, **kw) - d_obs, **kw)
    dm = W.random_field(m0.shape, 12, smooth_cells=3.0).astype(np.float64)
    t0 = 0.05 * np.abs(m0).mean() / np.abs(dm).max()
    f0 = phi(m0)
    r0, r1 = [], []
    for k in range(5):
        t = t0 / 2 ** k
        f = phi(m0 + t * dm)
        r0.append(abs(f - f0))
        r1.append(abs(f - f0 - t * np.sum(g * dm)))
    rates1 = [r1[i] / r1[i + 1] for i in range(4)]
    rates0 = [r0[i] / r0[i + 1] for i in range(4)]
    assert all(3.5 <= r <= 4.5 for r in rates1), rates1
    assert all(1.7 <= r <= 2.3 for r in rates0), rates0


# ------------------------------------------------------------------------------ invariances
def test_time_shift_is_bit_exact():
    wl, m, kw, nt = _setup(2)
    q = wl.q(0).astype(np.float64)
    k = 17
    d = O.forward(m, q, **kw)
    ds = O.forward(m, np.concatenate([np.zeros(k), q[:-k]]), **kw)
    assert np.array_equal(ds[k:], d[:-k])
    assert not ds[:k].any()


def test_mirror_symmetry_is_bit_exact_on_the_two_layer_survey():
    wl = W.make_config("c1_fwd")
    d = O.forward(wl.m(0), wl.q(0), **shot_kwargs(wl, 0))
    assert np.array_equal(d[:, :50], d[:, 100:50:-1])
    assert np.abs(d).max() > 0


def test_linearity_in_the_source():
    wl, m, kw, nt = _setup(2)
    rng = np.random.default_rng(5)
    q1, q2 = rng.standard_normal(nt), rng.standard_normal(nt)
    a, b = 0.7, -1.9
    lhs = O.forward(m, a * q1 + b * q2, **kw)
    rhs = a * O.forward(m, q1, **kw) + b * O.forward(m, q2, **kw)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.abs(rhs).max()
    assert not O.forward(m, np.zeros(nt), **kw).any()


def test_gradient_does_not_depend_on_checkpoint_segment():
    wl, m, kw, nt = _setup(2)
    dd = np.random.default_rng(6).standard_normal((nt, len(kw["rec"])))
    g_full = O.gradient(m, wl.q(0), dd, **kw)
    g_seg = O.gradient(m, wl.q(0), dd, segment=7, **kw)
    assert np.array_equal(g_full, g_seg)


def test_velocity_parameterisation_chain_rule_by_finite_differences():
    """d/dv of phi(m(v)) with m = 1/v^2 and phi(m) = <a, m> + 1/2 <m, B m>: the oracle's
    velocity_gradient(v, dphi/dm) against central differences of phi along random directions."""
    rng = np.random.default_rng(11)
    v = rng.uniform(1.5, 4.5, size=40)
    a = rng.standard_normal(40)
    Bm = rng.standard_normal((40, 40))
    B = Bm @ Bm.T / 40
    phi = lambda vv: a @ O.slowness2(vv) + 0.5 * O.slowness2(vv) @ B @ O.slowness2(vv)
    gm = a + B @ O.slowness2(v)
    gv = O.velocity_gradient(v, gm)
    for _ in range(4):
        e = rng.standard_normal(40)
        eps = 1e-5
        fd = (phi(v + eps * e) - phi(v - eps * e)) / (2 * eps)
        assert abs(fd - gv @ e) <= 1e-8 * max(1.0, abs(fd))
    assert np.allclose(O.slowness2(np.array([2.0, 0.5])), [0.25, 4.0], rtol=0, atol=0)
