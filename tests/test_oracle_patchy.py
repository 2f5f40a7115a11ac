"""Pins of the oracle's patchy-saturation rock physics R ("Putting it all together").

Each test checks the oracle against something it does not compute itself: the textbook
closed form of Gassmann's equation (the oracle uses the modulus-ratio form), the identity at
zero saturation and for a CO2 that is indistinguishable from brine, the harmonic (patchy)
mixing law read off the outputs, the fluid-density mixing, and central finite differences of
the complex-step pullback.  No GPU is involved.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

C = O.PATCHY_CONSTANTS


def _gassmann_textbook(k_dry, k_fl, phi, k_min):
    """Saturated bulk modulus from the dry-frame modulus (Gassmann 1951, the usual form)."""
    b = 1.0 - k_dry / k_min
    return k_dry + b * b / (phi / k_fl + (1.0 - phi) / k_min - k_dry / (k_min * k_min))


def _rock(n=500, seed=3):
    vp, rho, phi = (a.astype(np.float64) for a in W.reservoir_rock((n,), seed))
    return vp, rho, phi


def test_zero_saturation_is_the_identity():
    vp, rho, phi = _rock()
    vp_new, rho_new = O.patchy(np.zeros_like(vp), vp, rho, phi)
    assert np.allclose(vp_new, vp, rtol=1e-14, atol=0)
    assert np.array_equal(rho_new, rho)


def test_co2_with_the_properties_of_brine_changes_nothing():
    vp, rho, phi = _rock(seed=4)
    sw = np.random.default_rng(0).uniform(0, 1, vp.shape)
    same = dict(C, k_co2=C["k_brine"], rho_co2=C["rho_brine"])
    vp_new, rho_new = O.patchy(sw, vp, rho, phi, same)
    assert np.allclose(vp_new, vp, rtol=1e-13, atol=0)
    assert np.allclose(rho_new, rho, rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_full_saturation_matches_textbook_gassmann(seed):
    """Build a brine-saturated rock from a chosen dry frame with the textbook formula, then the
    oracle's fully CO2-saturated wavespeed must equal the textbook substitution with CO2."""
    rng = np.random.default_rng(seed)
    n = 200
    phi = rng.uniform(0.1, 0.35, n)
    rho = rng.uniform(2000.0, 2600.0, n)
    k_dry = rng.uniform(2e9, 20e9, n)
    k1 = _gassmann_textbook(k_dry, C["k_brine"], phi, C["k_min"])
    # vs = vp / sqrt(3): K1 = rho vp^2 (1 - 4/9) and mu = rho vp^2 / 3.
    vp_si = np.sqrt(9.0 * k1 / (5.0 * rho))
    mu = rho * vp_si ** 2 / 3.0
    k2 = _gassmann_textbook(k_dry, C["k_co2"], phi, C["k_min"])
    rho2 = rho - phi * (C["rho_brine"] - C["rho_co2"])
    want = np.sqrt((k2 + 4.0 * mu / 3.0) / rho2) / 1e3
    vp_new, rho_new = O.patchy(np.ones(n), vp_si / 1e3, rho, phi)
    assert np.allclose(vp_new, want, rtol=1e-12, atol=0)
    assert np.allclose(rho_new, rho2, rtol=1e-15, atol=0)


def test_patchy_mixing_is_harmonic_in_the_p_wave_modulus():
    """1 / (rho_new vp_new^2) is affine in the saturation (Hill average of the P-wave moduli of
    the brine and CO2 patches); rho_new is affine too, falling by phi (rho_brine - rho_co2)."""
    vp, rho, phi = _rock(seed=5)
    sws = np.linspace(0.0, 1.0, 5)
    inv_m, dens = [], []
    for s in sws:
        v, r = O.patchy(np.full_like(vp, s), vp, rho, phi)
        inv_m.append(1.0 / (r * (1e3 * v) ** 2))
        dens.append(r)
    inv_m, dens = np.array(inv_m), np.array(dens)
    for k, s in enumerate(sws):
        assert np.allclose(inv_m[k], (1 - s) * inv_m[0] + s * inv_m[-1], rtol=1e-12, atol=0)
        assert np.allclose(dens[k], rho - s * phi * (C["rho_brine"] - C["rho_co2"]), rtol=1e-14,
                           atol=0)
    # Not the arithmetic average: the halfway modulus lies strictly below the mean.
    m_half = 1.0 / inv_m[2]
    assert np.all(m_half < 0.5 * (1.0 / inv_m[0] + 1.0 / inv_m[-1]))


def test_pullback_matches_central_differences():
    vp, rho, phi = _rock(n=300, seed=6)
    rng = np.random.default_rng(1)
    sw = rng.uniform(0.05, 0.95, vp.shape)
    g_vp, g_rho = rng.standard_normal(vp.shape), rng.standard_normal(vp.shape)
    eps = 1e-6
    vp_p, rho_p = O.patchy(sw + eps, vp, rho, phi)
    vp_m, rho_m = O.patchy(sw - eps, vp, rho, phi)
    fd = g_vp * (vp_p - vp_m) / (2 * eps) + g_rho * (rho_p - rho_m) / (2 * eps)
    g = O.patchy_vjp(sw, vp, rho, phi, g_vp, g_rho)
    assert np.allclose(g, fd, rtol=1e-7, atol=1e-9 * np.abs(fd).max())
    g_v_only = O.patchy_vjp(sw, vp, rho, phi, g_vp)
    fd_v = g_vp * (vp_p - vp_m) / (2 * eps)
    assert np.allclose(g_v_only, fd_v, rtol=1e-7, atol=1e-9 * np.abs(fd_v).max())
    # In this soft reservoir rock CO2 lowers the wavespeed at every saturation (in a stiff frame
    # the density drop can win instead).
    assert np.all(O.patchy_vjp(sw, vp, rho, phi, np.ones_like(sw)) < 0)
