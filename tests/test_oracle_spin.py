"""Pins of the oracle's aligned-spin phase terms (the spinning TaylorF2 the
paper's chi_eff study of Sec. III implies; the coefficients come from the
literature cited in the oracle).

* Every spin-orbit term (1.5, 2.5, 3 with its tail, 3.5PN) and the 2PN
  spin-spin S1 S2 term equal the phase derived independently from the spin
  terms of the binding energy and flux by the stationary-phase relation
  (tests/pn_derivation.py: sympy series inversion), for several mass ratios.
* The energy's spin-orbit terms reduce, for a test mass, to the exact
  expansion of the Kerr circular-orbit energy; the flux's reduce to the
  black-hole-perturbation flux; the 2PN self-spin term of the phase equals,
  per body, the test-mass Kerr value derived from those two.
* Zero spins give the non-spinning waveform and likelihood bit for bit;
  equal masses make the two spins interchangeable; |chi| > 1 is out of the
  domain (-inf), a non-finite spin gives NaN.
"""
import math

import numpy as np
import pytest

import oracle
import pn_derivation as pnd
import synth


def _terms(q, chi1, chi2):
    eta = q / (1 + q) ** 2
    delta = (1 - q) / (1 + q)
    return oracle.pn_spin_terms(eta, delta, chi1, chi2)


@pytest.mark.parametrize("q", [1.0, 0.8, 0.5, 0.25, 0.1])
def test_spin_orbit_terms_match_energy_flux_derivation(q):
    x1 = 1.0 / (1.0 + q)
    for which in (1, 2):
        chi = (1.0, 0.0) if which == 1 else (0.0, 1.0)
        phi, phil = _terms(q, *chi)
        for k in (3, 6, 7):
            assert phi[k] == pytest.approx(pnd.spin_linear_term(k, x1, which), rel=1e-12, abs=1e-12), (k, which)
        assert phi[5] == pytest.approx(pnd.spin_linear_term(5, x1, which), rel=1e-12)
        assert phil[5] == pytest.approx(3.0 * phi[5], rel=1e-15)
        assert phil[[0, 1, 2, 3, 4, 6, 7]].tolist() == [0.0] * 7
        assert phi[0] == phi[1] == phi[2] == 0.0


@pytest.mark.parametrize("q", [1.0, 0.7, 0.3])
def test_spin_spin_terms(q):
    x1, x2 = 1.0 / (1.0 + q), q / (1.0 + q)
    both = _terms(q, 1.0, 1.0)[0][4]
    one = _terms(q, 1.0, 0.0)[0][4]
    two = _terms(q, 0.0, 1.0)[0][4]
    # S1 S2 term against the derivation from the energy and flux
    assert both - one - two == pytest.approx(pnd.spin_spin_term(x1), rel=1e-12)
    # self-spin terms: x_i^2 times the test-mass Kerr value, for each body
    self_coef = pnd.test_mass_self_spin_term()
    assert self_coef == pytest.approx(-405.0 / 8.0, rel=1e-15)
    assert one == pytest.approx(self_coef * x1 ** 2, rel=1e-12)
    assert two == pytest.approx(self_coef * x2 ** 2, rel=1e-12)
    # quadratic in each spin
    assert _terms(q, 0.5, 0.0)[0][4] == pytest.approx(0.25 * one, rel=1e-12)


def test_energy_and_flux_reduce_to_the_test_mass_kerr_values():
    import sympy as sp
    e, f = pnd._spin_energy_flux()
    kerr_e = pnd.kerr_energy_series(8)
    kerr_f = pnd.kerr_flux_spin_terms()
    a = pnd.kerr_a
    for k in (3, 5, 7):      # spin-orbit energy, test mass: x1 -> 1, chi1 = a
        lim = sp.expand(e[k]).subs({pnd.x1: 1, pnd.chi1: a, pnd.chi2: 0})
        assert sp.simplify(lim - kerr_e[k]) == 0, k
    nonspin = pnd._flux_coefficients()
    for k in (3, 5, 6):      # spin-orbit flux
        lim = sp.expand(f[k] - sp.sympify(nonspin[k]).subs(pnd.eta, pnd.x1 * (1 - pnd.x1)))
        lim = lim.subs({pnd.x1: 1, pnd.chi1: a, pnd.chi2: 0})
        assert sp.simplify(lim - kerr_f[k]) == 0, k
    # the Kerr energy without spin is the non-spinning test-mass energy
    ns = pnd._energy_coefficients()
    for k in (2, 4, 6):
        assert sp.simplify(kerr_e[k].subs(a, 0) - sp.sympify(ns[k]).subs(pnd.eta, 0)) == 0


def test_zero_spins_are_the_non_spinning_template():
    w = synth.bbh_3det_128s(6)
    g = w.grid
    n = 3000
    data = w.noise[:, :n] + oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, w.theta_inj[None])[0]
    th11 = np.hstack([w.theta, np.zeros((6, 2))])
    a = oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, w.theta)
    b = oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, th11)
    assert np.array_equal(a, b)
    la = oracle.lnl(g.f_low, g.delta_f, n, w.tensors, w.vertices, data, w.psd[:, :n], w.theta)
    lb = oracle.lnl(g.f_low, g.delta_f, n, w.tensors, w.vertices, data, w.psd[:, :n], th11)
    assert np.array_equal(la, lb)
    th5 = w.theta[:, :5]
    th7 = np.hstack([th5, np.zeros((6, 2))])
    assert np.array_equal(oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, th5),
                          oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, th7))


def test_spins_change_the_phase_only():
    w = synth.bbh_3det_128s(2)
    g = w.grid
    n = 2000
    th = np.hstack([w.theta, [[0.6, -0.3], [0.0, 0.0]]])
    h = oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, th)
    h0 = oracle.waveform(g.f_low, g.delta_f, n, w.tensors, w.vertices, w.theta)
    np.testing.assert_allclose(np.abs(h[0]), np.abs(h0[0]), rtol=1e-12)
    assert np.abs(np.angle(h[0] / h0[0])).max() > 0.1
    # the phase difference is the spin part of the PN series
    f = g.f_low + np.arange(n) * g.delta_f
    q = th[0, 1]
    eta = q / (1 + q) ** 2
    mtot = th[0, 0] * eta ** -0.6 * 1.3271244e20 / 299792458.0 ** 3
    v = np.cbrt(math.pi * mtot * f)
    dphi, dphil = _terms(q, 0.6, -0.3)
    dpsi = 3.0 / (128.0 * eta * v ** 5) * sum((dphi[k] + dphil[k] * np.log(v)) * v ** k for k in range(8))
    got = np.angle(h[0] / h0[0])          # h ~ e^{-i Psi}
    np.testing.assert_allclose(np.angle(np.exp(-1j * dpsi) / np.exp(1j * got)), 0.0, atol=1e-9)


def test_equal_masses_make_the_spins_interchangeable():
    a = _terms(1.0, 0.7, -0.2)
    b = _terms(1.0, -0.2, 0.7)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-14)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-14)


def test_spin_domain():
    w = synth.bbh_3det_128s(4)
    g = w.grid
    n = 500
    th = np.hstack([w.theta, [[0.2, 0.3], [1.01, 0.0], [0.0, -1.5], [np.nan, 0.0]]])
    data = w.noise[:, :n]
    out = oracle.lnl(g.f_low, g.delta_f, n, w.tensors, w.vertices, data, w.psd[:, :n], th)
    assert np.isfinite(out[0]) and out[1] == -np.inf and out[2] == -np.inf and np.isnan(out[3])
    edge = th[:1].copy()
    edge[0, 9:] = [1.0, -1.0]
    assert np.isfinite(oracle.lnl(g.f_low, g.delta_f, n, w.tensors, w.vertices, data, w.psd[:, :n], edge)[0])
