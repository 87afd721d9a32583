"""Pins of the oracle's two optional terms.

* Template end at the innermost stable circular orbit: the cut-off frequency is
  computed here from Kepler's law at r = 6 G M / c^2 (not from the oracle's
  closed form), and the in-band power of an optimally oriented source with a
  flat PSD is a difference of Hurwitz zeta values, sum_k (f_low + k df)^-7/3.
* The logarithm of the prefactor of Eq. (cbclike), -sum ln(2 pi S): closed
  forms for a flat and for a geometric PSD.
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle
import synth

GM_SUN = 1.3271244e20          # m^3 s^-2 (IAU 2015 B3)
C_SI = 299792458.0


def _kepler_isco_frequency(mc, q):
    """Gravitational-wave frequency (twice the orbital) of a circular orbit at
    r = 6 G M / c^2 around total mass M, from Kepler's third law."""
    eta = q / (1.0 + q) ** 2
    m_total = mc / eta ** 0.6                         # solar masses
    gm = GM_SUN * m_total
    r = 6.0 * gm / C_SI ** 2
    omega_orbit = math.sqrt(gm / r ** 3)
    return omega_orbit / math.pi


def _hurwitz_sum(a, k0, k1, df):
    """sum_{k=k0}^{k1-1} (df (a + k))^-7/3 via Hurwitz zeta."""
    return df ** (-7.0 / 3.0) * (special.zeta(7.0 / 3.0, a + k0) - special.zeta(7.0 / 3.0, a + k1))


@pytest.mark.parametrize("mc,q", [(30.0, 0.8), (26.0, 0.55), (34.0, 0.97)])
def test_isco_cut_keeps_power_below_the_orbit(mc, q):
    f_low, df, m = 20.0, 0.25, 4017
    f_isco = _kepler_isco_frequency(mc, q)
    k_last = math.floor((f_isco - f_low) / df)
    assert abs(f_low + k_last * df - f_isco) > 1e-6 and abs(f_low + (k_last + 1) * df - f_isco) > 1e-6
    th = np.array([[mc, q, 500.0, 0.3, 0.01]])
    tensor, vertex = np.eye(3)[None], np.zeros((1, 3))
    zero = np.zeros((1, m), complex)
    s0 = 1e-46
    full = oracle.lnl(f_low, df, m, tensor, vertex, zero, np.full((1, m), s0), th)[0]
    cut = oracle.lnl(f_low, df, m, tensor, vertex, zero, np.full((1, m), s0), th, isco=True)[0]
    a = f_low / df
    want = _hurwitz_sum(a, 0, k_last + 1, df) / _hurwitz_sum(a, 0, m, df)
    assert cut / full == pytest.approx(want, rel=1e-11)
    assert cut > full          # less template power, smaller |lnL| at zero data


@pytest.mark.parametrize("n_det", [0, 3])
def test_isco_waveform_is_the_full_waveform_then_zero(n_det):
    f_low, df, m = 20.0, 0.25, 801
    rng = np.random.default_rng(4)
    th = np.column_stack([rng.uniform(25, 35, 6), rng.uniform(0.5, 1, 6), rng.uniform(400, 1000, 6),
                          rng.uniform(0, 2 * np.pi, 6), rng.uniform(-0.1, 0.1, 6), rng.uniform(0, 2 * np.pi, 6),
                          np.arcsin(rng.uniform(-1, 1, 6)), rng.uniform(0, np.pi, 6),
                          np.arccos(rng.uniform(-1, 1, 6))])
    if n_det:
        tensors, vertices = synth.stack_detectors(synth.network(synth.seeds(5)["detectors"], n_det))
    else:
        tensors = vertices = None
    full = oracle.waveform(f_low, df, m, tensors, vertices, th)
    cut = oracle.waveform(f_low, df, m, tensors, vertices, th, isco=True)
    for s in range(th.shape[0]):
        k_last = math.floor((_kepler_isco_frequency(th[s, 0], th[s, 1]) - f_low) / df)
        assert 0 < k_last < m - 1
        np.testing.assert_array_equal(cut[s, :, :k_last + 1], full[s, :, :k_last + 1])
        assert np.all(cut[s, :, k_last + 1:] == 0)


def test_norm_flat_psd():
    f_low, df, m, s0 = 20.0, 0.25, 1001, 3.7e-47
    w_t, w_v = synth.stack_detectors(synth.network(synth.seeds(6)["detectors"], 2))
    rng = np.random.default_rng(1)
    data = rng.normal(size=(2, m)) * 1e-23 + 1j * rng.normal(size=(2, m)) * 1e-23
    th = np.array([[30.0, 0.8, 500.0, 0.1, 0.0, 1.0, 0.2, 0.3, 0.4], [28.0, 0.6, 700.0, 2.0, 0.05, 4.0, -0.5, 1.0, 2.0]])
    psd = np.full((2, m), s0)
    plain = oracle.lnl(f_low, df, m, w_t, w_v, data, psd, th)
    normed = oracle.lnl(f_low, df, m, w_t, w_v, data, psd, th, add_norm=True)
    want = -2 * m * math.log(2 * math.pi * s0)
    np.testing.assert_allclose(normed - plain, want, rtol=1e-12)


def test_norm_geometric_psd():
    # S_k = c r^k: sum_k ln(2 pi c r^k) = M ln(2 pi c) + ln(r) M (M - 1) / 2
    f_low, df, m, c, r = 20.0, 0.5, 777, 2e-46, 1.0007
    psd = (c * r ** np.arange(m))[None]
    th = np.array([[30.0, 0.8, 500.0, 0.1, 0.0]])
    zero = np.zeros((1, m), complex)
    plain = oracle.lnl(f_low, df, m, np.eye(3)[None], np.zeros((1, 3)), zero, psd, th)[0]
    normed = oracle.lnl(f_low, df, m, np.eye(3)[None], np.zeros((1, 3)), zero, psd, th, add_norm=True)[0]
    want = -(m * math.log(2 * math.pi * c) + math.log(r) * m * (m - 1) / 2)
    assert normed - plain == pytest.approx(want, rel=1e-12)


def test_norm_keeps_domain_rules():
    m = 101
    th = np.array([[30.0, 0.8, 500.0, 0.1, 0.0], [np.nan, 0.8, 500.0, 0.1, 0.0], [-1.0, 0.8, 500.0, 0.1, 0.0]])
    v = oracle.lnl(20.0, 0.25, m, np.eye(3)[None], np.zeros((1, 3)), np.zeros((1, m), complex),
                   np.full((1, m), 1e-46), th, add_norm=True, isco=True)
    assert np.isfinite(v[0]) and np.isnan(v[1]) and v[2] == -np.inf
