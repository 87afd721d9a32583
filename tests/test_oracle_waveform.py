"""Pins of the oracle's waveform amplitude, polarisations and time shifts.

* Amplitude: the stationary-phase amplitude of the Newtonian quadrupole chirp,
  (1/2) A_t(f) / sqrt(df/dt), with the time-domain face-on amplitude
  A_t = 4 Mc^(5/3) (pi f)^(2/3) / D and chirp rate
  df/dt = (96/5) pi^(8/3) Mc^(5/3) f^(11/3) (textbook quadrupole formulae),
  a different route from the oracle's closed form.
* The f^(-7/6) slope and the 1/d_L scaling.
* h_cross / h_plus = -i 2 cos(iota) / (1 + cos^2 iota).
* A shift of t_c by tau multiplies h by exp(-2 pi i f tau), the sign of the
  time translation in Sec. III of the paper.
"""
import math

import numpy as np
import pytest

import oracle

MSUN_S = 1.3271244e20 / 299792458.0 ** 3
MPC_S = 3.0856775814913673e22 / 299792458.0


def _h(theta, f_low=20.0, df=0.25, n=200, tensors=None, vertices=None):
    return oracle.waveform(f_low, df, n, tensors, vertices, np.atleast_2d(theta))


@pytest.mark.parametrize("mc,dl", [(30.0, 500.0), (1.2, 40.0), (8.0, 123.0)])
def test_amplitude_is_stationary_phase_quadrupole(mc, dl):
    th = [mc, 0.7, dl, 0.0, 0.0]
    f = 20.0 + 0.25 * np.arange(200)
    got = np.abs(_h(th)[0, 0])
    mcs, d = mc * MSUN_S, dl * MPC_S
    a_t = 4.0 * mcs ** (5 / 3) * (math.pi * f) ** (2 / 3) / d
    fdot = 96.0 / 5.0 * math.pi ** (8 / 3) * mcs ** (5 / 3) * f ** (11 / 3)
    np.testing.assert_allclose(got, 0.5 * a_t / np.sqrt(fdot), rtol=1e-13)


def test_amplitude_slope_and_distance():
    th = np.array([30.0, 0.8, 500.0, 1.0, 0.02])
    f = 20.0 + 0.25 * np.arange(200)
    a = np.abs(_h(th)[0, 0])
    slope = np.diff(np.log(a)) / np.diff(np.log(f))
    np.testing.assert_allclose(slope, -7 / 6, rtol=1e-9)
    th2 = th.copy()
    th2[2] *= 3.7
    np.testing.assert_allclose(np.abs(_h(th2)[0, 0]) * 3.7, a, rtol=1e-14)


@pytest.mark.parametrize("iota", [0.0, 0.3, 1.1, math.pi / 2 - 0.01, 2.5])
def test_polarisation_ratio(iota):
    th = [30.0, 0.8, 500.0, 0.4, 0.01, 1.0, 0.2, 0.3, iota]
    hp, hx = _h(th)[0]
    c = math.cos(iota)
    np.testing.assert_allclose(hx, hp * (-1j) * 2 * c / (1 + c * c), rtol=1e-13, atol=1e-40)


@pytest.mark.parametrize("tau", [0.003, -0.07, 0.25])
def test_tc_shift_is_exp_minus_2_pi_i_f_tau(tau):
    rng = np.random.default_rng(5)
    tensors = rng.standard_normal((2, 3, 3))
    tensors = tensors + tensors.transpose(0, 2, 1)
    vertices = rng.standard_normal((2, 3)) * 6e6
    th = np.array([28.0, 0.6, 700.0, 2.0, -0.05, 0.7, -0.4, 1.3, 0.8])
    th2 = th.copy()
    th2[4] += tau
    f = 20.0 + 0.25 * np.arange(200)
    a = _h(th, tensors=tensors, vertices=vertices)[0]
    b = _h(th2, tensors=tensors, vertices=vertices)[0]
    np.testing.assert_allclose(b, a * np.exp(-2j * math.pi * f * tau), rtol=1e-11)


def test_phic_enters_as_overall_phase():
    th = np.array([28.0, 0.6, 700.0, 2.0, -0.05, 0.7, -0.4, 1.3, 0.8])
    th2 = th.copy()
    th2[3] += 0.9
    a = _h(th)[0]
    b = _h(th2)[0]
    np.testing.assert_allclose(b, a * np.exp(0.9j), rtol=1e-12)


def test_detector_delay_between_sites():
    """Response of a detector displaced by r relative to one at the geocentre
    (same tensor) is delayed by -n.r/c: h_r = h_0 exp(2 pi i f n.r / c)."""
    tensor = np.diag([0.5, -0.5, 0.0])
    r = np.array([1.2e6, -3.0e6, 5.5e6])
    ra, dec = 2.1, -0.6
    th = np.array([28.0, 0.6, 700.0, 2.0, -0.05, ra, dec, 1.3, 0.8])
    h = _h(th, tensors=np.stack([tensor, tensor]), vertices=np.stack([np.zeros(3), r]))[0]
    n = np.array([math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)])
    f = 20.0 + 0.25 * np.arange(200)
    np.testing.assert_allclose(h[1], h[0] * np.exp(2j * math.pi * f * (n @ r) / 299792458.0), rtol=1e-11)


def test_five_parameter_rows_are_optimally_oriented():
    """5 columns == 9 columns with F+ = 1, Fx = 0, no delay, iota = 0: the plus
    polarisation itself."""
    th5 = np.array([30.0, 0.8, 500.0, 0.4, 0.01])
    th9 = np.concatenate([th5, [1.0, 0.2, 0.3, 0.0]])
    h5 = _h(th5, tensors=np.eye(3)[None], vertices=np.ones((1, 3)))[0, 0]
    hp = _h(th9)[0, 0]
    np.testing.assert_array_equal(h5, hp)


def test_out_of_domain_rows():
    th = np.array([[30.0, 0.8, 500.0, 0.4, 0.01], [-1.0, 0.8, 500.0, 0.4, 0.01], [30.0, np.nan, 500.0, 0.4, 0.01]])
    h = _h(th, n=4)
    assert np.isfinite(h[0]).all()
    assert np.isnan(h[1]).all() and np.isnan(h[2]).all()
