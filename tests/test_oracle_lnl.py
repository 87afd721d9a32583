"""Pins of the oracle's likelihood, Eq. (cbclike) of the paper (Sec. III).

* <h,h> on a flat PSD: with d = 0, lnL = -(1/2) <h,h> and for a Newtonian
  amplitude sum_k f_k^(-7/3) is a difference of Hurwitz zeta values,
  delta_f^(-7/3) [zeta(7/3, f_low/df) - zeta(7/3, f_low/df + M)].
* Noise statistics: at the injected parameters d - h is the noise alone, and
  with per-component variance S/(4 df) every bin contributes -Exp(1): lnL has
  mean -N_det M and standard deviation sqrt(N_det M).
* lnL(h = d) = 0 exactly and lnL < 0 elsewhere.
* phi_c enters h as exp(i phi_c), so lnL(phi_c) = C + a cos phi_c + b sin phi_c.
* <h,h> does not depend on t_c or phi_c.
"""
import math

import numpy as np
import pytest
from scipy.special import zeta

import oracle
import synth

MSUN_S = 1.3271244e20 / 299792458.0 ** 3
MPC_S = 3.0856775814913673e22 / 299792458.0


def _amp0(mc, dl):
    return math.sqrt(5 / 24) * math.pi ** (-2 / 3) * (mc * MSUN_S) ** (5 / 6) / (dl * MPC_S)


@pytest.mark.parametrize("f_low,df,m", [(20.0, 0.25, 4017), (20.0, 1 / 128, 20001), (10.0, 1.0, 17), (35.5, 0.5, 1)])
def test_flat_psd_inner_product_is_hurwitz_zeta(f_low, df, m):
    s0 = 2.5e-47
    th = np.array([[30.0, 0.8, 500.0, 1.1, 0.03]])
    got = oracle.lnl(f_low, df, m, np.eye(3)[None], np.zeros((1, 3)), np.zeros((1, m), complex),
                     np.full((1, m), s0), th)[0]
    a = f_low / df
    sum_f = df ** (-7 / 3) * (zeta(7 / 3, a) - zeta(7 / 3, a + m))
    hh = 4 * df * _amp0(30.0, 500.0) ** 2 / s0 * sum_f
    assert got == pytest.approx(-0.5 * hh, rel=1e-12)


def test_config1_grid_hurwitz_value():
    """sum_k f_k^(-7/3) on the 4017-bin grid (20..1024 Hz, df = 1/4)."""
    a = 20.0 / 0.25
    sum_f = 0.25 ** (-7 / 3) * (zeta(7 / 3, a) - zeta(7 / 3, a + 4017))
    f = 20.0 + 0.25 * np.arange(4017)
    assert math.fsum(f ** (-7 / 3)) == pytest.approx(0.05543260038357918, rel=1e-12)
    assert sum_f == pytest.approx(math.fsum(f ** (-7 / 3)), rel=1e-13)


def test_projected_inner_product_closed_form():
    """Three detectors on a flat PSD: <h_d,h_d> = 4 df A0^2 |F+ (1+c^2)/2 - i Fx c|^2 sum f^-7/3 / S0."""
    w = synth.small_event(1, 3, 300, 1)
    s0, m, df, f_low = 1e-46, 300, 0.5, 30.0
    th = np.array([[27.0, 0.9, 640.0, 0.2, 0.01, 1.9, 0.5, 2.2, 0.6]])
    got = oracle.lnl(f_low, df, m, w.tensors, w.vertices, np.zeros((3, m), complex), np.full((3, m), s0), th)[0]
    sum_f = math.fsum((f_low + df * np.arange(m)) ** (-7 / 3))
    c = math.cos(0.6)
    hh = 0.0
    for d in range(3):
        fp, fx = oracle.antenna(w.tensors[d], 1.9, 0.5, 2.2)
        hh += 4 * df * _amp0(27.0, 640.0) ** 2 * abs(fp * (1 + c * c) / 2 - 1j * fx * c) ** 2 * sum_f / s0
    assert got == pytest.approx(-0.5 * hh, rel=1e-12)


@pytest.mark.parametrize("which", ["1det", "3det"])
def test_noise_statistics_at_injection(which):
    if which == "1det":
        w = synth.bbh_1det_4s(4)
    else:
        w = synth.small_event(2, 3, 30000, 2)
    g = w.grid
    data = oracle.workload_data(w)
    val = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj[None])[0]
    n = w.n_det * g.n_bins
    z = (val + n) / math.sqrt(n)
    assert abs(z) < 5.0
    # the same number from the noise alone, without the waveform
    direct = -2 * g.delta_f * math.fsum((np.abs(w.noise) ** 2 / w.psd).ravel())
    assert val == pytest.approx(direct, rel=1e-12)


def test_noise_mean_over_realisations():
    vals = []
    for i in range(40):
        w = synth.small_event(10 + i, 2, 500, 1)
        data = oracle.workload_data(w)
        g = w.grid
        vals.append(oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd,
                               w.theta_inj[None])[0])
    n = 2 * 500
    mean = np.mean(vals)
    assert abs(mean + n) < 5 * math.sqrt(n / 40)
    assert np.std(vals) == pytest.approx(math.sqrt(n), rel=0.35)


def test_zero_at_noise_free_truth_and_negative_elsewhere():
    w = synth.small_event(3, 3, 1000, 16)
    g = w.grid
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    th = np.vstack([w.theta_inj, w.theta])
    vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, h, w.psd, th)
    assert vals[0] == 0.0
    assert (vals[1:] < 0).all()


def test_phic_dependence_is_a_sinusoid():
    w = synth.small_event(4, 3, 2000, 1)
    g = w.grid
    data = oracle.workload_data(w)
    base = w.theta_inj.copy()
    phis = np.linspace(0.0, 2 * math.pi, 9)[:-1]
    th = np.repeat(base[None], len(phis), 0)
    th[:, 3] = phis
    vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, th)
    a = np.stack([np.ones_like(phis), np.cos(phis), np.sin(phis)], 1)
    coef = np.linalg.solve(a[:3], vals[:3])
    np.testing.assert_allclose(a @ coef, vals, rtol=1e-11, atol=1e-9 * np.abs(vals).max())


def test_signal_power_independent_of_tc_and_phic():
    w = synth.small_event(5, 3, 800, 1)
    g = w.grid
    zero = np.zeros((3, g.n_bins), complex)
    th = np.repeat(w.theta_inj[None], 4, 0)
    th[1, 4] += 0.077
    th[2, 3] += 2.0
    th[3, 4] -= 0.05
    th[3, 3] += 0.5
    vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, zero, w.psd, th)
    np.testing.assert_allclose(vals, vals[0], rtol=1e-13)


def test_domain_rules():
    w = synth.small_event(6, 1, 50, 1)
    g = w.grid
    data = oracle.workload_data(w)
    good = w.theta_inj
    rows = np.repeat(good[None], 7, 0)
    rows[1, 0] = -3.0           # Mc <= 0
    rows[2, 1] = 1.5            # q > 1
    rows[3, 1] = 0.0            # q = 0
    rows[4, 2] = 0.0            # d_L = 0
    rows[5, 6] = np.nan         # NaN anywhere
    rows[6, 4] = np.inf         # non-finite
    vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, rows)
    assert np.isfinite(vals[0])
    assert (vals[1:5] == -np.inf).all()
    assert np.isnan(vals[5]) and np.isnan(vals[6])


def test_empty_batch_and_single_bin():
    w = synth.small_event(7, 2, 1, 3)
    g = w.grid
    data = oracle.workload_data(w)
    assert oracle.lnl(g.f_low, g.delta_f, 1, w.tensors, w.vertices, data, w.psd, np.zeros((0, 9))).shape == (0,)
    v = oracle.lnl(g.f_low, g.delta_f, 1, w.tensors, w.vertices, data, w.psd, w.theta)
    h = oracle.waveform(g.f_low, g.delta_f, 1, w.tensors, w.vertices, w.theta)
    brute = [-2 * g.delta_f * sum(abs(data[d, 0] - h[s, d, 0]) ** 2 / w.psd[d, 0] for d in range(2)) for s in range(3)]
    np.testing.assert_allclose(v, brute, rtol=1e-14)


def test_thread_count_does_not_change_results():
    w = synth.small_event(8, 3, 3000, 12)
    g = w.grid
    data = oracle.workload_data(w)
    a = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta, n_threads=1)
    b = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta, n_threads=4)
    np.testing.assert_array_equal(a, b)


def test_regression_fixture_1det_4s():
    """The stored oracle values (tests/golden/bbh_1det_4s_lnl.txt) still hold."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "bbh_1det_4s_lnl.txt")
    ref = np.loadtxt(path)
    w = synth.bbh_1det_4s(32)
    g = w.grid
    vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, oracle.workload_data(w), w.psd, w.theta)
    np.testing.assert_allclose(vals, ref, rtol=1e-14)
