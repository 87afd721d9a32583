"""Pins of the relative-binning oracle (Zackay, Dai & Venumadhav 2018, named
in Secs. I and V of arXiv:1904.02863 as the other route to long signals).

* The edge rule: the phase bound takes its closed-form values at the band
  ends (typed independently), the edges are those of a brute-force walk over
  a small grid, and no bin spans more than eps of the bound.
* At the fiducial point the ratio is exactly 1 and the estimate equals the
  full likelihood of Eq. (cbclike) (the exact oracle).
* With an edge at every grid bin the linear model is exact for any template,
  so the estimate equals the full likelihood for rows far from the fiducial;
  this needs every summary term (A0, A1, B0, B1, B2) with its sign and
  conjugation right.
* For any ratio that is linear inside every bin (random complex values at
  the edges, so |r| varies and the B1 and B2 terms matter), the estimate
  equals -<d - h, d - h>/2 with h = h0 r formed on every grid bin.
* Rows that differ from the fiducial only in d_L, phi_c, psi and iota have a
  ratio that is constant in frequency: exact with coarse bins.
* Summary totals: sum_b B0 = <h0, h0>, sum_b A0 = sum w d conj(h0) and
  sum_b (B1 + fm B0) = sum w |h0|^2 f, summed independently over the grid.
* Near the fiducial the error falls as eps shrinks (the method's claim), to
  below 0.01 at the ~10^3 bins of a neutron-star signal from 30 Hz (Sec. V).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import relbin as rb


@pytest.fixture(scope="module")
def event():
    w = synth.relbin_bns(30.0, 64.0, 3, 24)
    g = w.grid
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    snr = math.sqrt(float(np.sum(4.0 * g.delta_f * np.abs(h) ** 2 / w.psd)))
    w = synth.scale_distance(w, snr / 30.0)
    h *= 30.0 / snr
    return w, w.noise + h


def _exact(w, data, theta, add_norm=False):
    g = w.grid
    return oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, theta, add_norm=add_norm)


def test_phase_bound_closed_form():
    fmin, fmax, chi = 20.0, 1024.0, 1.3
    r = fmin / fmax
    lo = 2 * math.pi * chi * (-1.0 - 1.0 + r + r ** (5 / 3) + r ** (7 / 3))
    hi = 2 * math.pi * chi * (-(1 / r) ** (-5 / 3) - (1 / r) ** (-2 / 3) + 3.0)
    got = rb.phase_bound(np.array([fmin, fmax]), fmin, fmax, chi)
    np.testing.assert_allclose(got, [lo, hi], rtol=1e-14)
    f = np.linspace(fmin, fmax, 1000)
    assert np.all(np.diff(rb.phase_bound(f, fmin, fmax, chi)) > 0)


@pytest.mark.parametrize("f_low,df,n,chi,eps", [(20.0, 0.25, 3000, 1.0, 0.5), (30.0, 1 / 16, 20000, 1.0, 0.1),
                                                (10.0, 1.0, 500, 2.0, 0.05)])
def test_edges_brute_force(f_low, df, n, chi, eps):
    e = rb.edges(f_low, df, n, chi, eps)
    f = f_low + np.arange(n) * df
    fmin, fmax = f[0], f[-1]

    def bound(x):   # the same rule written term by term for one frequency
        return 2 * math.pi * chi * (-(x / fmin) ** (-5 / 3) - (x / fmin) ** (-2 / 3) + x / fmax
                                    + (x / fmax) ** (5 / 3) + (x / fmax) ** (7 / 3))
    base = bound(fmin)
    want, level = [0], 0
    for k in range(1, n):
        lv = math.floor((bound(f[k]) - base) / eps)
        if lv > level:
            want.append(k)
            level = lv
    if want[-1] != n - 1:
        want.append(n - 1)
    assert e.tolist() == want
    psi = rb.phase_bound(f, fmin, fmax, chi)
    for b in range(len(e) - 1):
        inner = psi[e[b]:e[b + 1]]
        assert inner[-1] - inner[0] < eps
    # at most one edge per eps step of the bound, plus the closing edge
    assert len(e) - 1 <= math.floor((psi[-1] - psi[0]) / eps) + 1


def test_fiducial_point_is_exact(event):
    w, data = event
    g = w.grid
    e = rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, 0.5)
    for add_norm in (False, True):
        s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e,
                       add_norm=add_norm)
        got = rb.lnl(s, w.tensors, w.vertices, w.theta_inj)[0]
        want = _exact(w, data, w.theta_inj[None], add_norm)[0]
        assert got == pytest.approx(want, rel=1e-12)
        # the signal part alone (the data term removed on both sides)
        assert got + 0.5 * s["dd"] + s["norm"] == pytest.approx(want + 0.5 * s["dd"] + s["norm"], abs=1e-7)


def test_every_bin_edges_are_exact():
    w = synth.relbin_bns(40.0, 4.0, 2, 6, index=8)
    g = w.grid
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    data = w.noise + 40.0 * h
    far = synth.near_fiducial(w.theta_inj, 6, np.random.default_rng(3), scale=300.0)
    far[:, 0] = w.theta_inj[0] * (1.0 + np.linspace(-0.02, 0.02, 6))
    e = np.arange(g.n_bins, dtype=np.int64)
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    got = rb.lnl(s, w.tensors, w.vertices, far)
    want = _exact(w, data, far)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    np.testing.assert_allclose(got + 0.5 * s["dd"], want + 0.5 * s["dd"], atol=1e-8 * np.abs(want).max())


def test_linear_ratio_is_exact(event):
    w, data = event
    g = w.grid
    e = rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, 0.5)
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    h0 = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    f = g.f_low + np.arange(g.n_bins) * g.delta_f
    rng = np.random.default_rng(4)
    for _ in range(3):
        r = rng.uniform(0.5, 1.5, (w.n_det, len(e))) * np.exp(1j * rng.uniform(-3, 3, (w.n_det, len(e))))
        h = np.empty_like(h0)
        for d in range(w.n_det):
            h[d] = h0[d] * (np.interp(f, s["fe"], r[d].real) + 1j * np.interp(f, s["fe"], r[d].imag))
        want = -0.5 * math.fsum((4.0 * g.delta_f * np.abs(data - h) ** 2 / w.psd).ravel().tolist())
        got = rb.lnl_from_ratio(s, r[None])[0]
        assert got == pytest.approx(want, rel=1e-12)
        assert got + 0.5 * s["dd"] == pytest.approx(want + 0.5 * s["dd"], abs=1e-8 * abs(want + 0.5 * s["dd"]) + 1e-8)


def test_constant_ratio_is_exact(event):
    w, data = event
    g = w.grid
    e = rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, 0.5)
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    th = np.repeat(w.theta_inj[None], 4, axis=0)
    th[:, 2] *= [0.7, 1.0, 1.3, 2.0]
    th[:, 3] += [0.0, 0.9, -2.0, 3.0]
    th[:, 7] += [0.3, 0.0, -0.2, 1.0]
    th[:, 8] += [0.0, 0.4, -0.3, 0.8]
    got = rb.lnl(s, w.tensors, w.vertices, th)
    want = _exact(w, data, th)
    np.testing.assert_allclose(got + 0.5 * s["dd"], want + 0.5 * s["dd"], atol=1e-8)


def test_summary_totals(event):
    w, data = event
    g = w.grid
    e = rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, 0.1)
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    h0 = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    f = g.f_low + np.arange(g.n_bins) * g.delta_f
    wgt = 4.0 * g.delta_f / w.psd
    fm = 0.5 * (s["fe"][:-1] + s["fe"][1:])
    for d in range(w.n_det):
        hh = math.fsum((wgt[d] * np.abs(h0[d]) ** 2).tolist())
        assert s["B0"][d].sum() == pytest.approx(hh, rel=1e-12)
        x = wgt[d] * data[d] * np.conj(h0[d])
        assert s["A0"][d].sum() == pytest.approx(math.fsum(x.real.tolist()) + 1j * math.fsum(x.imag.tolist()),
                                                 rel=1e-11)
        hf = math.fsum((wgt[d] * np.abs(h0[d]) ** 2 * f).tolist())
        assert (s["B1"][d] + fm * s["B0"][d]).sum() == pytest.approx(hf, rel=1e-12)
    assert s["dd"] == pytest.approx(math.fsum((wgt * np.abs(data) ** 2).ravel().tolist()), rel=1e-12)


def test_error_falls_with_eps(event):
    w, data = event
    g = w.grid
    want = _exact(w, data, w.theta)
    errs, bins = [], []
    for eps in (0.5, 0.1, 0.03):
        e = rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, eps)
        s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
        errs.append(np.abs(rb.lnl(s, w.tensors, w.vertices, w.theta) - want).max())
        bins.append(len(e) - 1)
    assert errs[0] > errs[1] > errs[2]
    assert 900 < bins[2] < 1200 and errs[2] < 0.01


def test_domain_rules(event):
    w, data = event
    g = w.grid
    e = rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, 0.5)
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    th = np.repeat(w.theta_inj[None], 3, axis=0)
    th[0, 4] = np.nan
    th[1, 1] = 1.2
    out = rb.lnl(s, w.tensors, w.vertices, th)
    assert np.isnan(out[0]) and out[1] == -np.inf and np.isfinite(out[2])
    with pytest.raises(ValueError):
        rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e[1:])
