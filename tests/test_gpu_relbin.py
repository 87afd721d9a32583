"""Relative binning on the GPU against the oracle (parity: the same estimate,
element by element on the same seeded inputs).

* Summary data A0, A1, B0, B1, B2 of every detector and bin, <d,d> and
  sum ln 2 pi S: within 1e-10 of the scale of each sum (the sum of the
  magnitudes of its terms, so that bins where a sum cancels are judged
  fairly).
* lnL of near-fiducial rows (30 Hz / 64 s, 3 detectors, 129,153 bins; 1,000
  rows, a ragged last group) for 63 and 1,033 bins: 1e-10 relative, and the
  signal part lnL + <d,d>/2 within 1e-8 absolute.
* An edge at every grid bin (2 detectors, 4 s, 8,001 bins): the estimate
  equals the full likelihood, checked against the exact oracle and against
  gw_lnl_batch.
* At the fiducial point the estimate equals gw_lnl_batch.
* Domain rows, GW_FLAG_ADD_NORM, five-parameter rows, no rows, argument errors.
* The benchmark's workload (15 Hz / 512 s, 3 detectors, 1,040,897 bins,
  1,039 bins of relative binning, 65,536 rows in the benchmark's launch):
  sampled rows against the oracle, 1e-10 relative.
* The longest band (5 Hz / 8192 s, 16,736,257 bins): totals, B0 of every bin
  and sampled rows against the oracle.
* Mixed precision (FP32 hardware phasor of the ratio): within 1e-3 of the
  FP64 pass at SNR 30 and 100.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import relbin as rb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def _event(f_low, duration, n_det, n_samples, snr=30.0, index=7):
    w = synth.relbin_bns(f_low, duration, n_det, n_samples, index=index)
    g = w.grid
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    rho = math.sqrt(float(np.sum(4.0 * g.delta_f * np.abs(h) ** 2 / w.psd)))
    w = synth.scale_distance(w, rho / snr)
    return w, w.noise + h * (snr / rho)


@pytest.fixture(scope="module")
def event():
    return _event(30.0, 64.0, 3, 1000)


def _dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in arrays]


def _prepare(gw, w, data, e, flags=0, theta0=None):
    d_t, s_t = _dev(data, w.psd)
    return gw.RelativeBinning(w.grid, w.tensors, w.vertices, d_t, s_t, w.theta_inj if theta0 is None else theta0, e,
                              flags=flags)


def test_summary_matches_oracle(gw, event):
    w, data = event
    g = w.grid
    e = gw.rb_edges(g, 1.0, 0.1)
    h = _prepare(gw, w, data, e, flags=gw.FLAG_ADD_NORM)
    raw, tot = h.summary()
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e, add_norm=True)
    h0 = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    f = g.f_low + np.arange(g.n_bins) * g.delta_f
    wgt = 4.0 * g.delta_f / w.psd
    assert raw.shape == (len(e) - 1, w.n_det, 7)
    for b, (lo, hi) in enumerate(rb.bin_ranges(e)):
        sl = slice(lo, hi + 1)
        x = np.abs(f[sl] - 0.5 * (f[e[b]] + f[e[b + 1]]))
        for d in range(w.n_det):
            m_dh = np.sum(wgt[d, sl] * np.abs(data[d, sl]) * np.abs(h0[d, sl]))
            m_hh = np.sum(wgt[d, sl] * np.abs(h0[d, sl]) ** 2)
            want = [s["A0"][d, b].real, s["A0"][d, b].imag, s["A1"][d, b].real, s["A1"][d, b].imag,
                    s["B0"][d, b], s["B1"][d, b], s["B2"][d, b]]
            scale = [m_dh, m_dh, m_dh * x.max(), m_dh * x.max(), m_hh, m_hh * x.max(), m_hh * x.max() ** 2]
            for i in range(7):
                assert abs(raw[b, d, i] - want[i]) <= 1e-10 * scale[i], (b, d, i)
    assert tot[0] == pytest.approx(s["dd"], rel=1e-12)
    assert tot[1] == pytest.approx(s["norm"], rel=1e-12)
    h.close()


@pytest.mark.parametrize("eps", [0.5, 0.03])
def test_lnl_matches_oracle(gw, event, eps):
    import torch
    w, data = event
    g = w.grid
    e = gw.rb_edges(g, 1.0, eps)
    h = _prepare(gw, w, data, e)
    (th,) = _dev(w.theta)
    got = h.lnl(th)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    want = rb.lnl(s, w.tensors, w.vertices, w.theta)
    print(f"eps {eps}: {len(e) - 1} bins, max |dlnL| {np.abs(got - want).max():.3e}", flush=True)
    np.testing.assert_allclose(got, want, rtol=1e-10)
    np.testing.assert_allclose(got + 0.5 * s["dd"], want + 0.5 * s["dd"], rtol=0, atol=1e-8)
    h.close()


def test_every_bin_edges_equal_full_likelihood(gw):
    import torch
    w, data = _event(40.0, 4.0, 2, 300, snr=40.0, index=8)
    g = w.grid
    far = synth.near_fiducial(w.theta_inj, 300, np.random.default_rng(3), scale=300.0)
    far[:, 0] = w.theta_inj[0] * (1.0 + np.linspace(-0.02, 0.02, 300))
    e = np.arange(g.n_bins, dtype=np.int64)
    h = _prepare(gw, w, data, e)
    (th,) = _dev(far)
    got = h.lnl(th)
    d_t, s_t = _dev(data, w.psd)
    full = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, th)
    torch.cuda.synchronize()
    got, full = got.cpu().numpy(), full.cpu().numpy()
    want = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, far)
    np.testing.assert_allclose(got, want, rtol=1e-10)
    np.testing.assert_allclose(got, full, rtol=1e-10)
    h.close()


def test_fiducial_row_equals_full_likelihood(gw, event):
    import torch
    w, data = event
    g = w.grid
    h = _prepare(gw, w, data, gw.rb_edges(g, 1.0, 0.5))
    (th,) = _dev(w.theta_inj[None])
    d_t, s_t = _dev(data, w.psd)
    got = h.lnl(th)
    full = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, th)
    torch.cuda.synchronize()
    assert got.item() == pytest.approx(full.item(), rel=1e-11)
    h.close()


def test_domain_flags_and_shapes(gw, event):
    import torch
    w, data = event
    g = w.grid
    e = gw.rb_edges(g, 1.0, 0.5)
    h = _prepare(gw, w, data, e)
    hn = _prepare(gw, w, data, e, flags=gw.FLAG_ADD_NORM)
    assert h.shape == (len(e) - 1, 3)
    th = np.repeat(w.theta_inj[None], 5, axis=0)
    th[0, 4] = np.nan
    th[1, 1] = 1.5
    th[2, 0] = -1.0
    th[3, 2] = 0.0
    (tt,) = _dev(th)
    a = h.lnl(tt).cpu().numpy()
    b = hn.lnl(tt).cpu().numpy()
    assert np.isnan(a[0]) and a[1] == a[2] == a[3] == -np.inf and np.isfinite(a[4])
    norm = float(np.sum(np.log(2.0 * math.pi * w.psd)))
    assert b[4] == pytest.approx(a[4] - norm, rel=1e-12)
    empty = torch.empty((0, 9), dtype=torch.float64, device="cuda:0")
    assert h.lnl(empty).numel() == 0
    h.close()
    hn.close()


def test_five_parameter_rows(gw):
    import torch
    w = synth.small_event(3, 1, 5000, 300, n_param=5)
    g = w.grid
    h0 = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    data = w.noise + h0
    e = gw.rb_edges(g, 1.0, 0.2)
    d_t, s_t = _dev(data, w.psd)
    h = gw.RelativeBinning(g, None, None, d_t, s_t, w.theta_inj, e)
    th = w.theta.copy()
    th[:, 0] = w.theta_inj[0] * (1.0 + 1e-4 * np.random.default_rng(1).standard_normal(len(th)))
    (tt,) = _dev(th)
    got = h.lnl(tt)
    torch.cuda.synchronize()
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    want = rb.lnl(s, w.tensors, w.vertices, th)
    np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-10)
    h.close()


def test_argument_errors(gw, event):
    w, data = event
    g = w.grid
    e = gw.rb_edges(g, 1.0, 0.5)
    for flags in (gw.FLAG_TERM_ISCO, gw.FLAG_DIRECT):
        with pytest.raises(gw.GwError):
            _prepare(gw, w, data, e, flags=flags)
    for bad in (e[1:], e[:-1], np.array([0, 5, 5, g.n_bins - 1])):
        with pytest.raises(gw.GwError):
            _prepare(gw, w, data, bad)
    th0 = w.theta_inj.copy()
    th0[1] = 2.0
    with pytest.raises(gw.GwError):
        _prepare(gw, w, data, e, theta0=th0)


def test_benchmark_workload_sampled_rows(gw):
    import torch
    w, data = _event(15.0, 512.0, 3, 65536, index=6)
    g = w.grid
    e = gw.rb_edges(g, 1.0, 0.03)
    print(f"{g.n_bins} bins, {len(e) - 1} relative-binning bins, {w.n_samples} rows", flush=True)
    h = _prepare(gw, w, data, e)
    (th,) = _dev(w.theta)
    got = h.lnl(th)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.isfinite(got).all()
    rows = np.unique(np.concatenate([np.arange(0, 65536, 4099), [255, 256, 65535]]))
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    want = rb.lnl(s, w.tensors, w.vertices, w.theta[rows])
    np.testing.assert_allclose(got[rows], want, rtol=1e-10)
    np.testing.assert_allclose(got[rows] + 0.5 * s["dd"], want + 0.5 * s["dd"], rtol=0, atol=1e-7)
    # the mixed pass in the same launch shape: every row within 1e-3 of the FP64 one
    mixed = h.lnl(th, precision="mixed")
    torch.cuda.synchronize()
    assert np.abs(mixed.cpu().numpy() - got).max() <= 1e-3
    # the approximation against the full likelihood near the fiducial
    exact = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta[rows[:6]])
    print(f"  max |RB - exact| over 6 rows: {np.abs(got[rows[:6]] - exact).max():.3e}", flush=True)
    assert np.abs(got[rows[:6]] - exact).max() < 0.05
    h.close()


def test_longest_band(gw):
    """5 Hz / 8192 s, one detector: 16,736,257 grid bins carried by ~10^3
    bins of relative binning; the summary's totals and sampled rows against
    the oracle."""
    import torch
    w, data = _event(5.0, 8192.0, 1, 512, index=9)
    g = w.grid
    e = gw.rb_edges(g, 1.0, 0.03)
    print(f"{g.n_bins} bins, {len(e) - 1} relative-binning bins", flush=True)
    h = _prepare(gw, w, data, e)
    raw, tot = h.summary()
    (th,) = _dev(w.theta)
    got = h.lnl(th)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    assert tot[0] == pytest.approx(s["dd"], rel=1e-12)
    np.testing.assert_allclose(raw[:, 0, 4], s["B0"][0], rtol=1e-10)
    rows = np.array([0, 1, 255, 256, 511])
    want = rb.lnl(s, w.tensors, w.vertices, w.theta[rows])
    np.testing.assert_allclose(got[rows], want, rtol=1e-10)
    np.testing.assert_allclose(got[rows] + 0.5 * s["dd"], want + 0.5 * s["dd"], rtol=0, atol=1e-7)
    h.close()


@pytest.mark.parametrize("snr", [30.0, 100.0])
def test_mixed_precision(gw, snr):
    """The FP32 hardware phasor of the ratio: |dlnL| <= 1e-3 against the FP64
    pass (and the oracle) for near-fiducial rows at SNR 30 and 100."""
    import torch
    w, data = _event(30.0, 64.0, 3, 1000, snr=snr)
    g = w.grid
    e = gw.rb_edges(g, 1.0, 0.03)
    h = _prepare(gw, w, data, e)
    (th,) = _dev(w.theta)
    a = h.lnl(th)
    b = h.lnl(th, precision="mixed")
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
    want = rb.lnl(s, w.tensors, w.vertices, w.theta[:50])
    print(f"SNR {snr}: max |mixed - fp64| {np.abs(b - a).max():.3e}", flush=True)
    assert np.abs(b - a).max() <= 1e-3
    assert np.abs(b[:50] - want).max() <= 1e-3
    with pytest.raises(KeyError):
        h.lnl(th, precision="fp16")
    h.close()


def test_single_bin_and_single_row(gw, event):
    """The smallest partition (one bin, two edges) and a batch of one row."""
    import torch
    w, data = event
    g = w.grid
    e = np.array([0, g.n_bins - 1], dtype=np.int64)
    h = _prepare(gw, w, data, e)
    assert h.shape == (1, 3)
    for rows in (w.theta[:1], w.theta[:37]):
        (th,) = _dev(rows)
        got = h.lnl(th)
        torch.cuda.synchronize()
        s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta_inj, e)
        np.testing.assert_allclose(got.cpu().numpy(), rb.lnl(s, w.tensors, w.vertices, rows), rtol=1e-10)
    h.close()
