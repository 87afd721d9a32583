"""Aligned-spin templates on the GPU against the oracle.

* gw_lnl_batch with 11- and 7-parameter rows (spins U[-1, 1]): FP64 within
  1e-10 relative (also with the template end), mixed within 1e-3; the
  3-detector 128 s benchmark batch with spins on sampled rows.
* gw_waveform_batch with spins, bin by bin within 1e-10 relative.
* Zero spins give exactly the non-spinning results (same kernels, same
  coefficients); |chi| > 1 gives -inf, a non-finite spin NaN.
* gw_lnl_ragged and relative binning with spinning rows against the oracle.
* The sampler with physical spins (11 coordinates, the last two passed on as
  chi1, chi2): the lnL its chains carry is the oracle's for 11-parameter
  rows, and the chains' effective spin chi_eff concentrates near the
  injection's instead of spreading over the prior.
"""
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


def _dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in arrays]


def _event(index, n_det, n_bins, n_samples, n_param):
    w = synth.small_event(index, n_det, n_bins, n_samples, n_param)
    rng = np.random.default_rng(index)
    inj = synth.add_spins(w.theta_inj, rng)[0]
    theta = synth.add_spins(w.theta, rng)
    g = w.grid
    data = w.noise + oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, inj[None])[0]
    return w, inj, theta, data


@pytest.mark.parametrize("index,n_det,n_bins,n_samples,n_param", [(1, 3, 4097, 300, 9), (2, 1, 4017, 257, 5),
                                                                  (3, 2, 2049, 64, 9)])
def test_lnl_with_spins_matches_oracle(gw, index, n_det, n_bins, n_samples, n_param):
    import torch
    w, inj, theta, data = _event(index, n_det, n_bins, n_samples, n_param)
    g = w.grid
    d_t, s_t, th_t = _dev(data, w.psd, theta)
    for flags, precision, tol in ((0, "fp64", None), (2, "fp64", None), (0, "mixed", 1e-3)):
        got = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, th_t, flags=flags, precision=precision)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        ref = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, theta,
                         isco=bool(flags & 2))
        err = np.abs(got - ref)
        print(f"P={n_param + 2} flags {flags} {precision}: max |dlnL| {err.max():.3e}", flush=True)
        assert (err <= (1e-10 * np.abs(ref) if tol is None else tol)).all()


def test_zero_spins_equal_non_spinning(gw):
    import torch
    w, inj, theta, data = _event(4, 3, 3001, 300, 9)
    g = w.grid
    th0 = theta.copy()
    th0[:, 9:] = 0.0
    d_t, s_t, t11, t9 = _dev(data, w.psd, th0, th0[:, :9])
    a = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, t11)
    b = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, t9)
    ha = gw.waveform_batch(g, w.tensors, w.vertices, t11[:5].contiguous())
    hb = gw.waveform_batch(g, w.tensors, w.vertices, t9[:5].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ha, hb)


def test_waveform_with_spins(gw):
    import torch
    for n_param in (9, 5):
        w, inj, theta, data = _event(5, 3, 3001, 7, n_param)
        g = w.grid
        (th,) = _dev(theta)
        got = gw.waveform_batch(g, w.tensors if n_param == 9 else None, w.vertices if n_param == 9 else None, th)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        if n_param == 5:
            ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, None, None, theta)
        else:
            ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, theta)
        err = np.abs(got - ref)
        print(f"P={n_param + 2}: max rel {(err / np.abs(ref)).max():.3e}", flush=True)
        assert (err <= 1e-10 * np.abs(ref)).all()


def test_spin_domain(gw):
    import torch
    w, inj, theta, data = _event(6, 2, 1000, 6, 9)
    g = w.grid
    th = theta.copy()
    th[0, 9] = 1.0001
    th[1, 10] = -2.0
    th[2, 9] = np.nan
    th[3, 9:] = [1.0, -1.0]
    d_t, s_t, th_t = _dev(data, w.psd, th)
    out = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, th_t)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    assert out[0] == -np.inf and out[1] == -np.inf and np.isnan(out[2]) and np.isfinite(out[3:]).all()


def test_benchmark_batch_with_spins_sampled_rows(gw):
    import torch
    w = synth.bbh_3det_128s(4096)
    rng = np.random.default_rng(11)
    inj = synth.add_spins(w.theta_inj, rng)[0]
    theta = synth.add_spins(w.theta, rng)
    g = w.grid
    data = w.noise + oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, inj[None])[0]
    d_t, s_t, th_t = _dev(data, w.psd, theta)
    got = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, th_t)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    rows = np.array([0, 1, 255, 256, 2047, 4095])
    ref = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, theta[rows])
    assert (np.abs(got[rows] - ref) <= 1e-10 * np.abs(ref)).all()


def test_ragged_with_spins(gw):
    import torch
    evs = synth.bns_ragged(n_events=6, n_samples=100, index=60, t_min=1.0, t_max=6.0)
    rng = np.random.default_rng(12)
    datas, psds, thetas = [], [], []
    for e in evs:
        g = e.grid
        inj = synth.add_spins(e.theta_inj, rng)[0]
        datas.append((e.noise + oracle.waveform(g.f_low, g.delta_f, g.n_bins, e.tensors, e.vertices,
                                                inj[None])[0]).ravel())
        psds.append(e.psd.ravel())
        thetas.append(synth.add_spins(e.theta, rng))
    events, total, rows = gw.make_events([e.grid for e in evs], [e.tensors for e in evs],
                                         [e.vertices for e in evs], [100] * len(evs))
    d_t, s_t, th_t = _dev(np.concatenate(datas), np.concatenate(psds), np.concatenate(thetas))
    out = gw.lnl_ragged(events, len(evs), d_t, s_t, th_t)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for i, e in enumerate(evs):
        g = e.grid
        pick = [0, 57, 99]
        ref = oracle.lnl(g.f_low, g.delta_f, g.n_bins, e.tensors, e.vertices, datas[i].reshape(e.psd.shape), e.psd,
                         thetas[i][pick])
        got = out[i * 100 + np.array(pick)]
        assert (np.abs(got - ref) <= 1e-10 * np.abs(ref)).all(), i


def test_relative_binning_with_spins(gw):
    import torch
    w = synth.relbin_bns(30.0, 64.0, 3, 500)
    g = w.grid
    rng = np.random.default_rng(13)
    inj = synth.add_spins(w.theta_inj, rng, 0.3)[0]
    theta = np.hstack([w.theta, inj[None, 9:] + 0.01 * rng.standard_normal((500, 2))])
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, inj[None])[0]
    rho = math.sqrt(float(np.sum(4.0 * g.delta_f * np.abs(h) ** 2 / w.psd)))
    inj[2] *= rho / 30.0
    theta[:, 2] *= rho / 30.0
    data = w.noise + h * (30.0 / rho)
    e = gw.rb_edges(g, 1.0, 0.1)
    d_t, s_t, th_t = _dev(data, w.psd, theta)
    hnd = gw.RelativeBinning(g, w.tensors, w.vertices, d_t, s_t, inj, e)
    got = hnd.lnl(th_t)
    fid = hnd.lnl(torch.from_numpy(inj[None]).to("cuda:0"))
    full = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, torch.from_numpy(inj[None]).to("cuda:0"))
    torch.cuda.synchronize()
    s = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, inj, e)
    want = rb.lnl(s, w.tensors, w.vertices, theta)
    np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-10)
    assert fid.item() == pytest.approx(full.item(), rel=1e-11)
    hnd.close()


def test_sampler_with_physical_spins(gw):
    import torch
    import oracle
    from paper_1904_02863_amd import sampler
    g = synth.make_grid(20.0, 256.0, 8.0)
    rng = synth.seeds(78)
    tensors, vertices = synth.stack_detectors(synth.network(rng["detectors"], 3))
    f = g.frequencies()
    s = np.ascontiguousarray(np.broadcast_to(synth.psd(f), (3, g.n_bins)))
    noise = np.stack([synth.noise(rng["noise"], s[d], g.delta_f) for d in range(3)])
    inj = np.array([12.0, 0.8, 300.0, 1.0, 0.01, 2.0, 0.3, 0.7, 0.6, 0.5, 0.3])
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, tensors, vertices, inj[None])[0]
    rho = math.sqrt(float(np.sum(4.0 * g.delta_f * np.abs(h) ** 2 / s)))
    inj[2] *= rho / 25.0
    data_np = noise + h * (25.0 / rho)
    d_t, s_t = _dev(data_np, s)
    ws = gw.Workspace(0)
    sd, ci = math.sin(inj[6]), math.cos(inj[8])
    lo = np.array([10.0, 0.5, 0.2 * inj[2], 0.0, -0.1, inj[5] - 0.05, sd - 0.05, inj[7] - 0.05, ci - 0.05, -1.0, -1.0])
    hi = np.array([14.0, 1.0, 3.0 * inj[2], 2 * math.pi, 0.1, inj[5] + 0.05, sd + 0.05, inj[7] + 0.05, ci + 0.05,
                   1.0, 1.0])
    prob = sampler.Problem(g, tensors, vertices, d_t, s_t, lo, hi, spins=True)
    p_inj = np.array([inj[0], inj[1], inj[2], inj[3], inj[4], inj[5], sd, inj[7], ci, inj[9], inj[10]])
    n = 1024
    r = np.random.default_rng(4)
    x0 = sampler.to_sampler_coords(prob, p_inj)[None] + r.normal(scale=1e-3, size=(n, 11))
    state = sampler.init_chains(prob, x0, ws)
    chol = np.diag(np.full(11, 1e-3))
    _, acc, _, chol, _ = sampler.run_random_walk(prob, state, 3000, 5, chol, ws, adapt_every=100)
    print(f"acceptance {acc:.3f}", flush=True)
    th, lp = gw.mcmc_to_theta(lo, hi, state.x, theta_cols=11)
    theta = th.cpu().numpy()
    carried = (state.lnp - lp).cpu().numpy()
    pick = np.random.default_rng(9).choice(n, 16, replace=False)
    want = oracle.lnl(g.f_low, g.delta_f, g.n_bins, tensors, vertices, data_np, s, theta[pick])
    np.testing.assert_allclose(carried[pick], want, rtol=1e-10, atol=1e-8)
    x1 = 1.0 / (1.0 + theta[:, 1])
    chi_eff = x1 * theta[:, 9] + (1.0 - x1) * theta[:, 10]
    inj_x1 = 1.0 / (1.0 + inj[1])
    inj_eff = inj_x1 * inj[9] + (1.0 - inj_x1) * inj[10]
    print(f"chi_eff: injection {inj_eff:.3f}, chains {chi_eff.mean():.3f} +- {chi_eff.std():.3f}", flush=True)
    # the prior alone would give chi_eff a spread of about 0.41 around 0
    assert chi_eff.std() < 0.3
    assert abs(chi_eff.mean() - inj_eff) < 3.0 * chi_eff.std() + 0.05
