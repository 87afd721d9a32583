"""GPU parity of the likelihood options against the oracle.

* GW_FLAG_DIRECT: the literal residual sum of Eq. (cbclike), accumulated per
  (sample, bin, detector);
* GW_FLAG_TERM_ISCO: every template ends at its innermost-stable-circular-
  orbit frequency (the split form then sums only the bins below it and takes
  Q from prefix sums; the chunks of the tile kernel cover only bins below the
  batch's largest cut-off);
* GW_FLAG_ADD_NORM: the log of the prod 1/(2 pi S) factor of Eq. (cbclike).

Bars: FP64 |dlnL| <= 1e-10 |lnL|; mixed path |dlnL| <= 1e-3 (SNR <= 100
data); waveform bins 1e-10 relative below the cut-off and exact zeros above.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10
DIRECT, ISCO, NORM = 1, 2, 4
COMBOS = [DIRECT, ISCO, NORM, DIRECT | ISCO, ISCO | NORM, DIRECT | ISCO | NORM]


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda", 0))


def _oracle(w, data, theta, flags):
    g = w.grid
    return oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, theta,
                      isco=bool(flags & ISCO), add_norm=bool(flags & NORM))


def _check(got, ref, label, rtol=RTOL, atol=0.0):
    err = np.abs(got - ref)
    bound = rtol * np.abs(ref) + atol
    print(f"{label}: max |dlnL| {err.max():.3e}, max rel {(err / np.abs(ref)).max():.3e}", flush=True)
    worst = int(np.argmax(err - bound))
    assert (err <= bound).all(), f"{label}: row {worst} got {got[worst]!r} oracle {ref[worst]!r}"


CASES = [
    # (seed, n_det, n_bins, n_samples, n_param): 20 Hz + k/4 Hz, so the cut-off
    # of these 25-35 solar-mass chirps (55-80 Hz) falls inside the band
    (21, 1, 3001, 300, 5),
    (22, 3, 3001, 257, 9),
    (23, 2, 700, 70, 9),
    (24, 8, 1500, 33, 9),
]


@pytest.mark.parametrize("flags", COMBOS)
@pytest.mark.parametrize("seed,n_det,n_bins,n_samples,n_param", CASES)
def test_flags_match_oracle_fp64(gw, flags, seed, n_det, n_bins, n_samples, n_param):
    import torch
    w = synth.small_event(seed, n_det, n_bins, n_samples, n_param)
    data = oracle.workload_data(w)
    got = gw.lnl_batch(w.grid, w.tensors, w.vertices, _dev(data), _dev(w.psd), _dev(w.theta), flags=flags)
    torch.cuda.synchronize()
    _check(got.cpu().numpy(), _oracle(w, data, w.theta, flags), f"flags {flags} seed {seed}")


@pytest.mark.parametrize("flags", [DIRECT, ISCO, DIRECT | ISCO | NORM])
def test_flags_mixed_precision(gw, flags):
    import torch
    w = synth.small_event(25, 3, 3001, 300, 9)
    data = oracle.workload_data(w)
    got = gw.lnl_batch(w.grid, w.tensors, w.vertices, _dev(data), _dev(w.psd), _dev(w.theta), flags=flags,
                       precision="mixed")
    torch.cuda.synchronize()
    _check(got.cpu().numpy(), _oracle(w, data, w.theta, flags), f"mixed flags {flags}", rtol=0.0, atol=1e-3)


def test_cutoff_below_the_band_leaves_only_the_data(gw):
    # total mass ~460 solar masses: f_isco ~ 9.6 Hz < f_low, so h = 0 everywhere
    # and lnL = -<d,d>/2 for every sample; every chunk of the tile kernel is empty
    import torch
    w = synth.small_event(26, 3, 2000, 40, 9)
    theta = w.theta.copy()
    theta[:, 0] = 200.0
    data = oracle.workload_data(w)
    for flags in (ISCO, DIRECT | ISCO):
        got = gw.lnl_batch(w.grid, w.tensors, w.vertices, _dev(data), _dev(w.psd), _dev(theta), flags=flags)
        torch.cuda.synchronize()
        ref = _oracle(w, data, theta, flags)
        _check(got.cpu().numpy(), ref, f"all below f_low, flags {flags}")
        assert np.ptp(ref) == 0.0


def test_mixed_cutoffs_within_one_batch(gw):
    # chirp masses spread over two decades so that some rows end in the
    # band's first bins, some past its top, and one below f_low
    import torch
    w = synth.small_event(27, 2, 6001, 260, 9)
    theta = w.theta.copy()
    theta[:, 0] = np.geomspace(1.0, 150.0, theta.shape[0])
    data = oracle.workload_data(w)
    for flags in (ISCO, DIRECT | ISCO, ISCO | NORM):
        got = gw.lnl_batch(w.grid, w.tensors, w.vertices, _dev(data), _dev(w.psd), _dev(theta), flags=flags)
        torch.cuda.synchronize()
        _check(got.cpu().numpy(), _oracle(w, data, theta, flags), f"spread cut-offs, flags {flags}")


def test_domain_rules_hold_with_flags(gw):
    import torch
    w = synth.small_event(28, 3, 800, 6, 9)
    theta = w.theta.copy()
    theta[1, 3] = np.nan
    theta[2, 0] = -1.0
    theta[3, 1] = 1.5
    data = oracle.workload_data(w)
    for flags in COMBOS:
        got = gw.lnl_batch(w.grid, w.tensors, w.vertices, _dev(data), _dev(w.psd), _dev(theta), flags=flags)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert np.isnan(g[1]) and g[2] == -np.inf and g[3] == -np.inf
        keep = [0, 4, 5]
        _check(g[keep], _oracle(w, data, theta[keep], flags), f"domain, flags {flags}")


@pytest.mark.parametrize("n_det", [0, 3])
def test_waveform_cutoff(gw, n_det):
    import torch
    w = synth.small_event(29, 3, 1201, 20, 9)
    g = w.grid
    tensors, vertices = (w.tensors, w.vertices) if n_det else (None, None)
    got = gw.waveform_batch(g, tensors, vertices, _dev(w.theta), flags=ISCO)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, tensors, vertices, w.theta, isco=True)
    zero = ref == 0
    assert zero.any() and (~zero).any()
    assert np.array_equal(got == 0, zero)
    err = np.abs(got[~zero] - ref[~zero])
    assert (err <= 1e-10 * np.abs(ref[~zero])).all(), f"max rel {(err / np.abs(ref[~zero])).max():.3e}"


def test_unknown_flag_bits_are_rejected(gw):
    w = synth.small_event(30, 1, 64, 2, 5)
    for bad in (8, 1 << 31):
        with pytest.raises(Exception, match="flag"):
            gw.lnl_batch(w.grid, w.tensors, w.vertices, _dev(w.noise), _dev(w.psd), _dev(w.theta), flags=bad)
    for bad in (DIRECT, NORM, 8):
        with pytest.raises(Exception, match="flag"):
            gw.waveform_batch(w.grid, w.tensors, w.vertices, _dev(w.theta), flags=bad)


def test_full_size_with_cutoff_and_direct_form(gw):
    """The 3-detector 128 s batch (259,585 bins, 4096 samples): with the ISCO
    end the tile kernel's chunks shrink to the bins below the largest cut-off
    (about 4% of the band); sampled rows against the oracle."""
    import torch
    w = synth.bbh_3det_128s(4096)
    g = w.grid
    data = w.noise + oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    rows = np.sort(np.random.default_rng(8).choice(4096, 6, replace=False))
    d, s, th = _dev(data), _dev(w.psd), _dev(w.theta)
    for flags in (ISCO, DIRECT, DIRECT | ISCO | NORM):
        got = gw.lnl_batch(g, w.tensors, w.vertices, d, s, th, flags=flags)
        torch.cuda.synchronize()
        _check(got.cpu().numpy()[rows], _oracle(w, data, w.theta[rows], flags), f"full size, flags {flags}")


@pytest.mark.parametrize("flags", [DIRECT, ISCO, DIRECT | ISCO | NORM])
def test_ragged_with_flags(gw, flags):
    import torch
    evs = synth.bns_ragged(n_events=7, n_samples=130, index=51, t_min=1.0, t_max=8.0)
    counts = [130, 1, 64, 129, 0, 17, 100][:len(evs)]
    datas, psds, thetas = [], [], []
    for e, n in zip(evs, counts):
        g = e.grid
        datas.append((e.noise + oracle.waveform(g.f_low, g.delta_f, g.n_bins, e.tensors, e.vertices,
                                                e.theta_inj[None])[0]).ravel())
        psds.append(e.psd.ravel())
        thetas.append(e.theta[:n])
    events, total, n_rows = gw.make_events([e.grid for e in evs], [e.tensors for e in evs],
                                           [e.vertices for e in evs], counts)
    ws = gw.Workspace(0)
    out = gw.lnl_ragged(events, len(evs), _dev(np.concatenate(datas)), _dev(np.concatenate(psds)),
                        _dev(np.concatenate(thetas)), flags=flags, workspace=ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    row = 0
    for i, (e, n) in enumerate(zip(evs, counts)):
        if n:
            g = e.grid
            ref = oracle.lnl(g.f_low, g.delta_f, g.n_bins, e.tensors, e.vertices, datas[i].reshape(3, g.n_bins),
                             e.psd, e.theta[:n], isco=bool(flags & ISCO), add_norm=bool(flags & NORM))
            _check(got[row:row + n], ref, f"ragged event {i} flags {flags}")
        row += n
    ws.close()
