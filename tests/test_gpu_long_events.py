"""Long neutron-star events (Sec. III: about 10^6 bins from 20 Hz, many more
from 10 Hz at design sensitivity and 5 Hz for future detectors): the phase
reaches ~10^4 turns at the lowest bins and the bin count grows to 1.7e7, so
these cases stress the exact fractional-turn reduction and the tiling.

Cases: 15 Hz / 512 s (1,040,897 bins, 3 detectors), 10 Hz / 2048 s
(4,173,825 bins, 2 detectors), 5 Hz / 8192 s (16,736,257 bins, 1 detector).
The injection is rescaled to network SNR 30.  Rows checked against the oracle:
the injection and three more, FP64 (1e-10 relative, with and without the
ISCO end, whose prefix sums then span up to 65,377 blocks) and mixed (1e-3).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


@pytest.mark.parametrize("f_low,duration,n_det,n_samples", [(15.0, 512.0, 3, 256), (10.0, 2048.0, 2, 128),
                                                            (5.0, 8192.0, 1, 64)])
def test_long_event_matches_oracle(gw, f_low, duration, n_det, n_samples):
    import torch
    w = synth.long_bns(f_low, duration, n_det, n_samples)
    g = w.grid
    print(f"{w.name}: {g.n_bins} bins x {n_det} detectors", flush=True)
    inj = w.theta_inj.copy()
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, inj[None])[0]
    snr = math.sqrt(float(np.sum(4.0 * g.delta_f * (h.real ** 2 + h.imag ** 2) / w.psd)))
    h *= 30.0 / snr
    inj[2] *= snr / 30.0
    data = w.noise + h
    del h
    theta = w.theta.copy()
    theta[0] = inj
    rows = np.array([0, 1, n_samples // 2, n_samples - 1])
    dev = torch.device("cuda", 0)
    d_t = torch.from_numpy(data).to(dev)
    s_t = torch.from_numpy(w.psd).to(dev)
    th_t = torch.from_numpy(theta).to(dev)
    for flags, precision, tol in ((0, "fp64", None), (2, "fp64", None), (0, "mixed", 1e-3)):
        got = gw.lnl_batch(g, w.tensors, w.vertices, d_t, s_t, th_t, flags=flags, precision=precision)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert np.isfinite(got).all()
        ref = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, theta[rows],
                         isco=bool(flags & 2))
        err = np.abs(got[rows] - ref)
        bound = 1e-10 * np.abs(ref) if tol is None else tol
        print(f"  flags {flags} {precision}: max |dlnL| {err.max():.3e} (max rel {(err / np.abs(ref)).max():.2e})",
              flush=True)
        assert (err <= bound).all()
