"""GPU parity of gw_waveform_batch (the template of Sec. II) against the oracle,
bin by bin: |h_gpu - h_oracle| <= 1e-10 |h_oracle| for every element."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def _run(gw, grid, tensors, vertices, theta):
    import torch
    th = torch.from_numpy(np.ascontiguousarray(theta)).to("cuda")
    out = gw.waveform_batch(grid, tensors, vertices, th)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(got, ref, label):
    assert got.shape == ref.shape
    err = np.abs(got - ref)
    rel = err / np.abs(ref)
    print(f"{label}: max rel {rel.max():.3e}", flush=True)
    assert (err <= RTOL * np.abs(ref)).all(), label


@pytest.mark.parametrize("n_bins", [1, 255, 256, 257, 4017])
def test_polarisations(gw, n_bins):
    w = synth.small_event(30, 1, n_bins, 9, 9)
    g = w.grid
    got = _run(gw, g, None, None, w.theta)
    ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, None, None, w.theta)
    _check(got, ref, f"polarisations M={n_bins}")


@pytest.mark.parametrize("n_det,n_param", [(1, 5), (3, 9), (8, 9)])
def test_detector_responses(gw, n_det, n_param):
    w = synth.small_event(31, n_det, 3001, 7, n_param)
    g = w.grid
    got = _run(gw, g, w.tensors, w.vertices, w.theta)
    ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta)
    _check(got, ref, f"responses det={n_det} P={n_param}")


def test_neutron_star_long_segment(gw):
    """A 256 s neutron-star event: phases of ~1e4 rad at 20 Hz."""
    ev = synth.bns_ragged(n_events=40, n_samples=3)
    e = max(ev, key=lambda x: x.grid.n_bins)
    g = e.grid
    got = _run(gw, g, e.tensors, e.vertices, e.theta)
    ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, e.tensors, e.vertices, e.theta)
    _check(got, ref, f"BNS {g.n_bins} bins")


def test_out_of_domain_rows_are_nan(gw):
    w = synth.small_event(32, 2, 100, 3, 9)
    th = w.theta.copy()
    th[1, 1] = 2.0
    th[2, 0] = np.nan
    got = _run(gw, w.grid, w.tensors, w.vertices, th)
    assert np.isfinite(got[0]).all()
    assert np.isnan(got[1:]).all()


@pytest.mark.parametrize("n_samples,n_bins", [(16, 1024), (17, 1025), (37, 3001), (100, 257)])
def test_sample_groups_and_span_tails(gw, n_samples, n_bins):
    """Blocks cover a group of samples x 1024 bins: whole and partial sample
    groups, whole and ragged bin spans."""
    w = synth.small_event(33, 3, n_bins, n_samples, 9)
    g = w.grid
    got = _run(gw, g, w.tensors, w.vertices, w.theta)
    ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta)
    _check(got, ref, f"S={n_samples} M={n_bins}")


def test_benchmark_batch_sampled(gw):
    """The benchmark's launch: 256 samples x 3 detectors x 259,585 bins
    (3.2 GB written); sampled rows against the oracle, every bin of them."""
    import torch
    w = synth.bbh_3det_128s(256)
    g = w.grid
    th = torch.from_numpy(w.theta).to("cuda")
    out = gw.waveform_batch(g, w.tensors, w.vertices, th)
    torch.cuda.synchronize()
    rows = [0, 3, 4, 127, 255]
    got = out[rows].cpu().numpy()
    del out
    ref = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta[rows])
    _check(got, ref, "benchmark batch")


def test_fill_writes_every_element():
    import torch

    import paper_1904_02863_amd as gw
    gw.load_library()
    for n in (1, 255, 256, 100_003, 3 * 259_585):
        out = torch.full((n,), complex(7.0, 7.0), dtype=torch.complex128, device="cuda:0")
        gw.fill_c128(out, complex(-1.5, 2.25))
        torch.cuda.synchronize()
        assert bool((out == complex(-1.5, 2.25)).all())
    empty = torch.empty(0, dtype=torch.complex128, device="cuda:0")
    gw.fill_c128(empty, 1.0)
