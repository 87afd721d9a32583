"""GPU parity of gw_lnl_batch (FP64 path) against the CPU oracle.

Bar: |lnL_gpu - lnL_oracle| <= 1e-10 |lnL_oracle| for every sample, the FP64
tolerance of the hot path.  Small cases compare every sample; at the full
3-detector 128 s size (259,585 bins, 4096 samples, the benchmark's launch) a
seeded sample of rows is checked one by one against the oracle.
"""
import math

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


def _to_gpu(w, data):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(np.ascontiguousarray(data)).to(dev), torch.from_numpy(w.psd).to(dev),
            torch.from_numpy(np.ascontiguousarray(w.theta)).to(dev))


def _gpu_lnl(gw, w, data, theta=None, **kw):
    import torch
    d, s, th = _to_gpu(w, data)
    if theta is not None:
        th = torch.from_numpy(np.ascontiguousarray(theta)).to(th.device)
    out = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _oracle_lnl(w, data, theta=None):
    g = w.grid
    return oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd,
                      w.theta if theta is None else theta)


def _assert_parity(got, ref, label=""):
    err = np.abs(got - ref)
    bound = RTOL * np.abs(ref)
    worst = int(np.argmax(err / np.maximum(bound, 1e-300)))
    print(f"{label}: max |dlnL| = {err.max():.3e}, max rel = {(err / np.abs(ref)).max():.3e}", flush=True)
    assert (err <= bound).all(), f"{label}: sample {worst} got {got[worst]!r} oracle {ref[worst]!r}"


SMALL_CASES = [
    # (seed, n_det, n_bins, n_samples, n_param)
    (1, 1, 1, 1, 5),
    (2, 1, 17, 3, 9),
    (3, 2, 511, 5, 9),
    (4, 3, 512, 256, 9),
    (5, 3, 513, 257, 9),
    (6, 3, 4097, 300, 9),
    (7, 8, 1000, 70, 9),
    (8, 5, 2049, 33, 9),
    (9, 1, 4017, 600, 5),
    (10, 4, 7777, 129, 9),
]


@pytest.mark.parametrize("seed,n_det,n_bins,n_samples,n_param", SMALL_CASES)
def test_small_cases_match_oracle(gw, seed, n_det, n_bins, n_samples, n_param):
    w = synth.small_event(seed, n_det, n_bins, n_samples, n_param)
    data = oracle.workload_data(w)
    got = _gpu_lnl(gw, w, data)
    ref = _oracle_lnl(w, data)
    _assert_parity(got, ref, f"seed {seed} det {n_det} bins {n_bins} S {n_samples} P {n_param}")


def test_one_detector_4s_workload_all_samples(gw):
    w = synth.bbh_1det_4s(1000)
    data = oracle.workload_data(w)
    got = _gpu_lnl(gw, w, data)
    ref = _oracle_lnl(w, data)
    _assert_parity(got, ref, "1 det 4 s 1000 samples")


def test_three_detector_128s_full_size_sampled(gw):
    """The benchmark's workload and launch: 4096 samples, 259,585 bins, 3 detectors.
    Every GPU value is finite; 24 seeded rows and the injection are checked
    against the oracle one by one."""
    w = synth.bbh_3det_128s(4096)
    data = oracle.workload_data(w)
    theta = w.theta.copy()
    theta[0] = w.theta_inj
    got = _gpu_lnl(gw, w, data, theta)
    assert np.isfinite(got).all()
    rows = np.sort(np.random.default_rng(99).choice(np.arange(1, 4096), 23, replace=False))
    rows = np.concatenate([[0], rows, [4095]])
    ref = _oracle_lnl(w, data, theta[rows])
    _assert_parity(got[rows], ref, "3 det 128 s sampled rows")
    # noise statistics at the injection: mean -N_det M, sd sqrt(N_det M)
    n = 3 * w.grid.n_bins
    assert abs(got[0] + n) < 5 * math.sqrt(n)


def test_three_detector_128s_every_row(gw):
    """All 4096 rows of the benchmark batch against the oracle (about 3.2e9
    sample-bin-detector terms; seconds on the host's cores)."""
    w = synth.bbh_3det_128s(4096)
    data = oracle.workload_data(w)
    got = _gpu_lnl(gw, w, data)
    ref = _oracle_lnl(w, data)
    _assert_parity(got, ref, "3 det 128 s, all 4096 rows")


def test_noise_free_maximum(gw):
    w = synth.small_event(20, 3, 3000, 40)
    g = w.grid
    h = oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None])[0]
    theta = np.vstack([w.theta_inj, w.theta])
    got = _gpu_lnl(gw, w, h, theta)
    # the split form reaches 0 up to rounding of <d,d>
    hh = 4 * g.delta_f * np.sum(np.abs(h) ** 2 / w.psd)
    assert abs(got[0]) <= 1e-12 * hh
    assert (got[1:] < got[0]).all()


def test_domain_rules_and_empty_batch(gw):
    import torch
    w = synth.small_event(21, 2, 300, 6)
    data = oracle.workload_data(w)
    theta = w.theta.copy()
    theta[1, 0] = -1.0
    theta[2, 1] = 1.2
    theta[3, 2] = 0.0
    theta[4, 5] = np.nan
    theta[5, 8] = np.inf
    got = _gpu_lnl(gw, w, data, theta)
    ref = _oracle_lnl(w, data, theta)
    assert np.isfinite(got[0]) and abs(got[0] - ref[0]) <= RTOL * abs(ref[0])
    assert (got[1:4] == -np.inf).all() and (ref[1:4] == -np.inf).all()
    assert np.isnan(got[4:]).all() and np.isnan(ref[4:]).all()
    out = gw.lnl_batch(w.grid, w.tensors, w.vertices, *_to_gpu(w, data)[:2],
                       torch.zeros((0, 9), dtype=torch.float64, device="cuda"))
    assert out.shape == (0,)


def test_invalid_psd_poisons_the_call(gw):
    w = synth.small_event(22, 2, 300, 4)
    data = oracle.workload_data(w)
    w.psd = w.psd.copy()
    w.psd[1, 17] = 0.0
    got = _gpu_lnl(gw, w, data)
    assert np.isnan(got).all()


def test_argument_errors(gw):
    import torch
    w = synth.small_event(23, 2, 100, 4)
    d, s, th = _to_gpu(w, oracle.workload_data(w))
    with pytest.raises(ValueError):
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d[:, :50], s, th)
    with pytest.raises(TypeError):
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s.float(), th)
    with pytest.raises(gw.GwError) as e:
        gw.lnl_batch((20.0, -1.0, 100), w.tensors, w.vertices, d, s, th)
    assert e.value.code == gw.GW_EINVAL
    with pytest.raises(gw.GwError) as e:
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th[:, :8].contiguous())
    assert e.value.code == gw.GW_EINVAL


def test_deterministic_and_stream_ordered(gw):
    import torch
    w = synth.small_event(24, 3, 20000, 700)
    data = oracle.workload_data(w)
    a = _gpu_lnl(gw, w, data)
    b = _gpu_lnl(gw, w, data)
    np.testing.assert_array_equal(a, b)
    d, s, th = _to_gpu(w, data)
    side = torch.cuda.Stream()
    ws = gw.Workspace(0)
    with torch.cuda.stream(side):
        out = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws)
    side.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), a)


def test_reserved_workspace_does_not_grow(gw):
    w = synth.small_event(25, 3, 5000, 300)
    data = oracle.workload_data(w)
    ws = gw.Workspace(0)
    ws.reserve(5000, 3, 300)
    before = ws.nbytes
    got = _gpu_lnl(gw, w, data, workspace=ws)
    assert ws.nbytes == before
    _assert_parity(got, _oracle_lnl(w, data), "reserved workspace")
