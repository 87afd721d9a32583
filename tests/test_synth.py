"""The seeded input generators: grids, PSD, detectors, noise, priors."""
import math

import numpy as np
import pytest

import synth


def test_grid_sizes():
    assert synth.make_grid(20.0, 1024.0, 4.0).n_bins == 4017
    g = synth.make_grid(20.0, 2048.0, 128.0)
    assert g.n_bins == 259585 and g.delta_f == 1 / 128
    assert g.frequencies()[-1] == 2048.0
    with pytest.raises(ValueError):
        synth.make_grid(20.0, 100.1, 4.0)


def test_psd_positive_with_minimum_near_228hz():
    f = np.linspace(5, 4096, 400000)
    s = synth.psd(f)
    assert (s > 0).all()
    i = np.argmin(s)
    assert 215 < f[i] < 240
    assert s[i] == pytest.approx(3.24e-48, rel=0.01)


def test_detector_tensor_geometry():
    for name, lat, lon in synth.SITES_DEG:
        det = synth.detector_at(name, lat, lon, 1.234)
        t = det.tensor
        np.testing.assert_allclose(t, t.T, atol=0)
        assert abs(np.trace(t)) < 1e-15
        np.testing.assert_allclose(np.linalg.eigvalsh(t), [-0.5, 0.0, 0.5], atol=1e-15)
        # the arms lie in the local tangent plane: the vertex is the null direction
        np.testing.assert_allclose(t @ det.vertex, 0.0, atol=1e-8)
        assert np.linalg.norm(det.vertex) == pytest.approx(synth.EARTH_RADIUS_M, rel=1e-15)


def test_noise_variance():
    rng = np.random.default_rng(0)
    s = np.full(400000, 4e-47)
    n = synth.noise(rng, s, 0.25)
    assert np.var(n.real) == pytest.approx(4e-47 / 1.0, rel=0.01)
    assert np.var(n.imag) == pytest.approx(4e-47 / 1.0, rel=0.01)
    assert abs(np.mean(n.real * n.imag)) < 3e-49


def test_prior_ranges_and_seeding():
    th = synth.Prior().sample(np.random.default_rng(1), 20000, 9)
    assert th.shape == (20000, 9)
    assert (th[:, 0] >= 25).all() and (th[:, 0] <= 35).all()
    assert (th[:, 1] >= 0.5).all() and (th[:, 1] <= 1).all()
    assert (np.abs(th[:, 6]) <= math.pi / 2).all()
    assert np.mean(np.sin(th[:, 6])) == pytest.approx(0.0, abs=0.03)
    assert np.mean(np.cos(th[:, 8])) == pytest.approx(0.0, abs=0.03)
    a = synth.bbh_1det_4s(10)
    b = synth.bbh_1det_4s(10)
    np.testing.assert_array_equal(a.theta, b.theta)
    np.testing.assert_array_equal(a.noise, b.noise)
    assert a.grid.n_bins == 4017 and a.n_param == 5


def test_ragged_durations():
    ev = synth.bns_ragged(n_events=32, n_samples=4)
    durs = [round(1 / e.grid.delta_f) for e in ev]
    assert all(8 <= t <= 256 for t in durs)
    assert all(abs(1 / e.grid.delta_f - t) < 1e-9 for e, t in zip(ev, durs))
    assert all(e.grid.n_bins == 2028 * t + 1 for e, t in zip(ev, durs))
    assert len(set(durs)) > 10
    mc = np.concatenate([e.theta[:, 0] for e in ev])
    assert (mc > 0.8).all() and (mc < 1.75).all()
