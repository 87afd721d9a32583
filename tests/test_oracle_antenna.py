"""Pins of the oracle's antenna patterns and time delays.

Convention-free invariants of F+ = D:e+, Fx = D:ex (the sign of psi and the
orientation of the sky basis are readings, and only invariants pin them):
* rotating psi by pi/4 maps (F+, Fx) to (Fx, -F+); by pi/2 flips both;
* F+^2 + Fx^2 is independent of psi and, in the detector frame with polar
  angle theta and azimuth phi, equals (1/4)(1 + cos^2 theta)^2 cos^2 2phi
  + cos^2 theta sin^2 2phi (Thorne 1987, in 300 Years of Gravitation);
* a source at the zenith of an L-shaped detector has F+^2 + Fx^2 = 1;
* over an isotropic sky and uniform psi, <F+^2> = <Fx^2> = 1/5.
Delays: -n.r/c gives -R_E/c for a zenith source, and never more than the
light travel time between two sites.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _dets():
    rng = np.random.default_rng(17)
    return synth.network(rng, 3)


@pytest.mark.parametrize("ra,dec,psi", [(0.3, 0.2, 0.1), (4.0, -1.1, 2.7), (2.2, 0.9, 1.0)])
def test_psi_rotations(ra, dec, psi):
    for det in _dets():
        fp, fx = oracle.antenna(det.tensor, ra, dec, psi)
        gp, gx = oracle.antenna(det.tensor, ra, dec, psi + math.pi / 4)
        hp, hx = oracle.antenna(det.tensor, ra, dec, psi + math.pi / 2)
        assert (gp, gx) == pytest.approx((fx, -fp), abs=1e-14)
        assert (hp, hx) == pytest.approx((-fp, -fx), abs=1e-14)


def test_thorne_detector_frame_formula():
    rng = np.random.default_rng(3)
    for det in _dets():
        w, vecs = np.linalg.eigh(det.tensor)       # eigenvalues -1/2, 0, +1/2
        ey, ez, ex = vecs[:, 0], vecs[:, 1], vecs[:, 2]
        for _ in range(50):
            ra, dec, psi = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-1, 1)), rng.uniform(0, math.pi)
            n = np.array([math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)])
            ct = n @ ez
            phi = math.atan2(n @ ey, n @ ex)
            expect = 0.25 * (1 + ct * ct) ** 2 * math.cos(2 * phi) ** 2 + ct * ct * math.sin(2 * phi) ** 2
            fp, fx = oracle.antenna(det.tensor, ra, dec, psi)
            assert fp * fp + fx * fx == pytest.approx(expect, abs=1e-13)


def test_zenith_source_has_unit_response():
    for name, lat, lon in synth.SITES_DEG:
        det = synth.detector_at(name, lat, lon, 0.7)
        for psi in (0.0, 0.4, 2.0):
            fp, fx = oracle.antenna(det.tensor, math.radians(lon), math.radians(lat), psi)
            assert fp * fp + fx * fx == pytest.approx(1.0, abs=1e-14)


def test_sky_average_is_one_fifth():
    rng = np.random.default_rng(11)
    det = _dets()[0]
    n = 40000
    ra = rng.uniform(0, 2 * math.pi, n)
    dec = np.arcsin(rng.uniform(-1, 1, n))
    psi = rng.uniform(0, math.pi, n)
    f = np.array([oracle.antenna(det.tensor, a, b, c) for a, b, c in zip(ra, dec, psi)])
    assert np.mean(f[:, 0] ** 2) == pytest.approx(0.2, abs=0.006)
    assert np.mean(f[:, 1] ** 2) == pytest.approx(0.2, abs=0.006)


def test_zenith_delay_and_light_travel_bound():
    for name, lat, lon in synth.SITES_DEG:
        det = synth.detector_at(name, lat, lon, 0.0)
        dt = oracle.delay(det.vertex, math.radians(lon), math.radians(lat))
        assert dt == pytest.approx(-synth.EARTH_RADIUS_M / 299792458.0, rel=1e-14)
    d = _dets()
    rng = np.random.default_rng(2)
    base = np.linalg.norm(d[0].vertex - d[1].vertex) / 299792458.0
    worst = 0.0
    for _ in range(500):
        ra, dec = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-1, 1))
        gap = abs(oracle.delay(d[0].vertex, ra, dec) - oracle.delay(d[1].vertex, ra, dec))
        worst = max(worst, gap)
        assert gap <= base * (1 + 1e-14)
    # along the baseline the bound is reached
    b = (d[1].vertex - d[0].vertex) / np.linalg.norm(d[1].vertex - d[0].vertex)
    ra, dec = math.atan2(b[1], b[0]), math.asin(b[2])
    gap = abs(oracle.delay(d[0].vertex, ra, dec) - oracle.delay(d[1].vertex, ra, dec))
    assert gap == pytest.approx(base, rel=1e-12)
