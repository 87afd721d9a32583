"""Seeded synthetic inputs for the batched TaylorF2 likelihood.

This module is shared by the CPU oracle's tests, the HIP path's tests and the
benchmark.  It holds none of the method's arithmetic: no waveform, antenna
pattern, time delay or likelihood.  It only builds what the likelihood of
Eq. (cbclike) takes as *inputs*: the frequency grid, the noise power spectral
density S(f), detector geometry (tensor and vertex), Gaussian noise, and
parameter samples drawn from box priors.  Injected signals are added by the
caller with whichever waveform generator it is allowed to use.

Conventions (the readings are listed in the design notes):

* Frequency grid: f_k = f_low + k * delta_f, k = 0 .. M-1, both ends of
  [f_low, f_high] included, so M = (f_high - f_low) / delta_f + 1.  With
  delta_f = 1/T this is the paper's T of Eq. (cbclike) (Sec. III).
* Noise: n_k = sqrt(S_k / (4 delta_f)) * (N(0,1) + i N(0,1)), independent per
  bin and detector; then E|n_k|^2 = S_k / (2 delta_f) and each bin contributes
  -1 on average to Eq. (cbclike)'s exponent.
* Detectors: a spherical Earth, sites near the LIGO Hanford, LIGO Livingston
  and Virgo locations, x-arm azimuth drawn from the seed (measured from local
  north towards east), y-arm 90 degrees further, both in the local tangent
  plane; tensor D = (x x^T - y y^T) / 2.
* Parameter vector theta (one row per sample), in this column order:
  [Mc (solar masses, detector frame), q = m2/m1 <= 1, d_L (Mpc), phi_c (rad),
   t_c (s), RA (rad), Dec (rad), psi (rad), iota (rad)].
  Rows with 5 columns carry the first five only (an optimally oriented
  source); rows with 9 carry all of them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Root seed: every configuration draws from SeedSequence(ROOT_SEED + index).
ROOT_SEED = 1904_02863

EARTH_RADIUS_M = 6.371e6
# Geodetic sites (degrees): LIGO Hanford, LIGO Livingston, Virgo.
SITES_DEG = (
    ("H", 46.45, -119.41),
    ("L", 30.56, -90.77),
    ("V", 43.63, 10.50),
)

PARAM_NAMES = ("mc", "q", "dl", "phic", "tc", "ra", "dec", "psi", "iota")


@dataclasses.dataclass(frozen=True)
class Grid:
    f_low: float
    delta_f: float
    n_bins: int

    @property
    def f_high(self) -> float:
        return self.f_low + (self.n_bins - 1) * self.delta_f

    def frequencies(self) -> np.ndarray:
        k = np.arange(self.n_bins, dtype=np.float64)
        return self.f_low + k * self.delta_f


def make_grid(f_low: float, f_high: float, duration: float) -> Grid:
    """Grid of one segment of `duration` seconds: delta_f = 1/duration, both
    f_low and f_high are bins (they must lie on the grid)."""
    delta_f = 1.0 / duration
    span = (f_high - f_low) * duration
    n = int(round(span))
    if abs(span - n) > 1e-9 * max(1.0, span):
        raise ValueError("f_high - f_low is not a whole number of bins")
    return Grid(float(f_low), float(delta_f), n + 1)


def psd(f: np.ndarray) -> np.ndarray:
    """Analytic one-sided noise PSD used by every workload (1/Hz):
    S(f) = 1e-49 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)],
    x = f / 215 Hz.  Positive on (0, inf)."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return 1e-49 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))


@dataclasses.dataclass(frozen=True)
class Detector:
    name: str
    tensor: np.ndarray   # (3, 3) float64, symmetric, trace-free
    vertex: np.ndarray   # (3,) float64, metres, Earth-fixed


def detector_at(name: str, lat_deg: float, lon_deg: float, azimuth: float) -> Detector:
    """L-shaped detector at a geodetic site on a spherical Earth with its
    x-arm at `azimuth` (radians from north towards east)."""
    lat, lon = math.radians(lat_deg), math.radians(lon_deg)
    vertex = EARTH_RADIUS_M * np.array(
        [math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])
    east = np.array([-math.sin(lon), math.cos(lon), 0.0])
    north = np.array([-math.sin(lat) * math.cos(lon), -math.sin(lat) * math.sin(lon), math.cos(lat)])
    xarm = math.cos(azimuth) * north + math.sin(azimuth) * east
    yarm = -math.sin(azimuth) * north + math.cos(azimuth) * east
    tensor = 0.5 * (np.outer(xarm, xarm) - np.outer(yarm, yarm))
    return Detector(name, tensor, vertex)


def network(rng: np.random.Generator, n_det: int) -> list[Detector]:
    """The first `n_det` sites (n_det <= 8; sites repeat with fresh arm
    orientations beyond the third) with seeded arm azimuths."""
    if not 1 <= n_det <= 8:
        raise ValueError("n_det must be in 1..8")
    dets = []
    for i in range(n_det):
        name, lat, lon = SITES_DEG[i % len(SITES_DEG)]
        dets.append(detector_at(f"{name}{i // len(SITES_DEG) or ''}", lat, lon, rng.uniform(0.0, 2.0 * math.pi)))
    return dets


def stack_detectors(dets: list[Detector]) -> tuple[np.ndarray, np.ndarray]:
    """(n_det, 3, 3) tensors and (n_det, 3) vertices as contiguous float64."""
    return (np.ascontiguousarray(np.stack([d.tensor for d in dets]), dtype=np.float64),
            np.ascontiguousarray(np.stack([d.vertex for d in dets]), dtype=np.float64))


def noise(rng: np.random.Generator, psd_values: np.ndarray, delta_f: float) -> np.ndarray:
    """Complex Gaussian noise with per-component variance S / (4 delta_f)."""
    s = np.asarray(psd_values, dtype=np.float64)
    sigma = np.sqrt(s / (4.0 * delta_f))
    re = rng.standard_normal(s.shape)
    im = rng.standard_normal(s.shape)
    return sigma * (re + 1j * im)


@dataclasses.dataclass(frozen=True)
class Prior:
    """Box prior. Mc, q, d_L, phi_c, t_c, RA, psi uniform; Dec uniform in
    sin(Dec); iota uniform in cos(iota)."""
    mc: tuple[float, float] = (25.0, 35.0)
    q: tuple[float, float] = (0.5, 1.0)
    dl: tuple[float, float] = (400.0, 1000.0)
    tc: tuple[float, float] = (-0.1, 0.1)

    def sample(self, rng: np.random.Generator, n: int, n_param: int = 9) -> np.ndarray:
        if n_param not in (5, 9):
            raise ValueError("n_param must be 5 or 9")
        th = np.empty((n, n_param), dtype=np.float64)
        th[:, 0] = rng.uniform(*self.mc, n)
        th[:, 1] = rng.uniform(*self.q, n)
        th[:, 2] = rng.uniform(*self.dl, n)
        th[:, 3] = rng.uniform(0.0, 2.0 * math.pi, n)
        th[:, 4] = rng.uniform(*self.tc, n)
        if n_param == 9:
            th[:, 5] = rng.uniform(0.0, 2.0 * math.pi, n)
            th[:, 6] = np.arcsin(rng.uniform(-1.0, 1.0, n))
            th[:, 7] = rng.uniform(0.0, math.pi, n)
            th[:, 8] = np.arccos(rng.uniform(-1.0, 1.0, n))
        return th


def component_masses_to_mc_q(m1: np.ndarray, m2: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(m1, m2) -> (chirp mass, q = min/max).  Used to express the neutron
    star prior of the ragged workload in the theta columns."""
    lo, hi = np.minimum(m1, m2), np.maximum(m1, m2)
    mc = (lo * hi) ** 0.6 / (lo + hi) ** 0.2
    return mc, lo / hi


def seeds(index: int) -> dict[str, np.random.Generator]:
    """Independent generators {detectors, injection, noise, samples} of one
    workload, spawned from SeedSequence(ROOT_SEED + index)."""
    children = np.random.SeedSequence(ROOT_SEED + index).spawn(4)
    return {name: np.random.Generator(np.random.PCG64(ss))
            for name, ss in zip(("detectors", "injection", "noise", "samples"), children)}


@dataclasses.dataclass
class Workload:
    """Everything of one single-event workload except the injected signal.

    `noise` is (n_det, M) complex128; the caller forms data = noise + h(theta_inj).
    """
    name: str
    grid: Grid
    n_param: int
    tensors: np.ndarray      # (n_det, 3, 3)
    vertices: np.ndarray     # (n_det, 3)
    psd: np.ndarray          # (n_det, M)
    noise: np.ndarray        # (n_det, M) complex128
    theta_inj: np.ndarray    # (n_param,)
    theta: np.ndarray        # (S, n_param)

    @property
    def n_det(self) -> int:
        return self.tensors.shape[0]

    @property
    def n_samples(self) -> int:
        return self.theta.shape[0]


def _single_event(name: str, index: int, n_det: int, duration: float, f_low: float, f_high: float,
                  n_param: int, n_samples: int, prior: Prior) -> Workload:
    g = seeds(index)
    grid = make_grid(f_low, f_high, duration)
    dets = network(g["detectors"], n_det)
    tensors, vertices = stack_detectors(dets)
    f = grid.frequencies()
    s = np.ascontiguousarray(np.broadcast_to(psd(f), (n_det, grid.n_bins)))
    nz = np.ascontiguousarray(np.stack([noise(g["noise"], s[d], grid.delta_f) for d in range(n_det)]))
    inj = np.array([30.0, 0.8, 500.0, g["injection"].uniform(0.0, 2.0 * math.pi),
                    g["injection"].uniform(-0.1, 0.1)])
    if n_param == 9:
        ri = g["injection"]
        inj = np.concatenate([inj, [ri.uniform(0.0, 2.0 * math.pi), math.asin(ri.uniform(-1.0, 1.0)),
                                    ri.uniform(0.0, math.pi), math.acos(ri.uniform(-1.0, 1.0))]])
    theta = prior.sample(g["samples"], n_samples, n_param)
    return Workload(name, grid, n_param, tensors, vertices, s, nz, inj, theta)


def bbh_1det_4s(n_samples: int = 1000) -> Workload:
    """One detector, 4 s at 2048 Hz sampling, 20-1024 Hz, delta_f = 1/4 Hz
    (4017 bins), optimally oriented source (5 parameters)."""
    return _single_event("bbh-1det-4s", 0, 1, 4.0, 20.0, 1024.0, 5, n_samples, Prior())


def bbh_3det_128s(n_samples: int = 4096) -> Workload:
    """Three detectors, 128 s at 4096 Hz sampling, 20-2048 Hz,
    delta_f = 1/128 Hz (259,585 bins per detector), 9 parameters."""
    return _single_event("bbh-3det-128s", 1, 3, 128.0, 20.0, 2048.0, 9, n_samples, Prior())


def small_event(index: int, n_det: int, n_bins: int, n_samples: int, n_param: int = 9,
                f_low: float = 20.0, delta_f: float = 0.25) -> Workload:
    """Small seeded event for parity tests: any bin count, any detector count."""
    g = seeds(100 + index)
    grid = Grid(f_low, delta_f, n_bins)
    tensors, vertices = stack_detectors(network(g["detectors"], n_det))
    f = grid.frequencies()
    s = np.ascontiguousarray(np.broadcast_to(psd(f), (n_det, n_bins)))
    nz = np.ascontiguousarray(np.stack([noise(g["noise"], s[d], delta_f) for d in range(n_det)]))
    theta = Prior().sample(g["samples"], n_samples, n_param)
    inj = Prior().sample(g["injection"], 1, n_param)[0]
    return Workload(f"small-{index}", grid, n_param, tensors, vertices, s, nz, inj, theta)


@dataclasses.dataclass
class RaggedEvent:
    grid: Grid
    tensors: np.ndarray
    vertices: np.ndarray
    psd: np.ndarray
    noise: np.ndarray
    theta_inj: np.ndarray
    theta: np.ndarray


def bns_ragged(n_events: int = 256, n_samples: int = 512, index: int = 2,
               t_min: float = 8.0, t_max: float = 256.0) -> list[RaggedEvent]:
    """Neutron-star-like events of uneven duration: T_e = round(exp(U[ln t_min,
    ln t_max])) seconds, 20-2048 Hz, 3 detectors, m1, m2 ~ U[1, 2] solar
    masses, d_L ~ U[40, 200] Mpc, each with its own proposals."""
    g = seeds(index)
    dets = network(g["detectors"], 3)
    tensors, vertices = stack_detectors(dets)
    events = []
    for _ in range(n_events):
        dur = float(max(t_min, round(math.exp(g["samples"].uniform(math.log(t_min), math.log(t_max))))))
        grid = make_grid(20.0, 2048.0, dur)
        f = grid.frequencies()
        s = np.ascontiguousarray(np.broadcast_to(psd(f), (3, grid.n_bins)))
        nz = np.ascontiguousarray(np.stack([noise(g["noise"], s[d], grid.delta_f) for d in range(3)]))

        def draw(rng, n):
            m1 = rng.uniform(1.0, 2.0, n)
            m2 = rng.uniform(1.0, 2.0, n)
            mc, q = component_masses_to_mc_q(m1, m2)
            th = Prior(dl=(40.0, 200.0)).sample(rng, n, 9)
            th[:, 0], th[:, 1] = mc, q
            return th
        inj = draw(g["injection"], 1)[0]
        theta = draw(g["samples"], n_samples)
        events.append(RaggedEvent(grid, tensors, vertices, s, nz, inj, theta))
    return events


def population_samples(n_events: int, n_per_event: int, index: int = 5) -> np.ndarray:
    """Stand-in posterior samples for population studies: [7, n_events, n]
    with fields m1, q, a1, a2, cos t1, cos t2, ln p(theta | 0).

    Each event has a true (m1, q, a1, a2, cos t1, cos t2): m1 log-uniform in
    [8, 60] solar masses, q U[0.3, 1], a U[0, 1], cos t U[-1, 1].  Its samples
    scatter around the truth with measurement-like widths (m1 10-25%,
    q 0.15, a 0.25, cos t 0.5), kept inside the support of the sampling prior
    (uniform in m1 on [2, 100], in q on [0.05, 1], in a on [0, 1], in cos t on
    [-1, 1]) by redrawing; ln p(theta | 0) is that prior's log density."""
    g = seeds(index)
    rng = g["samples"]
    truth = g["injection"]
    m1_t = np.exp(truth.uniform(math.log(8.0), math.log(60.0), n_events))
    q_t = truth.uniform(0.3, 1.0, n_events)
    a_t = truth.uniform(0.0, 1.0, (2, n_events))
    c_t = truth.uniform(-1.0, 1.0, (2, n_events))
    rel = truth.uniform(0.10, 0.25, n_events)
    lo = np.array([2.0, 0.05, 0.0, 0.0, -1.0, -1.0])
    hi = np.array([100.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    centre = np.stack([m1_t, q_t, a_t[0], a_t[1], c_t[0], c_t[1]])          # [6, events]
    width = np.stack([rel * m1_t, np.full(n_events, 0.15), np.full(n_events, 0.25), np.full(n_events, 0.25),
                      np.full(n_events, 0.5), np.full(n_events, 0.5)])
    out = np.empty((7, n_events, n_per_event))
    for f in range(6):
        x = centre[f][:, None] + width[f][:, None] * rng.standard_normal((n_events, n_per_event))
        bad = (x < lo[f]) | (x > hi[f])
        while bad.any():
            x[bad] = (np.broadcast_to(centre[f][:, None], x.shape)[bad]
                      + np.broadcast_to(width[f][:, None], x.shape)[bad] * rng.standard_normal(int(bad.sum())))
            bad = (x < lo[f]) | (x > hi[f])
        out[f] = x
    out[6] = -float(np.log(hi - lo).sum())
    return out


def long_bns(f_low: float, duration: float, n_det: int, n_samples: int, index: int = 6) -> Workload:
    """A long neutron-star event: f_low .. 2048 Hz in `duration` seconds
    (15 Hz / 512 s: 1,040,897 bins; 10 Hz / 2048 s: 4,173,825; 5 Hz / 8192 s:
    16,736,257), m1, m2 ~ U[1, 2] solar masses, d_L ~ U[40, 200] Mpc, the
    coalescence time within +-0.1 s of the segment's reference time."""
    g = seeds(index)
    grid = make_grid(f_low, 2048.0, duration)
    tensors, vertices = stack_detectors(network(g["detectors"], n_det))
    f = grid.frequencies()
    s = np.ascontiguousarray(np.broadcast_to(psd(f), (n_det, grid.n_bins)))
    nz = np.ascontiguousarray(np.stack([noise(g["noise"], s[d], grid.delta_f) for d in range(n_det)]))

    def draw(rng, n):
        m1 = rng.uniform(1.0, 2.0, n)
        m2 = rng.uniform(1.0, 2.0, n)
        mc, q = component_masses_to_mc_q(m1, m2)
        th = Prior(dl=(40.0, 200.0)).sample(rng, n, 9)
        th[:, 0], th[:, 1] = mc, q
        return th
    inj = draw(g["injection"], 1)[0]
    theta = draw(g["samples"], n_samples)
    return Workload(f"bns-{f_low:g}hz-{duration:g}s", grid, 9, tensors, vertices, s, nz, inj, theta)


def near_fiducial(theta0: np.ndarray, n_samples: int, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """Parameter rows scattered around theta0 the way a binary-neutron-star
    posterior is (the regime of relative binning): chirp mass to ~1e-5
    relative, q +-0.05 (kept in (0, 1]), d_L +-10 %, phi_c +-0.3 rad, t_c
    +-0.3 ms, sky position +-0.02 rad, psi and iota +-0.1 rad; `scale`
    widens or narrows every spread."""
    th = np.repeat(np.asarray(theta0, dtype=np.float64)[None], n_samples, axis=0)
    z = rng.standard_normal((n_samples, th.shape[1]))
    spread = np.array([1e-5 * th[0, 0], 0.05, 0.1 * th[0, 2], 0.3, 3e-4, 0.02, 0.02, 0.1, 0.1])[:th.shape[1]]
    th = th + scale * spread * z
    th[:, 1] = np.minimum(np.abs(th[:, 1]), 1.0)
    return th


def relbin_bns(f_low: float, duration: float, n_det: int, n_samples: int, index: int = 7) -> Workload:
    """A neutron-star event for relative binning: the grid, noise and
    detectors of `long_bns` (f_low .. 2048 Hz), an injection with m1, m2 in
    [1.2, 1.6] solar masses at 100 Mpc, and rows near the injection
    (`near_fiducial`).  Callers that want a given SNR scale the distance of
    the injection and of every row with `scale_distance`."""
    g = seeds(index)
    grid = make_grid(f_low, 2048.0, duration)
    tensors, vertices = stack_detectors(network(g["detectors"], n_det))
    f = grid.frequencies()
    s = np.ascontiguousarray(np.broadcast_to(psd(f), (n_det, grid.n_bins)))
    nz = np.ascontiguousarray(np.stack([noise(g["noise"], s[d], grid.delta_f) for d in range(n_det)]))
    rng = g["injection"]
    m1, m2 = rng.uniform(1.2, 1.6, 2)
    mc, q = component_masses_to_mc_q(np.array([m1]), np.array([m2]))
    inj = Prior(dl=(100.0, 100.0)).sample(rng, 1, 9)[0]
    inj[0], inj[1] = mc[0], q[0]
    theta = near_fiducial(inj, n_samples, g["samples"])
    return Workload(f"bns-relbin-{f_low:g}hz-{duration:g}s", grid, 9, tensors, vertices, s, nz, inj, theta)


def scale_distance(w: Workload, factor: float) -> Workload:
    """The same workload with the luminosity distance of the injection and of
    every row multiplied by `factor` (the signal amplitude scales as 1/d_L)."""
    inj = w.theta_inj.copy()
    th = w.theta.copy()
    inj[2] *= factor
    th[:, 2] *= factor
    return dataclasses.replace(w, theta_inj=inj, theta=th)


def add_spins(theta: np.ndarray, rng: np.random.Generator, bound: float = 1.0) -> np.ndarray:
    """theta with two aligned-spin columns chi1, chi2 ~ U[-bound, bound]
    appended (5 -> 7 or 9 -> 11 parameters)."""
    th = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    return np.hstack([th, rng.uniform(-bound, bound, (th.shape[0], 2))])
