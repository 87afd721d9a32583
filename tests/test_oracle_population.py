"""Pins of the population oracle (Eq. (poplike), Sec. IV).

* Each model factor integrates to one (adaptive quadrature).
* Special cases typed independently: a pure power law with beta = 0, a
  uniform spin magnitude (Beta(1, 1)), an isotropic tilt distribution
  (xi = 0); the Gaussian peak against scipy.stats.truncnorm; the spin
  magnitude against scipy.stats.beta.
* The importance-sampling identity behind the recycling: with samples drawn
  from p(theta | Lambda0) (independent scipy/numpy samplers) and that density
  as the sampling prior (written with scipy.stats), every weight at Lambda0 is
  1, so ln L(Lambda0) = 0; at another Lambda the mean weight is 1 within its
  Monte Carlo error, so ln L ~ 0 per event.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import population as pop

LAMBDA0 = np.array([2.3, 1.2, 6.0, 70.0, 0.15, 33.0, 4.0, 2.0, 5.0, 0.6, 0.5, 0.9])


def _independent_density(m1, q, a1, a2, c1, c2, h):
    """p(theta | Lambda) written with scipy.stats distributions."""
    alpha, beta, mmin, mmax, lam, mpp, sigpp, ach, bch, xi, s1, s2 = h
    pl_norm = (mmax ** (1 - alpha) - mmin ** (1 - alpha)) / (1 - alpha)
    tn = stats.truncnorm((mmin - mpp) / sigpp, (mmax - mpp) / sigpp, loc=mpp, scale=sigpp)
    in_m = (m1 >= mmin) & (m1 <= mmax)
    p_m1 = np.where(in_m, (1 - lam) * np.clip(m1, mmin, mmax) ** (-alpha) / pl_norm + lam * tn.pdf(m1), 0.0)
    lo = mmin / m1
    in_q = in_m & (q >= lo) & (q <= 1)
    p_q = np.where(in_q, (beta + 1) * q ** beta / (1 - lo ** (beta + 1)), 0.0)
    p_a = stats.beta(ach, bch).pdf(a1) * stats.beta(ach, bch).pdf(a2)
    t1 = stats.truncnorm(-2 / s1, 0.0, loc=1.0, scale=s1)
    t2 = stats.truncnorm(-2 / s2, 0.0, loc=1.0, scale=s2)
    p_t = (1 - xi) / 4 + xi * t1.pdf(c1) * t2.pdf(c2)
    return p_m1 * p_q * p_a * p_t


def _draw(rng, n, h):
    """Samples from p(theta | Lambda) by inverse CDFs and scipy samplers."""
    alpha, beta, mmin, mmax, lam, mpp, sigpp, ach, bch, xi, s1, s2 = h
    u = rng.uniform(size=n)
    a1 = 1 - alpha
    pl = (mmin ** a1 + u * (mmax ** a1 - mmin ** a1)) ** (1 / a1)
    tn = stats.truncnorm((mmin - mpp) / sigpp, (mmax - mpp) / sigpp, loc=mpp, scale=sigpp)
    peak = tn.rvs(size=n, random_state=rng)
    m1 = np.where(rng.uniform(size=n) < lam, peak, pl)
    lo = (mmin / m1) ** (beta + 1)
    q = (lo + rng.uniform(size=n) * (1 - lo)) ** (1 / (beta + 1))
    a_1 = rng.beta(ach, bch, n)
    a_2 = rng.beta(ach, bch, n)
    aligned = rng.uniform(size=n) < xi
    t1 = stats.truncnorm(-2 / s1, 0.0, loc=1.0, scale=s1).rvs(size=n, random_state=rng)
    t2 = stats.truncnorm(-2 / s2, 0.0, loc=1.0, scale=s2).rvs(size=n, random_state=rng)
    c1 = np.where(aligned, t1, rng.uniform(-1, 1, n))
    c2 = np.where(aligned, t2, rng.uniform(-1, 1, n))
    return np.stack([m1, q, a_1, a_2, c1, c2])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_each_factor_integrates_to_one(seed):
    rng = np.random.default_rng(seed)
    h = LAMBDA0 + rng.uniform(-0.3, 0.3, 12) * np.array([1, 1, 5, 40, 0.3, 20, 5, 3, 3, 1, 1, 1])
    h[4], h[9] = np.clip(h[4], 0, 1), np.clip(h[9], 0, 1)
    h[10], h[11] = abs(h[10]) + 0.1, abs(h[11]) + 0.1
    h[7], h[8] = abs(h[7]) + 0.5, abs(h[8]) + 0.5
    assert pop.hyper_valid(h) == 1
    mmin, mmax = h[2], h[3]
    mass, _ = integrate.dblquad(lambda q, m: pop.mass_density(m, q, h), mmin, mmax,
                                lambda m: mmin / m, lambda m: 1.0, epsabs=1e-11, epsrel=1e-10)
    assert mass == pytest.approx(1.0, rel=1e-8)
    spin, _ = integrate.quad(lambda a: pop.spin_magnitude_density(a, h), 0.0, 1.0, epsabs=1e-12)
    assert spin == pytest.approx(1.0, rel=1e-9)
    tilt, _ = integrate.dblquad(lambda c2, c1: pop.spin_tilt_density(c1, c2, h), -1, 1, -1, 1, epsabs=1e-12)
    assert tilt == pytest.approx(1.0, rel=1e-9)


def test_special_cases():
    h = np.array([2.0, 0.0, 5.0, 50.0, 0.0, 30.0, 3.0, 1.0, 1.0, 0.0, 0.5, 0.5])
    m1 = np.array([5.5, 10.0, 49.0])
    q = np.array([1.0, 0.6, 0.2])
    # pure power law alpha = 2 on [5, 50], flat q on [5/m1, 1]
    want = m1 ** -2 / (1 / 5 - 1 / 50) / (1 - 5 / m1)
    np.testing.assert_allclose(pop.mass_density(m1, q, h), want, rtol=1e-14)
    assert pop.mass_density(np.array([5.0]), np.array([1.0]), h)[0] == 0.0
    np.testing.assert_allclose(pop.spin_magnitude_density(np.array([0.1, 0.5, 0.99]), h), 1.0, rtol=1e-14)
    np.testing.assert_allclose(pop.spin_tilt_density(np.array([-0.9, 0.3]), np.array([0.0, 1.0]), h), 0.25)
    h2 = h.copy()
    h2[7], h2[8] = 2.0, 1.0     # Beta(2, 1) = 2 a
    np.testing.assert_allclose(pop.spin_magnitude_density(np.array([0.25, 0.75]), h2), [0.5, 1.5], rtol=1e-14)
    # outside the supports
    assert pop.mass_density(np.array([4.9, 51.0, 20.0]), np.array([0.5, 0.5, 0.2]), h).tolist() == [0.0, 0.0, 0.0]


def test_density_matches_scipy_distributions():
    rng = np.random.default_rng(5)
    x = _draw(rng, 2000, LAMBDA0)
    got = pop.population_density(x, LAMBDA0)
    want = _independent_density(*x, LAMBDA0)
    np.testing.assert_allclose(got, want, rtol=1e-11)


def test_recycling_identity():
    rng = np.random.default_rng(11)
    n_events, n = 6, 20000
    fields = np.stack([_draw(rng, n, LAMBDA0) for _ in range(n_events)], axis=1)   # [6, events, n]
    ln_prior = np.log(_independent_density(*fields, LAMBDA0))
    samples = np.concatenate([fields, ln_prior[None]], axis=0)
    assert abs(pop.lnl(samples, LAMBDA0)[0]) < 1e-11
    # another population: the mean weight of each event estimates
    # int p(theta | Lambda) dtheta = 1, within its Monte Carlo error
    h = LAMBDA0.copy()
    h[0], h[4], h[7], h[9] = 1.8, 0.3, 2.5, 0.4
    w = pop.population_density(fields, h) / np.exp(ln_prior)
    se = w.std(axis=1) / math.sqrt(n)
    assert np.all(np.abs(w.mean(axis=1) - 1.0) < 5 * se)
    assert pop.lnl(samples, h)[0] == pytest.approx(np.log(w.mean(axis=1)).sum(), abs=1e-12)


def test_domain_rules():
    s = np.zeros((7, 2, 3))
    s[0], s[1], s[2], s[3], s[4], s[5] = 30.0, 0.8, 0.3, 0.3, 0.5, 0.5
    assert np.isfinite(pop.lnl(s, LAMBDA0)[0])
    bad = [LAMBDA0.copy() for _ in range(5)]
    bad[0][2] = 80.0          # m_min > m_max
    bad[1][6] = 0.0           # zero peak width
    bad[2][4] = 1.5           # mixing fraction above 1
    bad[3][7] = -1.0          # alpha_chi <= 0
    bad[4][11] = np.nan
    out = pop.lnl(s, np.array(bad))
    assert out[:4].tolist() == [-np.inf] * 4 and np.isnan(out[4])
    s2 = s.copy()
    s2[0, 1] = 200.0          # every sample of event 1 above m_max
    assert pop.lnl(s2, LAMBDA0)[0] == -np.inf
