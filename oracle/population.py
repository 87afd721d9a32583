"""FP64 CPU oracle of the population likelihood -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
use this module; the HIP library never imports or calls it.

What it computes: the recycled hierarchical likelihood of Eq. (poplike),
Sec. IV of arXiv:1904.02863 (Talbot, Smith, Thrane & Poole 2019), without
the rate and selection terms R^N e^{-R VT(Lambda)} (the paper leaves VT out
of its timings; R is a separate factor):

    ln L(Lambda) = sum_i ln[ (1/n_i) sum_j p(theta_ij | Lambda) / p(theta_ij | 0) ],

theta_ij the j-th posterior sample of event i drawn under the sampling prior
p(theta | 0).  The paper names, but does not print, the population models it
times (Sec. IV): the mass model of Talbot & Thrane (2018, ApJ 856, 173), the
spin-magnitude model of Wysocki et al. (2018) and the spin-orientation model
of Talbot & Thrane (2017, PRD 96, 023012).  This file writes them out as
follows (readings, each listed in the design notes):

* primary mass, a mixture of a power law and a Gaussian peak on
  [m_min, m_max] (the smoothing of the low-mass edge taken at zero width):
      p(m1) = (1 - lam) m1^-alpha / Z_pl + lam N(m1; mu_m, sigma_m) / Z_g,
      Z_pl = int_{m_min}^{m_max} m^-alpha dm,  Z_g the Gaussian mass in
      [m_min, m_max];
* mass ratio q = m2/m1 given m1, a power law on [m_min/m1, 1]:
      p(q | m1) = q^beta / int_{m_min/m1}^1 x^beta dx
  (zero at m1 = m_min, where that range is a single point);
* spin magnitudes a1, a2 independent, Beta(alpha_chi, beta_chi) on [0, 1];
* cosines of the spin tilts: a mixture of isotropic and a product of two
  Gaussians centred on aligned spins, each truncated to [-1, 1]:
      p(c1, c2) = (1 - xi)/4 + xi N_T(c1; 1, sigma_1) N_T(c2; 1, sigma_2).

Hyper-parameters outside their domain (m_min >= m_max, a width <= 0, a
mixing fraction outside [0, 1], alpha_chi or beta_chi <= 0) give -inf; any
non-finite hyper-parameter gives NaN.  An event whose samples all have zero
population density gives ln 0 = -inf.

Every integral above has a closed form; the code evaluates it with
scipy.special and plain numpy, sample by sample, in the order of the
equation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

# Order of the hyper-parameters in a row of `hyper`.
HYPER_NAMES = ("alpha", "beta", "mmin", "mmax", "lam", "mpp", "sigpp",
               "alpha_chi", "beta_chi", "xi", "sigma_1", "sigma_2")
# Order of the per-sample fields.
FIELD_NAMES = ("m1", "q", "a1", "a2", "cos_t1", "cos_t2", "ln_prior")


def _power_law_norm(alpha: float, lo: float, hi: float) -> float:
    """int_lo^hi m^-alpha dm."""
    if alpha == 1.0:
        return math.log(hi / lo)
    return (hi ** (1.0 - alpha) - lo ** (1.0 - alpha)) / (1.0 - alpha)


def _gauss_mass(mu: float, sigma: float, lo: float, hi: float) -> float:
    """Probability mass of N(mu, sigma) inside [lo, hi]."""
    return 0.5 * (special.erf((hi - mu) / (sigma * math.sqrt(2.0))) - special.erf((lo - mu) / (sigma * math.sqrt(2.0))))


def _normal_pdf(x, mu, sigma):
    return np.exp(-0.5 * ((x - mu) / sigma) ** 2) / (sigma * math.sqrt(2.0 * math.pi))


def hyper_valid(h) -> int:
    """1 evaluate, 0 out of domain (-inf), -1 non-finite (NaN)."""
    h = np.asarray(h, dtype=np.float64)
    if not np.isfinite(h).all():
        return -1
    alpha, beta, mmin, mmax, lam, mpp, sigpp, ach, bch, xi, s1, s2 = h
    if not (0.0 < mmin < mmax) or sigpp <= 0 or not (0.0 <= lam <= 1.0) or ach <= 0 or bch <= 0:
        return 0
    if not (0.0 <= xi <= 1.0) or s1 <= 0 or s2 <= 0:
        return 0
    return 1


def mass_density(m1, q, h):
    """p(m1 | Lambda) p(q | m1, Lambda) for arrays m1, q."""
    alpha, beta, mmin, mmax, lam, mpp, sigpp = h[:7]
    m1 = np.asarray(m1, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    inside = (m1 >= mmin) & (m1 <= mmax)
    m1s = np.where(inside, m1, mmin)
    p_pl = m1s ** (-alpha) / _power_law_norm(alpha, mmin, mmax)
    p_g = _normal_pdf(m1s, mpp, sigpp) / _gauss_mass(mpp, sigpp, mmin, mmax)
    p_m1 = np.where(inside, (1.0 - lam) * p_pl + lam * p_g, 0.0)
    qmin = mmin / m1s
    # at m1 = m_min the mass-ratio range shrinks to the point q = 1 (zero density)
    q_ok = inside & (m1s > mmin) & (q >= qmin) & (q <= 1.0)
    qs = np.where(q_ok, q, 1.0)
    qm = np.where(q_ok, qmin, 0.5)
    if beta == -1.0:
        zq = -np.log(qm)
    else:
        zq = (1.0 - qm ** (1.0 + beta)) / (1.0 + beta)
    p_q = np.where(q_ok, qs ** beta / zq, 0.0)
    return p_m1 * p_q


def spin_magnitude_density(a, h):
    """Beta(alpha_chi, beta_chi) density of a on [0, 1]."""
    ach, bch = h[7], h[8]
    a = np.asarray(a, dtype=np.float64)
    ok = (a >= 0.0) & (a <= 1.0)
    aa = np.where(ok, a, 0.5)
    ln_b = special.betaln(ach, bch)
    return np.where(ok, np.exp((ach - 1.0) * np.log(aa) + (bch - 1.0) * np.log1p(-aa) - ln_b), 0.0)


def spin_tilt_density(c1, c2, h):
    """(1 - xi)/4 + xi N_T(c1; 1, sigma_1) N_T(c2; 1, sigma_2) on [-1, 1]^2."""
    xi, s1, s2 = h[9], h[10], h[11]
    c1 = np.asarray(c1, dtype=np.float64)
    c2 = np.asarray(c2, dtype=np.float64)
    ok = (np.abs(c1) <= 1.0) & (np.abs(c2) <= 1.0)
    t1 = _normal_pdf(c1, 1.0, s1) / _gauss_mass(1.0, s1, -1.0, 1.0)
    t2 = _normal_pdf(c2, 1.0, s2) / _gauss_mass(1.0, s2, -1.0, 1.0)
    return np.where(ok, (1.0 - xi) / 4.0 + xi * t1 * t2, 0.0)


def population_density(fields, h):
    """p(theta | Lambda) for the fields m1, q, a1, a2, cos_t1, cos_t2 (arrays)."""
    m1, q, a1, a2, c1, c2 = fields[:6]
    return (mass_density(m1, q, h) * spin_magnitude_density(a1, h) * spin_magnitude_density(a2, h)
            * spin_tilt_density(c1, c2, h))


def lnl(samples, hyper) -> np.ndarray:
    """ln L(Lambda) of Eq. (poplike) for every row of hyper [K, 12].

    samples: [7, n_events, n_per_event] -- m1, q, a1, a2, cos_t1, cos_t2 and
    the log of the sampling prior density p(theta | 0) of each sample."""
    s = np.asarray(samples, dtype=np.float64)
    hyper = np.atleast_2d(np.asarray(hyper, dtype=np.float64))
    out = np.empty(hyper.shape[0])
    for k, h in enumerate(hyper):
        v = hyper_valid(h)
        if v < 0:
            out[k] = np.nan
            continue
        if v == 0:
            out[k] = -np.inf
            continue
        total = 0.0
        for i in range(s.shape[1]):
            w = population_density(s[:6, i], h) / np.exp(s[6, i])
            mean = math.fsum(w.tolist()) / w.size
            total += math.log(mean) if mean > 0 else -math.inf
        out[k] = total
    return out
