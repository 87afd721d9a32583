"""Chain diagnostics: the bulk ESS estimator recovers the closed-form
integrated autocorrelation time of AR(1) chains, tau = (1 + rho)/(1 - rho);
the KS helper separates equal and shifted samples."""
import numpy as np
import pytest

from paper_1904_02863_amd import diagnostics


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.8, 0.9])
def test_ess_of_ar1_chains(rho):
    rng = np.random.default_rng(int(rho * 100))
    m, n = 16, 4000
    x = np.empty((m, n))
    x[:, 0] = rng.standard_normal(m) / np.sqrt(1 - rho ** 2)
    e = rng.standard_normal((m, n))
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    expected = m * n * (1 - rho) / (1 + rho)
    assert diagnostics.ess(x) == pytest.approx(expected, rel=0.1)


def test_min_ess_and_ks():
    rng = np.random.default_rng(3)
    draws = rng.standard_normal((8, 500, 3))
    draws[:, :, 2] = np.cumsum(draws[:, :, 2], axis=1) * 0.01     # a slowly mixing parameter
    low, per = diagnostics.min_ess(draws)
    assert low == per[2] and per[0] > 10 * per[2]
    a = rng.standard_normal((3000, 2))
    b = rng.standard_normal((3000, 2))
    b[:, 1] += 0.3
    p = diagnostics.ks_pvalues(a, b)
    assert p[0] > 1e-3 and p[1] < 1e-6
