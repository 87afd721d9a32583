"""Convergence diagnostics of many parallel chains (host side, numpy/scipy).

* Effective sample size: rank-normalised split-chain bulk ESS of Vehtari,
  Gelman, Simpson, Carpenter & Buerkner, "Rank-normalization, folding, and
  localization: an improved R-hat", Bayesian Analysis 16 (2021): draws are
  split in half per chain, replaced by normal scores of their pooled ranks, and
  the ESS follows from the multi-chain autocorrelation with Geyer's initial
  monotone positive-sequence truncation.
* Two-sample Kolmogorov-Smirnov test per marginal (scipy).
"""
from __future__ import annotations

import numpy as np
from scipy import special, stats


def _rank_normalise(x: np.ndarray) -> np.ndarray:
    """Normal scores of the pooled (average) ranks: Phi^-1((r - 3/8) / (S + 1/4))."""
    flat = x.ravel()
    r = stats.rankdata(flat, method="average").reshape(x.shape)
    return special.ndtri((r - 0.375) / (flat.size + 0.25))


def _autocov(x: np.ndarray) -> np.ndarray:
    """Autocovariance of each row at every lag (FFT), biased estimator."""
    m, n = x.shape
    xc = x - x.mean(axis=1, keepdims=True)
    size = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(xc, size, axis=1)
    return np.fft.irfft(f * np.conj(f), size, axis=1)[:, :n] / n


def ess(chains: np.ndarray) -> float:
    """Bulk ESS of one parameter from draws [n_chains, n_draws]."""
    x = np.asarray(chains, dtype=np.float64)
    m, n = x.shape
    half = n // 2
    x = np.concatenate([x[:, :half], x[:, n - half:]], axis=0)     # split chains
    x = _rank_normalise(x)
    m, n = x.shape
    acov = _autocov(x)
    chain_mean = x.mean(axis=1)
    w = acov[:, 0].mean() * n / (n - 1.0)
    b = n * chain_mean.var(ddof=1) if m > 1 else 0.0
    var_plus = (n - 1.0) / n * w + b / n
    if var_plus <= 0:
        return float(m * n)
    rho = 1.0 - (w - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: sums of adjacent pairs, positive and non-increasing
    tau = -1.0
    prev = np.inf
    for t in range(0, n - 1, 2):
        p = rho[t] + rho[t + 1]
        if p < 0:
            break
        p = min(p, prev)
        prev = p
        tau += 2.0 * p
    return float(m * n / max(tau, 1.0 / np.log10(m * n)))


def min_ess(draws: np.ndarray) -> tuple[float, np.ndarray]:
    """draws [n_chains, n_draws, n_params] -> (min over parameters, per-parameter ESS)."""
    per = np.array([ess(draws[:, :, j]) for j in range(draws.shape[2])])
    return float(per.min()), per


def ks_pvalues(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Two-sample KS p-value per column of a [n, p] and b [m, p]."""
    return np.array([stats.ks_2samp(a[:, j], b[:, j]).pvalue for j in range(a.shape[1])])
