"""FP64 CPU oracle of the relative-binning likelihood -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
use this module; the HIP library never imports or calls it.

arXiv:1904.02863 (Sec. V, and the survey of earlier speed-ups in Sec. I)
names relative binning (Zackay, Dai & Venumadhav 2018, arXiv:1806.08792) as
the companion of GPU waveforms for long signals: a binary-neutron-star signal
needs only ~10^3 unevenly spaced frequencies, and no exponential over the full
grid is evaluated per sample.  The method, as written here:

* A fiducial template h0 (a good-fit parameter point theta0) is fixed once.
  The grid f_k = f_low + k df is cut into bins by edges e_0 = 0 < e_1 < ... <
  e_B = M - 1 (grid indices); bin b holds k in [e_b, e_{b+1}), the last bin
  also k = e_B.
* Within bin b the ratio r_det(f) = h_det(f; theta) / h0_det(f) is taken as
  linear, r0 + r1 (f - fm), with fm = (f_lo + f_hi)/2 the bin centre and
  r0 = (r(f_lo) + r(f_hi))/2, r1 = (r(f_hi) - r(f_lo)) / (f_hi - f_lo) from
  the ratio at the two edges, f_lo = f_{e_b}, f_hi = f_{e_{b+1}}.
* Summary data per detector and bin, with w_k = 4 df / S_k:
      A0 = sum w d conj(h0),  A1 = sum w d conj(h0) (f - fm),
      B0 = sum w |h0|^2,      B1 = sum w |h0|^2 (f - fm),  B2 = sum w |h0|^2 (f - fm)^2.
  Then <d, h> ~ Re sum_b [A0 conj(r0) + A1 conj(r1)] and
      <h, h> ~ sum_b [B0 |r0|^2 + 2 B1 Re(r0 conj(r1)) + B2 |r1|^2],
  and Eq. (cbclike) becomes lnL = <d,h> - <h,h>/2 - <d,d>/2, the last term
  exact (<d,d> = sum_det sum_k w |d|^2).
  Reading: the |r1|^2 B2 term, which Zackay et al. drop as second order, is
  kept, so that the estimate is exact whenever r is linear inside every bin
  (for instance with an edge at every grid bin).  With the Newtonian
  amplitude of this template |r| does not depend on f, so the B1 term
  vanishes up to rounding for every template; it is kept for generality.
* Bin edges (Zackay et al., Sec. III): a bound on how much the phase of a
  template near theta0 can differ from the fiducial one,
      dPsi(f) = 2 pi chi sum_i sgn(g_i) (f / f*_i)^g_i,
      g = (-5/3, -2/3, 1, 5/3, 7/3),  f*_i = f_min for g_i < 0, f_max otherwise
  (f_min, f_max the first and last grid frequency), is increasing in f; an
  edge is put at the first grid bin where dPsi has advanced by another eps
  since f_min, so that dPsi changes by at most eps across a bin.

Per-sample domain rules are those of the full likelihood: a non-finite
parameter gives NaN; Mc <= 0, q outside (0, 1] or dL <= 0 give -inf.
Templates are never ended at f_isco here (the ratio to a fiducial that has
ended would be undefined).
"""
from __future__ import annotations

import math

import numpy as np

from . import waveform, waveform_at

GAMMAS = (-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0)


def phase_bound(f, f_min: float, f_max: float, chi: float = 1.0) -> np.ndarray:
    """dPsi(f) of the edge rule (radians)."""
    f = np.asarray(f, dtype=np.float64)
    total = np.zeros_like(f)
    for g in GAMMAS:
        fstar = f_min if g < 0 else f_max
        total = total + math.copysign(1.0, g) * (f / fstar) ** g
    return 2.0 * math.pi * chi * total


def edges(f_low: float, delta_f: float, n_bins: int, chi: float = 1.0, eps: float = 0.5) -> np.ndarray:
    """Grid indices of the bin edges: 0, every k at which floor((dPsi(f_k) -
    dPsi(f_0)) / eps) steps up, and n_bins - 1."""
    if n_bins < 2 or not (eps > 0.0) or not (chi > 0.0):
        raise ValueError("need n_bins >= 2, eps > 0, chi > 0")
    k = np.arange(n_bins)
    f = f_low + k * delta_f
    psi = phase_bound(f, f[0], f[-1], chi)
    level = np.floor((psi - psi[0]) / eps)
    out = [0]
    for j in range(1, n_bins):
        if level[j] > level[j - 1]:
            out.append(j)
    if out[-1] != n_bins - 1:
        out.append(n_bins - 1)
    return np.array(out, dtype=np.int64)


def bin_ranges(e: np.ndarray):
    """(first, last) grid index of every bin; the last bin includes its upper edge."""
    B = len(e) - 1
    return [(int(e[b]), int(e[b + 1]) - (0 if b == B - 1 else 1)) for b in range(B)]


def summary(f_low: float, delta_f: float, n_bins: int, tensors, vertices, data, psd, theta0, e,
            add_norm: bool = False) -> dict:
    """Summary data of the fiducial theta0 for bin edges e.

    Returns A0, A1 (complex) and B0, B1, B2 (real), each [n_det, B]; dd =
    <d, d>; norm = sum ln(2 pi S) (0 unless add_norm); h0e = the fiducial
    responses at the edges [n_det, B + 1]; fe = the edge frequencies."""
    e = np.asarray(e, dtype=np.int64)
    n_det = np.asarray(tensors).reshape(-1, 9).shape[0]
    data = np.asarray(data, dtype=np.complex128).reshape(n_det, n_bins)
    psd = np.asarray(psd, dtype=np.float64).reshape(n_det, n_bins)
    if len(e) < 2 or e[0] != 0 or e[-1] != n_bins - 1 or np.any(np.diff(e) <= 0):
        raise ValueError("edges must rise strictly from 0 to n_bins - 1")
    h0 = waveform(f_low, delta_f, n_bins, tensors, vertices, np.atleast_2d(theta0))[0]
    f = f_low + np.arange(n_bins) * delta_f
    w = 4.0 * delta_f / psd
    B = len(e) - 1
    out = {k: np.zeros((n_det, B), dtype=np.complex128 if k in ("A0", "A1") else np.float64)
           for k in ("A0", "A1", "B0", "B1", "B2")}
    for b, (lo, hi) in enumerate(bin_ranges(e)):
        fm = 0.5 * (f[e[b]] + f[e[b + 1]])
        sl = slice(lo, hi + 1)
        x = f[sl] - fm
        for d in range(n_det):
            dh = w[d, sl] * data[d, sl] * np.conj(h0[d, sl])
            hh = w[d, sl] * np.abs(h0[d, sl]) ** 2
            out["A0"][d, b] = dh.sum()
            out["A1"][d, b] = (dh * x).sum()
            out["B0"][d, b] = hh.sum()
            out["B1"][d, b] = (hh * x).sum()
            out["B2"][d, b] = (hh * x * x).sum()
    out["dd"] = float(np.sum(w * np.abs(data) ** 2))
    out["norm"] = float(np.sum(np.log(2.0 * math.pi * psd))) if add_norm else 0.0
    out["fe"] = f[e]
    out["h0e"] = h0[:, e]
    return out


def lnl_from_ratio(summ: dict, r: np.ndarray) -> np.ndarray:
    """The estimate of lnL from the ratio r = h / h0 at the bin edges,
    r [S, n_det, B + 1] complex (the template enters only through r)."""
    fe = summ["fe"]
    df = fe[1:] - fe[:-1]
    r0 = 0.5 * (r[:, :, :-1] + r[:, :, 1:])
    r1 = (r[:, :, 1:] - r[:, :, :-1]) / df
    dh = np.real(summ["A0"][None] * np.conj(r0) + summ["A1"][None] * np.conj(r1)).sum(axis=(1, 2))
    hh = (summ["B0"][None] * np.abs(r0) ** 2 + 2.0 * summ["B1"][None] * np.real(r0 * np.conj(r1))
          + summ["B2"][None] * np.abs(r1) ** 2).sum(axis=(1, 2))
    return dh - 0.5 * hh - 0.5 * summ["dd"] - summ["norm"]


def lnl(summ: dict, tensors, vertices, theta) -> np.ndarray:
    """Relative-binning lnL of every row of theta from the summary data."""
    th = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    he = waveform_at(summ["fe"], tensors, vertices, th)                # [S, n_det, B + 1]
    out = lnl_from_ratio(summ, he / summ["h0e"][None])
    # domain rules of the full likelihood (the ratio of a NaN row is NaN already)
    for s, row in enumerate(th):
        if not np.isfinite(row).all():
            out[s] = np.nan
        elif not (row[0] > 0.0 and 0.0 < row[1] <= 1.0 and row[2] > 0.0):
            out[s] = -np.inf
    return out
