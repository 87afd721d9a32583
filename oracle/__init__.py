"""FP64 CPU oracle of the batched TaylorF2 likelihood -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its Python
binding) never imports, links or calls it, and the two share no code.

The arithmetic lives in ``gw_oracle.c`` (plain C, no fast-math, no FMA
contraction, Neumaier-compensated sums); this module compiles it with gcc into
``liboracle.so`` next to the source and wraps it with ctypes.  Every function
states the passage of arXiv:1904.02863 or of the cited literature it follows
in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared"]

_lib = None


def build(force: bool = False) -> str:
    """Compile gw_oracle.c with gcc (no-op when the library is newer than the
    source unless `force`)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        p = ctypes.c_void_p
        lib.oracle_pn_coefficients.argtypes = [d, p, p]
        lib.oracle_pn_spin_terms.argtypes = [d, d, d, d, p, p]
        lib.oracle_pn_phase.argtypes = [d, d, d]
        lib.oracle_pn_phase.restype = d
        lib.oracle_antenna.argtypes = [p, d, d, d, p, p]
        lib.oracle_delay.argtypes = [p, d, d]
        lib.oracle_delay.restype = d
        lib.oracle_waveform.argtypes = [d, d, i64, i32, p, p, p, i32, i64, i32, p]
        lib.oracle_waveform_at.argtypes = [p, i64, i32, p, p, p, i32, i64, p]
        lib.oracle_lnl.argtypes = [d, d, i64, i32, p, p, p, p, p, i32, i64, i32, i32, p, i32]
        lib.oracle_max_threads.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def pn_coefficients(eta: float) -> tuple[np.ndarray, np.ndarray]:
    """TaylorF2 coefficients (phi_k, phi_k^l), k = 0..7, at symmetric mass ratio eta."""
    phi, phil = np.zeros(8), np.zeros(8)
    _load().oracle_pn_coefficients(float(eta), _ptr(phi), _ptr(phil))
    return phi, phil


def pn_spin_terms(eta: float, delta: float, chi1: float, chi2: float) -> tuple[np.ndarray, np.ndarray]:
    """Aligned-spin additions to (phi_k, phi_k^l), k = 0..7, for symmetric mass
    ratio eta, delta = (m1 - m2)/M and spins chi1 (heavier body), chi2."""
    phi, phil = np.zeros(8), np.zeros(8)
    _load().oracle_pn_spin_terms(float(eta), float(delta), float(chi1), float(chi2), _ptr(phi), _ptr(phil))
    return phi, phil


def pn_phase(mc: float, q: float, f) -> np.ndarray:
    """Post-Newtonian part of the TaylorF2 phase at frequencies f."""
    lib = _load()
    return np.array([lib.oracle_pn_phase(float(mc), float(q), float(x)) for x in np.atleast_1d(f)])


def antenna(tensor, ra: float, dec: float, psi: float) -> tuple[float, float]:
    """(F+, Fx) of a detector tensor for a source at (ra, dec) with polarisation psi."""
    t = _f64(tensor).reshape(9)
    fp, fx = ctypes.c_double(), ctypes.c_double()
    _load().oracle_antenna(_ptr(t), float(ra), float(dec), float(psi), ctypes.byref(fp), ctypes.byref(fx))
    return fp.value, fx.value


def delay(vertex, ra: float, dec: float) -> float:
    """Arrival time at the detector vertex minus arrival time at the geocentre (s)."""
    return _load().oracle_delay(_ptr(_f64(vertex).reshape(3)), float(ra), float(dec))


def _det_arrays(tensors, vertices, n_det):
    if n_det == 0:
        return np.zeros(9), np.zeros(3)
    t = _f64(tensors).reshape(n_det, 9)
    v = _f64(vertices).reshape(n_det, 3)
    return t, v


def waveform(f_low: float, delta_f: float, n_bins: int, tensors, vertices, theta, isco: bool = False) -> np.ndarray:
    """Detector responses, shape (S, n_det, M) complex128; with tensors None,
    the polarisations (S, 2, M) instead.  isco: zero above each template's
    innermost-stable-circular-orbit frequency."""
    th = _f64(np.atleast_2d(theta))
    n_det = 0 if tensors is None else np.asarray(tensors).reshape(-1, 9).shape[0]
    t, v = _det_arrays(tensors, vertices, n_det)
    n_out = n_det if n_det else 2
    out = np.empty((th.shape[0], n_out, int(n_bins)), dtype=np.complex128)
    rc = _load().oracle_waveform(float(f_low), float(delta_f), int(n_bins), n_det, _ptr(t), _ptr(v),
                                 _ptr(th), th.shape[1], th.shape[0], int(bool(isco)), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_waveform rejected its arguments")
    return out


def waveform_at(freqs, tensors, vertices, theta) -> np.ndarray:
    """Detector responses at an arbitrary list of frequencies, shape
    (S, n_det, len(freqs)) complex128 (no template end)."""
    th = _f64(np.atleast_2d(theta))
    fr = _f64(np.atleast_1d(freqs))
    n_det = np.asarray(tensors).reshape(-1, 9).shape[0]
    t, v = _det_arrays(tensors, vertices, n_det)
    out = np.empty((th.shape[0], n_det, fr.size), dtype=np.complex128)
    rc = _load().oracle_waveform_at(_ptr(fr), fr.size, n_det, _ptr(t), _ptr(v), _ptr(th), th.shape[1],
                                    th.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("oracle_waveform_at rejected its arguments")
    return out


def lnl(f_low: float, delta_f: float, n_bins: int, tensors, vertices, data, psd, theta,
        n_threads: int = 0, isco: bool = False, add_norm: bool = False) -> np.ndarray:
    """lnL = -2 delta_f sum_d sum_k |d - h|^2 / S for every row of theta
    (templates ended at f_isco with `isco`; plus -sum ln(2 pi S) with
    `add_norm`)."""
    th = _f64(np.atleast_2d(theta))
    n_det = np.asarray(tensors).reshape(-1, 9).shape[0]
    t, v = _det_arrays(tensors, vertices, n_det)
    dat = np.ascontiguousarray(data, dtype=np.complex128).reshape(n_det, int(n_bins))
    s = _f64(psd).reshape(n_det, int(n_bins))
    out = np.empty(th.shape[0])
    rc = _load().oracle_lnl(float(f_low), float(delta_f), int(n_bins), n_det, _ptr(t), _ptr(v), _ptr(dat),
                            _ptr(s), _ptr(th), th.shape[1], th.shape[0], int(bool(isco)), int(bool(add_norm)),
                            _ptr(out), int(n_threads))
    if rc != 0:
        raise ValueError("oracle_lnl rejected its arguments")
    return out


def max_threads() -> int:
    """Threads an OpenMP region of the oracle uses by default."""
    return _load().oracle_max_threads()


def workload_data(w) -> np.ndarray:
    """data = noise + detector response to the workload's injection, computed
    by this oracle (a synthetic-input helper for the tests)."""
    g = w.grid
    h = waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta_inj[None, :])[0]
    return np.ascontiguousarray(w.noise + h)
