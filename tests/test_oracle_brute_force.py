"""The oracle against a 50-digit brute force (mpmath) on grids of up to 16
bins, and property tests drawn across the prior box (hypothesis).

The brute force evaluates Eq. (cbclike) from the template formulas with
every phase coefficient taken from the exact sympy derivation of
tests/pn_derivation.py (energy balance, aligned-spin terms included), not
from the oracle's table; the 2.5PN constant is the reading phi_5 = q_5 / 3 of
the oracle (a constant phase otherwise absorbed into phi_c).  The antenna
pattern, delay and polarisations are written out again at 50 digits.  It
checks that the oracle's FP64 arithmetic reaches its formula to ~1e-12.

Property tests (hypothesis, rows across the prior box): d = h(theta0) gives
lnL(theta0) = 0 and lnL(theta) <= 0; the template scales as 1/d_L; phi_c
multiplies it by a pure phase; t_c shifts it by e^{-2 pi i f dt}; <h,h> does
not depend on t_c or phi_c.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import sympy as sp
from hypothesis import given, settings, strategies as st

import oracle
import pn_derivation as pnd
import synth

mp.mp.dps = 50
GM_SUN = mp.mpf("1.3271244e20")
C_SI = mp.mpf(299792458)
MPC = mp.mpf("3.0856775814913673e22")


def _coefficients(q, chi1, chi2):
    """(p_k, q_k) at 50 digits for mass ratio q and aligned spins, from the
    exact derivation: the non-spinning series plus the spin-orbit terms
    linear in each spin and the 2PN spin-spin terms."""
    q_exact = sp.Rational(repr(float(q)))     # the double's decimal value, exactly
    eta = q_exact / (1 + q_exact) ** 2
    x1 = 1 / (1 + q_exact)
    p, qq = pnd.phase_coefficients()
    sp_p, sp_q = pnd.spin_phase_coefficients()
    out_p, out_q = [], []
    for k in range(8):
        pk = qq[5] / 3 if k == 5 else p[k]
        base_p = sp.sympify(pk).subs(pnd.eta, eta)
        base_q = sp.sympify(qq[k]).subs(pnd.eta, eta)
        if chi1 != 0.0 or chi2 != 0.0:
            exp_p = sp.expand(sp_q[5] / 3 if k == 5 else sp_p[k])
            exp_q = sp.expand(sp_q[k])
            for which, chi in ((pnd.chi1, chi1), (pnd.chi2, chi2)):
                other = pnd.chi2 if which is pnd.chi1 else pnd.chi1
                c = sp.Rational(repr(float(chi)))
                base_p += exp_p.coeff(which, 1).subs(other, 0).subs(pnd.x1, x1) * c
                base_q += exp_q.coeff(which, 1).subs(other, 0).subs(pnd.x1, x1) * c
            if k == 4:
                c1, c2 = sp.Rational(repr(float(chi1))), sp.Rational(repr(float(chi2)))
                base_p += exp_p.coeff(pnd.chi1, 1).coeff(pnd.chi2, 1).subs(pnd.x1, x1) * c1 * c2
                # self-spin: x_i^2 times the test-mass Kerr value (pinned in test_oracle_spin)
                base_p += sp.Rational(-405, 8) * (x1 ** 2 * c1 ** 2 + (1 - x1) ** 2 * c2 ** 2)
        out_p.append(mp.mpf(str(sp.N(base_p, 60))))
        out_q.append(mp.mpf(str(sp.N(base_q, 60))))
    return out_p, out_q


def _response(th, tensor, vertex, f, coef):
    """Detector response at frequency f (50 digits); coef = _coefficients of the row."""
    mc, q, dl, phic, tc = (mp.mpf(repr(float(x))) for x in th[:5])
    ra, dec, psi, iota = (mp.mpf(repr(float(x))) for x in th[5:9])
    eta = q / (1 + q) ** 2
    msun_s = GM_SUN / C_SI ** 3
    mtot = mc * eta ** mp.mpf("-0.6") * msun_s
    pk, qk = coef
    v = mp.cbrt(mp.pi * mtot * f)
    series = sum((pk[k] + qk[k] * mp.log(v)) * v ** k for k in range(8))
    psi_f = 2 * mp.pi * f * tc - phic - mp.pi / 4 + 3 / (128 * eta * v ** 5) * series
    amp = mp.sqrt(mp.mpf(5) / 24) * mp.pi ** (-mp.mpf(2) / 3) * (mc * msun_s) ** (mp.mpf(5) / 6) \
        / (dl * MPC / C_SI) * f ** (-mp.mpf(7) / 6)
    ci = mp.cos(iota)
    hp = amp * (1 + ci * ci) / 2 * mp.expj(-psi_f)
    hx = -1j * amp * ci * mp.expj(-psi_f)
    n = [mp.cos(dec) * mp.cos(ra), mp.cos(dec) * mp.sin(ra), mp.sin(dec)]
    ea = [-mp.sin(ra), mp.cos(ra), mp.mpf(0)]
    ed = [-mp.sin(dec) * mp.cos(ra), -mp.sin(dec) * mp.sin(ra), mp.cos(dec)]
    x = [mp.cos(psi) * ea[i] + mp.sin(psi) * ed[i] for i in range(3)]
    y = [-mp.sin(psi) * ea[i] + mp.cos(psi) * ed[i] for i in range(3)]
    d = [[mp.mpf(repr(float(tensor[i][j]))) for j in range(3)] for i in range(3)]
    fp = sum(d[i][j] * (x[i] * x[j] - y[i] * y[j]) for i in range(3) for j in range(3))
    fx = sum(d[i][j] * (x[i] * y[j] + y[i] * x[j]) for i in range(3) for j in range(3))
    dt = -sum(n[i] * mp.mpf(repr(float(vertex[i]))) for i in range(3)) / C_SI
    return (fp * hp + fx * hx) * mp.expj(-2 * mp.pi * f * dt)


@pytest.mark.parametrize("f_low,delta_f,n_bins,spins", [(20.0, 0.25, 16, False), (300.0, 1.0 / 128, 9, True),
                                                        (1500.0, 0.25, 5, True), (41.0, 4.0, 1, False)])
def test_oracle_against_50_digit_brute_force(f_low, delta_f, n_bins, spins):
    w = synth.small_event(40, 3, n_bins, 3, 9, f_low=f_low, delta_f=delta_f)
    theta = synth.add_spins(w.theta, np.random.default_rng(2), 0.9) if spins else w.theta
    data = w.noise
    got_h = oracle.waveform(f_low, delta_f, n_bins, w.tensors, w.vertices, theta)
    got_l = oracle.lnl(f_low, delta_f, n_bins, w.tensors, w.vertices, data, w.psd, theta)
    for s, th in enumerate(theta):
        coef = _coefficients(th[1], *((th[9], th[10]) if len(th) == 11 else (0.0, 0.0)))
        total = mp.mpf(0)
        for d in range(3):
            for k in range(n_bins):
                f = mp.mpf(repr(float(f_low + k * delta_f)))
                h = _response(th, w.tensors[d], w.vertices[d], f, coef)
                g = got_h[s, d, k]
                assert abs(complex(h) - g) <= 1e-12 * abs(complex(h)), (s, d, k)
                r = mp.mpc(complex(data[d, k])) - h
                total += (r.real ** 2 + r.imag ** 2) / mp.mpf(repr(float(w.psd[d, k])))
        want = float(-2 * mp.mpf(repr(delta_f)) * total)
        assert got_l[s] == pytest.approx(want, rel=1e-12)


# ---------------------------------------------------------------- properties
BOX = dict(mc=(25.0, 35.0), q=(0.5, 1.0), dl=(400.0, 1000.0), phic=(0.0, 2 * math.pi), tc=(-0.1, 0.1),
           ra=(0.0, 2 * math.pi), sindec=(-1.0, 1.0), psi=(0.0, math.pi), cosiota=(-1.0, 1.0))
_W = synth.small_event(41, 3, 64, 1, 9)


def _row(u):
    v = {k: lo + (hi - lo) * x for (k, (lo, hi)), x in zip(BOX.items(), u)}
    return np.array([v["mc"], v["q"], v["dl"], v["phic"], v["tc"], v["ra"], math.asin(v["sindec"]), v["psi"],
                     math.acos(v["cosiota"])])


unit = st.lists(st.floats(0.0, 1.0), min_size=9, max_size=9)


def _h(th):
    g = _W.grid
    return oracle.waveform(g.f_low, g.delta_f, g.n_bins, _W.tensors, _W.vertices, np.atleast_2d(th))


@settings(max_examples=40, deadline=None)
@given(unit, unit)
def test_noise_free_data_peak_at_truth(u0, u1):
    g = _W.grid
    t0, t1 = _row(u0), _row(u1)
    data = _h(t0)[0]
    out = oracle.lnl(g.f_low, g.delta_f, g.n_bins, _W.tensors, _W.vertices, data, _W.psd, np.stack([t0, t1]))
    assert out[0] == 0.0
    assert out[1] <= 0.0


@settings(max_examples=40, deadline=None)
@given(unit, st.floats(0.25, 4.0), st.floats(-3.0, 3.0), st.floats(-0.05, 0.05))
def test_template_symmetries(u, scale, dphi, dtc):
    g = _W.grid
    t = _row(u)
    h = _h(t)[0]
    far = t.copy()
    far[2] *= scale
    np.testing.assert_allclose(_h(far)[0], h / scale, rtol=1e-13)
    rot = t.copy()
    rot[3] += dphi
    np.testing.assert_allclose(_h(rot)[0], h * np.exp(1j * dphi), rtol=1e-11, atol=1e-11 * np.abs(h).max())
    shift = t.copy()
    shift[4] += dtc
    f = g.f_low + np.arange(g.n_bins) * g.delta_f
    np.testing.assert_allclose(_h(shift)[0], h * np.exp(-2j * math.pi * f * dtc), rtol=1e-9,
                               atol=1e-9 * np.abs(h).max())
    power = lambda x: float(np.sum(np.abs(x) ** 2 / _W.psd))
    assert power(_h(rot)[0]) == pytest.approx(power(h), rel=1e-12)
    assert power(_h(shift)[0]) == pytest.approx(power(h), rel=1e-12)
