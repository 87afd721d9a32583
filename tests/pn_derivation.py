"""Independent derivation of the TaylorF2 phase from the post-Newtonian
binding energy E(v) and gravitational-wave flux F(v) (test helper).

The energy and flux of a non-spinning quasi-circular binary through 3.5PN are
those of Blanchet, Living Rev. Relativ. 17, 2 (2014), Eqs. (233) and (314),
with x = v^2 and the 3PN flux logarithm ln(16 x) = ln 16 + 2 ln v.  In the
stationary-phase approximation the frequency-domain phase obeys

    d^2 Psi / df^2 = 2 pi dt/df,    dt/dv = -(dE/dv) / F,    f = v^3 / (pi M),

so, with E = -(eta M v^2 / 2) eps(v) and F = (32/5) eta^2 v^10 Fl(v),

    d^2 Psi / df^2 = (5 pi^2 M^2 / (48 eta)) v^-11 R(v),
    R(v) = (2 eps + v eps') / (2 Fl)   re-expanded to relative order v^7.

Writing Psi = 3/(128 eta) sum_k (p_k + q_k ln v) v^(k-5) and applying
d/df = (pi M / (3 v^2)) d/dv twice term by term gives, with n = k - 5,

    p_k n (n-3) + q_k (2n - 3) = 40 r_k,     q_k n (n-3) = 40 r_k^l,

where R = sum_k (r_k + r_k^l ln v) v^k.  p_5 multiplies a constant phase and
is not fixed by the derivation (it is absorbed into phi_c).  Nothing here
uses the oracle's coefficient table.
"""
from __future__ import annotations

import functools

import sympy as sp

v, eta, ell = sp.symbols("v eta ell")
_R = sp.Rational
_pi, _gamma = sp.pi, sp.EulerGamma
ORDER = 8   # k = 0 .. 7 (3.5PN)


def _energy_coefficients():
    """eps(v) = sum e_k v^k (Blanchet 2014, Eq. 233)."""
    return {0: 1, 2: -_R(3, 4) - eta / 12, 4: -_R(27, 8) + _R(19, 8) * eta - eta ** 2 / 24,
            6: -_R(675, 64) + (_R(34445, 576) - _R(205, 96) * _pi ** 2) * eta
               - _R(155, 96) * eta ** 2 - _R(35, 5184) * eta ** 3}


def _flux_coefficients():
    """Fl(v) = sum F_k v^k with the 3PN log written through ell = ln v
    (Blanchet 2014, Eq. 314)."""
    return {0: 1, 1: 0, 2: -_R(1247, 336) - _R(35, 12) * eta, 3: 4 * _pi,
            4: -_R(44711, 9072) + _R(9271, 504) * eta + _R(65, 18) * eta ** 2,
            5: -(_R(8191, 672) + _R(583, 24) * eta) * _pi,
            6: (_R(6643739519, 69854400) + _R(16, 3) * _pi ** 2 - _R(1712, 105) * _gamma
                - _R(856, 105) * sp.log(16) + (-_R(134543, 7776) + _R(41, 48) * _pi ** 2) * eta
                - _R(94403, 3024) * eta ** 2 - _R(775, 324) * eta ** 3) - _R(1712, 105) * ell,
            7: (-_R(16285, 504) + _R(214745, 1728) * eta + _R(193385, 3024) * eta ** 2) * _pi}


@functools.lru_cache(maxsize=None)
def r_series():
    """(r_k, r_k^l), k = 0..7, as sympy expressions in eta."""
    e = _energy_coefficients()
    fl = _flux_coefficients()
    num = [0] * ORDER
    for k, c in e.items():
        num[k] = c * (1 + _R(k, 2))          # coefficient of v^k in (2 eps + v eps') / 2
    fc = [fl.get(k, 0) for k in range(ORDER)]
    inv = [0] * ORDER
    inv[0] = 1
    for k in range(1, ORDER):                 # power series of 1 / Fl
        inv[k] = sp.expand(-sum(fc[j] * inv[k - j] for j in range(1, k + 1)))
    r = [sp.expand(sum(num[j] * inv[k - j] for j in range(k + 1))) for k in range(ORDER)]
    return tuple(x.coeff(ell, 0) for x in r), tuple(x.coeff(ell, 1) for x in r)


@functools.lru_cache(maxsize=None)
def phase_coefficients():
    """(p, q): dicts k -> sympy expression in eta; p has no entry for k = 5."""
    rk, rl = r_series()
    p, q = {}, {}
    for k in range(ORDER):
        n = k - 5
        if k == 5:
            if sp.expand(rl[5]) != 0:
                raise AssertionError("unexpected ln v term at 2.5PN in R")
            q[5] = -40 * rk[5] / 3
            continue
        q[k] = 40 * rl[k] / (n * (n - 3))
        p[k] = (40 * rk[k] - q[k] * (2 * n - 3)) / (n * (n - 3))
    return p, q


def numeric_phase_coefficients(eta_value: float, digits: int = 30):
    """(p_k, q_k) evaluated at eta = eta_value (p[5] is None)."""
    p, q = phase_coefficients()
    pv = [None if k == 5 else float(sp.N(p[k].subs(eta, eta_value), digits)) for k in range(ORDER)]
    qv = [float(sp.N(sp.sympify(q[k]).subs(eta, eta_value), digits)) for k in range(ORDER)]
    return pv, qv


def numeric_r(eta_value: float):
    """(r_k, r_k^l) at eta = eta_value as floats."""
    rk, rl = r_series()
    return ([float(sp.N(sp.sympify(x).subs(eta, eta_value), 30)) for x in rk],
            [float(sp.N(sp.sympify(x).subs(eta, eta_value), 30)) for x in rl])


# ---------------------------------------------------------------- aligned spins
# Spin terms of the energy and flux for spins along the orbital angular
# momentum, with S_l = m1^2 chi1 + m2^2 chi2 and Sigma_l = M (m2 chi2 - m1 chi1)
# in units of M^2 (s and sig below), delta = (m1 - m2)/M and x1 = m1/M:
#  * spin-orbit energy at v^3, v^5, v^7 and flux at v^3, v^5, v^6 (tail),
#    v^7: Blanchet, Living Rev. Relativ. 17, 2 (2014), Eqs. (414)-(415);
#  * spin-spin (S1 S2) energy and flux at v^4: Kidder, PRD 52, 821 (1995),
#    for aligned spins S1.S2 - 3 (L.S1)(L.S2) = -2 S1 S2 and
#    -103 S1.S2 + 289 (L.S1)(L.S2) = 186 S1 S2.
x1, chi1, chi2 = sp.symbols("x1 chi1 chi2")


def _spin_energy_flux():
    x2 = 1 - x1
    eta_x = x1 * x2
    dl = x1 - x2
    s = x1 ** 2 * chi1 + x2 ** 2 * chi2
    sig = x2 * chi2 - x1 * chi1
    e = {k: sp.sympify(c).subs(eta, eta_x) for k, c in _energy_coefficients().items()}
    f = {k: sp.sympify(c).subs(eta, eta_x) for k, c in _flux_coefficients().items()}
    e[3] = _R(14, 3) * s + 2 * dl * sig
    e[5] = (11 - _R(61, 9) * eta_x) * s + dl * (3 - _R(10, 3) * eta_x) * sig
    e[7] = ((_R(135, 4) - _R(367, 4) * eta_x + _R(29, 12) * eta_x ** 2) * s
            + dl * (_R(27, 4) - 39 * eta_x + _R(5, 4) * eta_x ** 2) * sig)
    e[4] = e[4] - 2 * eta_x * chi1 * chi2
    f[3] = f[3] - (4 * s + _R(5, 4) * dl * sig)
    f[5] = f[5] + (-_R(9, 2) + _R(272, 9) * eta_x) * s + (-_R(13, 16) + _R(43, 4) * eta_x) * dl * sig
    f[6] = f[6] - 16 * _pi * s - _R(31, 6) * _pi * dl * sig
    f[7] = f[7] + ((_R(476645, 6804) + _R(6172, 189) * eta_x - _R(2810, 27) * eta_x ** 2) * s
                   + (_R(9535, 336) + _R(1849, 126) * eta_x - _R(1501, 36) * eta_x ** 2) * dl * sig)
    f[4] = f[4] + _R(31, 8) * eta_x * chi1 * chi2
    return e, f


def _phase_from(e, fl, order=ORDER):
    num = [0] * order
    for k, c in e.items():
        if k < order:
            num[k] = c * (1 + _R(k, 2))
    fc = [fl.get(k, 0) for k in range(order)]
    inv = [0] * order
    inv[0] = 1
    for k in range(1, order):
        inv[k] = sp.expand(-sum(fc[j] * inv[k - j] for j in range(1, k + 1)))
    r = [sp.expand(sum(num[j] * inv[k - j] for j in range(k + 1))) for k in range(order)]
    rk, rl = [x.coeff(ell, 0) for x in r], [x.coeff(ell, 1) for x in r]
    p, q = {}, {}
    for k in range(order):
        n = k - 5
        if k == 5:
            q[5] = -40 * rk[5] / 3
            continue
        q[k] = 40 * rl[k] / (n * (n - 3))
        p[k] = (40 * rk[k] - q[k] * (2 * n - 3)) / (n * (n - 3))
    return p, q


@functools.lru_cache(maxsize=None)
def spin_phase_coefficients():
    """(p, q) with aligned spins: sympy expressions in x1, chi1, chi2."""
    e, f = _spin_energy_flux()
    return _phase_from(e, f)


def spin_linear_term(k: int, x1_value, which: int = 1) -> float:
    """Coefficient of chi_which (the other spin zero) in p_k (k != 5) or in
    q_5 / 3 (the 2.5PN term, which appears as phi_5 (1 + 3 ln v))."""
    p, q = spin_phase_coefficients()
    expr = q[5] / 3 if k == 5 else p[k]
    ex = sp.expand(expr)
    own, other = (chi1, chi2) if which == 1 else (chi2, chi1)
    lin = ex.coeff(own, 1).subs(other, 0)
    return float(sp.N(lin.subs(x1, x1_value), 30))


def spin_spin_term(x1_value) -> float:
    """Coefficient of chi1 chi2 in p_4."""
    p, _ = spin_phase_coefficients()
    return float(sp.N(sp.expand(p[4]).coeff(chi1, 1).coeff(chi2, 1).subs(x1, x1_value), 30))


# Test-mass limit (m2 -> 0) around a Kerr black hole of spin a: the binding
# energy of circular equatorial orbits, E/mu = (1 - 2u + a u^(3/2)) /
# sqrt(1 - 3u + 2a u^(3/2)) - 1 with u = M/r and M omega = u^(3/2) / (1 + a
# u^(3/2)) (Bardeen, Press & Teukolsky 1972), expanded here exactly, and the
# flux of black-hole perturbation theory through v^6 (Tagoshi, Shibata, Tanaka
# & Sasaki 1996): the spin enters as -11/4 a v^3, +33/16 a^2 v^4,
# -59/16 a v^5 and -65/6 pi a v^6.
kerr_a = sp.symbols("kerr_a")


@functools.lru_cache(maxsize=None)
def kerr_energy_series(order: int = 8):
    """eps(v) = E / (-mu v^2 / 2) for the test mass, coefficients v^0..v^(order-1)."""
    w, y = sp.symbols("w y", positive=True)
    e_w = (1 - 2 * w ** 2 + kerr_a * w ** 3) / sp.sqrt(1 - 3 * w ** 2 + 2 * kerr_a * w ** 3) - 1
    w_y = y
    for _ in range(order + 2):       # w = y (1 + a w^3)^(1/3), iterated to the series order
        w_y = sp.series(y * (1 + kerr_a * w_y ** 3) ** _R(1, 3), y, 0, order + 2).removeO()
    e_y = sp.series(e_w.subs(w, w_y), y, 0, order + 2).removeO()
    eps = sp.expand(sp.simplify(e_y / (-y ** 2 / 2)))
    return {k: sp.expand(eps.coeff(y, k)) for k in range(order)}


def kerr_flux_spin_terms():
    return {3: -_R(11, 4) * kerr_a, 4: _R(33, 16) * kerr_a ** 2, 5: -_R(59, 16) * kerr_a,
            6: -_R(65, 6) * _pi * kerr_a}


def test_mass_self_spin_term() -> float:
    """Coefficient of a^2 in p_4 for the test mass around Kerr."""
    e = kerr_energy_series(5)
    f = {0: 1, 2: -_R(1247, 336), 3: 4 * _pi + kerr_flux_spin_terms()[3],
         4: -_R(44711, 9072) + kerr_flux_spin_terms()[4]}
    p, _ = _phase_from({k: e[k] for k in range(5)}, f, order=5)
    return float(sp.N(sp.expand(p[4]).coeff(kerr_a, 2), 30))
