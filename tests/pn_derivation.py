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
