"""Generates the polynomial coefficients of the device sine/cosine in
gw_device_math.h (run:  python paper_1904_02863_amd/csrc/gen_sincos.py).

Method: argument reduction plus polynomials (Cody & Waite, Software Manual for
the Elementary Functions, 1980), applied to phases measured in turns.  The
kernels need e^{-i Phi} for Phi = 2 pi x; they take r = x - rint(x), which is
exact, so |r| <= 1/2 and e^{-i Phi} = e^{-2 pi i r}, and rebuild it from the
half angle pi r with cos 2 pi r = 1 - 2 sin^2 pi r, sin 2 pi r = 2 sin pi r cos pi r.
With z = r^2 the polynomials carry the double angle's factors:

    s2 = sqrt(2) sin(pi r)  = r P(z),               P of degree 7 (odd, degree 15)
    c2 = -sqrt(2) cos(pi r) = -sqrt(2) + z C(z),    C of degree 6 (even, degree 14)

so that cos 2 pi r = 1 - s2^2 (one FMA with a negated operand) and
-sin 2 pi r = s2 c2 (one multiply).

P and C are fitted by weighted least squares on Chebyshev nodes in 60-digit
arithmetic (weights r and r^2 make the fit minimise the absolute error of sin
and cos), which lands within a small factor of the minimax error; the script
then evaluates the double-precision Horner scheme exactly as the kernels do
and reports its worst absolute error against mpmath.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 60
RMAX = mp.mpf(1) / 2
SIN_DEG = 7
COS_DEG = 6
NODES = 400


def fit(target, weight, deg):
    zmax = RMAX ** 2
    zs = [zmax * (1 - mp.cos(mp.pi * (j + mp.mpf(0.5)) / NODES)) / 2 for j in range(NODES)]
    a = mp.matrix(NODES, deg + 1)
    b = mp.matrix(NODES, 1)
    for i, z in enumerate(zs):
        w = weight(z)
        for k in range(deg + 1):
            a[i, k] = w * z ** k
        b[i] = w * target(z)
    q, r = mp.qr(a)
    coef = mp.lu_solve(r[:deg + 1, :deg + 1], (q.T * b)[:deg + 1, 0])
    return [coef[k] for k in range(deg + 1)]


SQRT2 = mp.sqrt(2)


def p_true(z):
    r = mp.sqrt(z)
    return SQRT2 * mp.sin(mp.pi * r) / r if z > 0 else SQRT2 * mp.pi


def c_true(z):
    r = mp.sqrt(z)
    return SQRT2 * (1 - mp.cos(mp.pi * r)) / z if z > 0 else SQRT2 * mp.pi ** 2 / 2


def horner(coef, z):
    p = coef[-1]
    for c in reversed(coef[:-1]):
        p = p * z + c              # the kernels use fma; the error bound is of the same size
    return p


def main():
    p = [float(x) for x in fit(p_true, lambda z: mp.sqrt(z), SIN_DEG)]
    c = [float(x) for x in fit(c_true, lambda z: z, COS_DEG)]
    worst_s = worst_c = 0.0
    for r in np.linspace(-0.5, 0.5, 20001):
        z = r * r
        s2 = r * horner(p, z)
        c2 = -float(SQRT2) + z * horner(c, z)
        re = 1.0 - s2 * s2
        im = s2 * c2
        worst_s = max(worst_s, abs(float(mp.cos(2 * mp.pi * r) - re)))
        worst_c = max(worst_c, abs(float(-mp.sin(2 * mp.pi * r) - im)))
    print("// sqrt(2) sin(pi r) = r P(z), z = r^2, coefficients z^0 .. z^7")
    for k, x in enumerate(p):
        print(f"#define GW_SINPI_P{k} {x!r}")
    print("// -sqrt(2) cos(pi r) = -sqrt(2) + z C(z), coefficients z^0 .. z^6")
    for k, x in enumerate(c):
        print(f"#define GW_COSPI_C{k} {x!r}")
    print(f"#define GW_SQRT2 {float(SQRT2)!r}")
    print(f"// worst absolute error of e^(-2 pi i r) in double: re {worst_s:.3e}, im {worst_c:.3e}")


if __name__ == "__main__":
    main()
