"""Generates the polynomial coefficients of the device sine/cosine in
gw_device_math.h (run:  python paper_1904_02863_amd/csrc/gen_sincos.py).

Method: the classic argument-reduction-plus-polynomial scheme (Cody & Waite,
Software Manual for the Elementary Functions, 1980).  The kernels only ever
need e^{-i Phi} for a phase Phi reduced to h = Phi/2 - n pi, |h| <= pi/2, and
rebuild e^{-i Phi} from the half angle with cos Phi = 1 - 2 sin^2 h and
sin Phi = 2 sin h cos h.  On |h| <= pi/2, with z = h^2:

    sin h = h + h z S(z),   S of degree 7  (odd polynomial of degree 17)
    cos h = 1 + z C(z),     C of degree 7  (even polynomial of degree 16)

S and C are fitted by weighted least squares on Chebyshev nodes in 60-digit
arithmetic (the weights h^3 and h^2 make the fit minimise the absolute error
of sin and cos), which lands within a small factor of the minimax error; the
script then evaluates the double-precision Horner scheme exactly as the
kernels do and reports its worst absolute error against mpmath.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 60
HALF_PI = mp.pi / 2
DEG = 7
NODES = 400


def fit(target, weight):
    zmax = HALF_PI ** 2
    zs = [zmax * (1 - mp.cos(mp.pi * (j + mp.mpf(0.5)) / NODES)) / 2 for j in range(NODES)]
    a = mp.matrix(NODES, DEG + 1)
    b = mp.matrix(NODES, 1)
    for i, z in enumerate(zs):
        w = weight(z)
        for k in range(DEG + 1):
            a[i, k] = w * z ** k
        b[i] = w * target(z)
    q, r = mp.qr(a)
    coef = mp.lu_solve(r[:DEG + 1, :DEG + 1], (q.T * b)[:DEG + 1, 0])
    return [coef[k] for k in range(DEG + 1)]


def s_true(z):
    h = mp.sqrt(z)
    return (mp.sin(h) - h) / (h * z) if z > 0 else mp.mpf(-1) / 6


def c_true(z):
    h = mp.sqrt(z)
    return (mp.cos(h) - 1) / z if z > 0 else mp.mpf(-1) / 2


def main():
    s = fit(s_true, lambda z: z ** mp.mpf(1.5))
    c = fit(c_true, lambda z: z)
    sd = [float(x) for x in s]
    cd = [float(x) for x in c]
    hs = np.linspace(-float(HALF_PI), float(HALF_PI), 20001)
    worst_s = worst_c = 0.0
    for h in hs:
        z = h * h
        p = sd[DEG]
        for k in range(DEG - 1, -1, -1):
            p = p * z + sd[k]      # the kernels use fma; the error bound is of the same size
        sv = h + (h * z) * p
        p = cd[DEG]
        for k in range(DEG - 1, -1, -1):
            p = p * z + cd[k]
        cv = 1.0 + z * p
        worst_s = max(worst_s, abs(float(mp.sin(h) - sv)))
        worst_c = max(worst_c, abs(float(mp.cos(h) - cv)))
    print("// sin h = h + h z S(z), S coefficients z^0 .. z^7")
    for k, x in enumerate(sd):
        print(f"#define GW_SIN_S{k} {x!r}")
    print("// cos h = 1 + z C(z), C coefficients z^0 .. z^7")
    for k, x in enumerate(cd):
        print(f"#define GW_COS_C{k} {x!r}")
    print(f"// worst absolute error in double: sin {worst_s:.3e}, cos {worst_c:.3e}")


if __name__ == "__main__":
    main()
