// Device-side mathematics of the TaylorF2 likelihood kernels (gfx950, FP64).
//
// * gw_phasor_half: e^{-i Phi} from the half phase Phi/2.  Cody-Waite
//   reduction of Phi/2 by multiples of pi to |h| <= pi/2 (two-constant pi,
//   fused multiply-adds), polynomial sine and cosine of h, then the double
//   angle: cos Phi = 1 - 2 sin^2 h, -sin Phi = -2 sin h cos h.  Working on the
//   half angle removes the quadrant bookkeeping of a pi/2 reduction: every
//   step is a floating-point multiply-add, which is what the vector ALU issues
//   fastest.  Coefficients come from gen_sincos.py (worst absolute error of
//   the polynomials in double: 2.1e-16).
// * gw_pn_coefficients: the non-spinning TaylorF2 phase coefficients through
//   3.5PN, Buonanno, Iyer, Ochsner, Pan & Sathyaprakash, PRD 80, 084043 (2009),
//   Eq. (3.18), with the 2.5PN term written phi_5 (1 + 3 ln v) and the 3PN log
//   term -6848/21 ln v.  (The waveform model itself is named, not printed, in
//   Sec. II of arXiv:1904.02863.)
#pragma once

#include <hip/hip_runtime.h>

#define GW_PI 3.141592653589793
#define GW_PI_HI 3.141592653589793              // double nearest pi
#define GW_PI_LO 1.2246467991473532e-16         // pi - GW_PI_HI
#define GW_INV_PI 0.3183098861837907
#define GW_EULER_GAMMA 0.5772156649015329
#define GW_LN4 1.3862943611198906
#define GW_C_SI 299792458.0                     // m / s
#define GW_GM_SUN_SI 1.3271244e20               // m^3 s^-2, IAU 2015 B3 nominal solar mass parameter
#define GW_MPC_SI 3.0856775814913673e22         // m
#define GW_MSUN_S (GW_GM_SUN_SI / (GW_C_SI * GW_C_SI * GW_C_SI))   // solar mass in seconds
#define GW_MPC_S (GW_MPC_SI / GW_C_SI)                             // 1 Mpc / c in seconds

// sin h = h + h z S(z), z = h^2, |h| <= pi/2
#define GW_SIN_S0 -0.16666666666666666
#define GW_SIN_S1 0.008333333333333106
#define GW_SIN_S2 -0.0001984126984118389
#define GW_SIN_S3 2.7557319207506058e-06
#define GW_SIN_S4 -2.5052106585314903e-08
#define GW_SIN_S5 1.6058926918823753e-10
#define GW_SIN_S6 -7.642691997901776e-13
#define GW_SIN_S7 2.71829976216082e-15
// cos h = 1 + z C(z)
#define GW_COS_C0 -0.49999999999999983
#define GW_COS_C1 0.04166666666666432
#define GW_COS_C2 -0.0013888888888784095
#define GW_COS_C3 2.480158727891725e-05
#define GW_COS_C4 -2.7557316506299984e-07
#define GW_COS_C5 2.0876566876526882e-09
#define GW_COS_C6 -1.1463018651812344e-11
#define GW_COS_C7 4.6100912366850437e-14

// (re, im) = e^{-i Phi} given half = Phi / 2.
__device__ __forceinline__ void gw_phasor_half(double half, double &re, double &im)
{
    const double n = __builtin_rint(half * GW_INV_PI);
    double h = __builtin_fma(-n, GW_PI_HI, half);
    h = __builtin_fma(-n, GW_PI_LO, h);
    const double z = h * h;
    double s = GW_SIN_S7;
    s = __builtin_fma(s, z, GW_SIN_S6);
    s = __builtin_fma(s, z, GW_SIN_S5);
    s = __builtin_fma(s, z, GW_SIN_S4);
    s = __builtin_fma(s, z, GW_SIN_S3);
    s = __builtin_fma(s, z, GW_SIN_S2);
    s = __builtin_fma(s, z, GW_SIN_S1);
    s = __builtin_fma(s, z, GW_SIN_S0);
    s = __builtin_fma(h * z, s, h);
    double c = GW_COS_C7;
    c = __builtin_fma(c, z, GW_COS_C6);
    c = __builtin_fma(c, z, GW_COS_C5);
    c = __builtin_fma(c, z, GW_COS_C4);
    c = __builtin_fma(c, z, GW_COS_C3);
    c = __builtin_fma(c, z, GW_COS_C2);
    c = __builtin_fma(c, z, GW_COS_C1);
    c = __builtin_fma(c, z, GW_COS_C0);
    c = __builtin_fma(z, c, 1.0);
    const double m = -2.0 * s;
    re = __builtin_fma(m, s, 1.0);
    im = m * c;
}

// TaylorF2 coefficients phi[k], phi_log[k] (k = 0..7) at symmetric mass ratio eta.
__device__ __forceinline__ void gw_pn_coefficients(double eta, double phi[8], double phi_log[8])
{
    const double pi2 = GW_PI * GW_PI;
    const double eta2 = eta * eta;
    const double eta3 = eta2 * eta;
#pragma unroll
    for (int k = 0; k < 8; ++k) { phi[k] = 0.0; phi_log[k] = 0.0; }
    phi[0] = 1.0;
    phi[2] = 3715.0 / 756.0 + (55.0 / 9.0) * eta;
    phi[3] = -16.0 * GW_PI;
    phi[4] = 15293365.0 / 508032.0 + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * eta2;
    phi[5] = GW_PI * (38645.0 / 756.0 - (65.0 / 9.0) * eta);
    phi_log[5] = 3.0 * phi[5];
    phi[6] = 11583231236531.0 / 4694215680.0 - (640.0 / 3.0) * pi2 - (6848.0 / 21.0) * GW_EULER_GAMMA
           - (6848.0 / 21.0) * GW_LN4
           + (-15737765635.0 / 3048192.0 + (2255.0 / 12.0) * pi2) * eta
           + (76055.0 / 1728.0) * eta2 - (127825.0 / 1296.0) * eta3;
    phi_log[6] = -6848.0 / 21.0;
    phi[7] = GW_PI * (77096675.0 / 254016.0 + (378515.0 / 1512.0) * eta - (74045.0 / 756.0) * eta2);
}
