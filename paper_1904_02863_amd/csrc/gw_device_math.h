// Device-side mathematics of the TaylorF2 likelihood kernels (gfx950, FP64).
//
// * gw_phasor_turns: e^{-2 pi i x} for a phase x measured in turns.  The
//   reduction r = x - rint(x) is exact (|r| <= 1/2) and keeps the absolute
//   accuracy x already has; sin(pi r) and cos(pi r) come from polynomials in
//   r^2 and e^{-2 pi i r} from the double angle,
//   cos 2 pi r = 1 - 2 sin^2 pi r, -sin 2 pi r = -2 sin pi r cos pi r.
//   Working on the half angle removes the quadrant bookkeeping of a quarter-
//   turn reduction: every step is a floating-point multiply or multiply-add,
//   which the vector ALU issues at full rate.  The polynomials carry the
//   double angle's factors (sqrt(2) sin, -sqrt(2) cos), so the double angle
//   costs one FMA and one multiply.  Coefficients come from gen_sincos.py.
// * gw_phasor_table: the same phasor from a table of N = 2048 roots of unity
//   (each rounded once) and degree-3/4 polynomials of the remainder, at most
//   half a table step (14 operations instead of 20, and more accurate); the
//   phase comes in scaled by N and the hot loops keep the table in LDS.
// * gw_pn_coefficients: the non-spinning TaylorF2 phase coefficients through
//   3.5PN, Buonanno, Iyer, Ochsner, Pan & Sathyaprakash, PRD 80, 084043 (2009),
//   Eq. (3.18), with the 2.5PN term written phi_5 (1 + 3 ln v) and the 3PN log
//   term -6848/21 ln v.  (The waveform model itself is named, not printed, in
//   Sec. II of arXiv:1904.02863.)
// * gw_pn_spin_terms: the aligned-spin additions for spins chi1, chi2 along
//   the orbital angular momentum, written body by body (x_i = m_i / M):
//   spin-orbit at 1.5PN (Kidder 1995), 2.5PN (Blanchet, Buonanno & Faye
//   2006; it enters as phi_5 (1 + 3 ln v)), 3PN with its tail (Blanchet 2014,
//   Living Rev. Relativ. 17, 2) and 3.5PN (Bohe, Marsat, Faye & Blanchet
//   2013); spin-spin at 2PN, S1 S2 (Kidder 1995) and the black-hole
//   quadrupole-monopole and self-spin terms (Poisson 1998).  The chi_eff
//   study of Sec. III of arXiv:1904.02863 implies a spinning template.
#pragma once

#include <hip/hip_runtime.h>

#include "gw_phasor_table.h"

#define GW_PI 3.141592653589793
#define GW_TWO_PI 6.283185307179586
#define GW_EULER_GAMMA 0.5772156649015329
#define GW_LN4 1.3862943611198906
#define GW_C_SI 299792458.0                     // m / s
#define GW_GM_SUN_SI 1.3271244e20               // m^3 s^-2, IAU 2015 B3 nominal solar mass parameter
#define GW_MPC_SI 3.0856775814913673e22         // m
#define GW_MSUN_S (GW_GM_SUN_SI / (GW_C_SI * GW_C_SI * GW_C_SI))   // solar mass in seconds
#define GW_MPC_S (GW_MPC_SI / GW_C_SI)                             // 1 Mpc / c in seconds

// sqrt(2) sin(pi r) = r P(z), z = r^2, |r| <= 1/2
#define GW_SINPI_P0 4.442882938158362
#define GW_SINPI_P1 -7.308249499994611
#define GW_SINPI_P2 3.6064765714243108
#define GW_SINPI_P3 -0.8474880236471133
#define GW_SINPI_P4 0.11617181135328143
#define GW_SINPI_P5 -0.010423245306932737
#define GW_SINPI_P6 0.000658941477865297
#define GW_SINPI_P7 -2.981954552480099e-05
// -sqrt(2) cos(pi r) = -sqrt(2) + z C(z)
#define GW_COSPI_C0 6.9788641996378855
#define GW_COSPI_C1 -5.739885734846492
#define GW_COSPI_C2 1.8883467136058691
#define GW_COSPI_C3 -0.33280771296175876
#define GW_COSPI_C4 0.03649596496885426
#define GW_COSPI_C5 -0.0027264665642378824
#define GW_COSPI_C6 0.00014206007015282065
#define GW_SQRT2 1.4142135623730951

// (re, im) = e^{-2 pi i x}: with s2 = sqrt(2) sin(pi r) and c2 = -sqrt(2) cos(pi r),
// re = cos 2 pi r = 1 - s2^2 and im = -sin 2 pi r = s2 c2 (20 floating-point
// operations; worst absolute error 5e-15).
__device__ __forceinline__ void gw_phasor_turns(double x, double &re, double &im)
{
    const double r = x - __builtin_rint(x);
    const double z = r * r;
    double p = GW_SINPI_P7;
    p = __builtin_fma(p, z, GW_SINPI_P6);
    p = __builtin_fma(p, z, GW_SINPI_P5);
    p = __builtin_fma(p, z, GW_SINPI_P4);
    p = __builtin_fma(p, z, GW_SINPI_P3);
    p = __builtin_fma(p, z, GW_SINPI_P2);
    p = __builtin_fma(p, z, GW_SINPI_P1);
    p = __builtin_fma(p, z, GW_SINPI_P0);
    const double s2 = r * p;
    double c = GW_COSPI_C6;
    c = __builtin_fma(c, z, GW_COSPI_C5);
    c = __builtin_fma(c, z, GW_COSPI_C4);
    c = __builtin_fma(c, z, GW_COSPI_C3);
    c = __builtin_fma(c, z, GW_COSPI_C2);
    c = __builtin_fma(c, z, GW_COSPI_C1);
    c = __builtin_fma(c, z, GW_COSPI_C0);
    const double c2 = __builtin_fma(z, c, -GW_SQRT2);
    re = __builtin_fma(-s2, s2, 1.0);
    im = s2 * c2;
}

// (re, im) = e^{-2 pi i x} for the scaled phase y = N x (x in turns, N =
// GW_PHTAB_N) from the table tab[k] = e^{-2 pi i k / N} ((re, im) pairs, in
// LDS) and short polynomials of the remainder: j = rint(y) by the
// round-to-integer of adding 1.5 * 2^52 (|y| < 2^51), r = y - j exactly
// (|r| <= 1/2), e^{-2 pi i x} = tab[j mod N] (cos(2 pi r / N) - i sin(2 pi r / N));
// j mod N comes from the low bits of the sum.  14 operations; worst absolute
// error 1.6e-16 (gen_phasor_table.py).
__device__ __forceinline__ void gw_phasor_table(double y, const double2 *__restrict__ tab, double &re, double &im)
{
    constexpr double kRound = 6755399441055744.0;       // 1.5 * 2^52
    const double t = y + kRound;
    const double r = y - (t - kRound);
    const double2 e = tab[__double2loint(t) & (GW_PHTAB_N - 1)];
    const double z = r * r;
    const double s = r * __builtin_fma(z, GW_PHTAB_S3, GW_PHTAB_S1);
    const double c = __builtin_fma(z, __builtin_fma(z, GW_PHTAB_C4, GW_PHTAB_C2), 1.0);
    re = __builtin_fma(e.x, c, e.y * s);
    im = __builtin_fma(e.y, c, -(e.x * s));
}

// The table of gw_phasor_table, (cos 2 pi k / N, -sin 2 pi k / N); each
// kernel that uses it copies it into LDS with gw_stage_phasor_table.
static __constant__ __align__(16) double gw_phasor_table_src[GW_PHTAB_N][2] = {GW_PHTAB_VALUES};

// Copies the table into tab (LDS, GW_PHTAB_N entries) with the threads of a
// block of block_threads threads; the caller's next barrier publishes it.
__device__ __forceinline__ void gw_stage_phasor_table(double2 *tab, int block_threads)
{
    for (int i = threadIdx.x; i < GW_PHTAB_N; i += block_threads)
        tab[i] = make_double2(gw_phasor_table_src[i][0], gw_phasor_table_src[i][1]);
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

// Aligned-spin additions to phi[k] and phi_log[5] (see the header comment);
// x1 = m1/M of the heavier body, x2 = 1 - x1, eta = x1 x2.
__device__ __forceinline__ void gw_pn_spin_terms(double x1, double x2, double chi1, double chi2, double phi[8],
                                                 double phi_log[8])
{
    const double eta = x1 * x2, eta2 = eta * eta;
    double so3 = 0.0, so5 = 0.0, so6 = 0.0, so7 = 0.0;
    const double xs[2] = {x1, x2}, cs[2] = {chi1, chi2};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double x = xs[i], c = cs[i];
        so3 += x * (25.0 + 38.0 / 3.0 * x) * c;
        so5 -= x * (13915.0 / 84.0 - 10.0 / 3.0 * eta + x * (12760.0 / 81.0 + 170.0 / 9.0 * eta)) * c;
        so6 += GW_PI * x * (1490.0 / 3.0 + 260.0 * x) * c;
        so7 += x * (-170978035.0 / 48384.0 + 2876425.0 / 672.0 * eta + 4735.0 / 144.0 * eta2 +
                    x * (-7189233785.0 / 1524096.0 + 458555.0 / 3024.0 * eta - 5345.0 / 72.0 * eta2)) * c;
    }
    phi[3] += so3;
    phi[4] += -395.0 / 4.0 * eta * chi1 * chi2 - 405.0 / 8.0 * (x1 * x1 * chi1 * chi1 + x2 * x2 * chi2 * chi2);
    phi[5] += so5;
    phi_log[5] += 3.0 * so5;
    phi[6] += so6;
    phi[7] += so7;
}
