// Device-side evaluation of the TaylorF2 template shared by the likelihood,
// waveform and relative-binning kernels: the per-frequency tables and the
// phase at detector 0 in turns from a sample's record (the record layout is
// described with RecordField in gw_internal.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "gw_internal.h"

namespace gw {

// f_k = f_low + k df, rounded the same way wherever a kernel needs it.
__device__ __forceinline__ double bin_frequency(double f_low, double df, int64_t k)
{
    return __dadd_rn(f_low, __dmul_rn((double)k, df));
}

// Tables of frequency f: u = f^(1/3), u^2, u^-5, ln u, f and the amplitude f^-7/6.
__device__ __forceinline__ void freq_tables(double f, Tab1 &t1, Tab2 &t2)
{
    const double u = cbrt(f);
    Tab1 a;
    a.u = u;
    a.u2 = u * u;
    a.um5 = pow(f, -5.0 / 3.0);
    a.lnu = log(f) / 3.0;
    t1 = a;
    Tab2 b;
    b.f = f;
    b.amp = pow(f, -7.0 / 6.0);
    t2 = b;
}

// Phase at detector 0 for one frequency, in turns (Horner in u, see RecordField).
struct PhaseCoef {
    double c8, c7, c6, c6l, c5, c5l, c4, c3, c2, c0;
};

__device__ __forceinline__ double turns_phase(const PhaseCoef &c, const Tab1 &t)
{
    const double t6 = __builtin_fma(c.c6l, t.lnu, c.c6);
    const double t5 = __builtin_fma(c.c5l, t.lnu, c.c5);
    double p = __builtin_fma(c.c8, t.u, c.c7);
    p = __builtin_fma(p, t.u, t6);
    p = __builtin_fma(p, t.u, t5);
    p = __builtin_fma(p, t.u, c.c4);
    p = __builtin_fma(p, t.u, c.c3);
    p = __builtin_fma(p, t.u, c.c2);
    p = __builtin_fma(p, t.u2, c.c0);
    return p * t.um5;
}

__device__ __forceinline__ PhaseCoef load_coef(const double *__restrict__ rec, int64_t ns, int64_t s)
{
    PhaseCoef c;
    c.c8 = rec[kRecC8 * ns + s];
    c.c7 = rec[kRecC7 * ns + s];
    c.c6 = rec[kRecC6 * ns + s];
    c.c6l = rec[kRecC6L * ns + s];
    c.c5 = rec[kRecC5 * ns + s];
    c.c5l = rec[kRecC5L * ns + s];
    c.c4 = rec[kRecC4 * ns + s];
    c.c3 = rec[kRecC3 * ns + s];
    c.c2 = rec[kRecC2 * ns + s];
    c.c0 = rec[kRecC0 * ns + s];
    return c;
}

// Every coefficient times k; with k a power of two the phase comes out scaled
// by k exactly.
__device__ __forceinline__ PhaseCoef scale_coef(PhaseCoef c, double k)
{
    c.c8 *= k;
    c.c7 *= k;
    c.c6 *= k;
    c.c6l *= k;
    c.c5 *= k;
    c.c5l *= k;
    c.c4 *= k;
    c.c3 *= k;
    c.c2 *= k;
    c.c0 *= k;
    return c;
}

}  // namespace gw
