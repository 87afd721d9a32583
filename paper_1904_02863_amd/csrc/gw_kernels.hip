// HIP kernels of the batched TaylorF2 likelihood for gfx950 (MI355X).
//
// The likelihood is Eq. (cbclike) of arXiv:1904.02863 (Sec. III).  With the
// noise-weighted inner product <a, b> = 4 df sum a* b / S its exponent splits
// exactly (an algebraic identity, not an approximation) into
//     lnL = -1/2 <d,d> + sum_det [ Re <d, h_det> - 1/2 <h_det, h_det> ].
// For the TaylorF2 template h_det,k = P_det a_k e^{-i Phi_det,k} with
// a_k = f_k^-7/6 and a per-(sample, detector) complex amplitude P_det, so
//     <h_det, h_det> = |P_det|^2 Q_det,         Q_det = 4 df sum_k a_k^2 / S_det,k
//     <d, h_det>     = P_det Z_det,             Z_det = sum_k D_det,k e^{-i Phi_det,k}
//     D_det,k = 4 df a_k conj(d_det,k) / S_det,k.
// Only Z needs a pass over (sample, bin, detector); <d,d>, Q and D are built
// once per event.  The per-detector phases differ by the time translation
// exp(-2 pi i f dt_det) described after Eq. (cbclike):
//     Phi_det,k = Phi_0,k + 2 pi f_k delta_det,  delta_det = dt_det - dt_0,
// so e^{-i Phi_0} is evaluated once per (sample, bin) with the polynomial
// phasor of gw_device_math.h.  For the other detectors the rotation
// e^{-2 pi i f_k delta} = R_last rho^(k - k_last), rho = e^{-2 pi i df delta},
// is applied by Horner's rule over the bins of a tile,
//     S <- S conj(rho) + D_k e^{-i Phi_0,k},   Z += R_last S at the tile end,
// with R_last evaluated exactly once per tile.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gw_device_math.h"
#include "gw_internal.h"

// Tuning of the tile kernel's inner loop: bins per unrolled step, and the
// number of waves per SIMD the register allocation must leave room for.
#ifndef GW_TILE_UNROLL
#define GW_TILE_UNROLL 4
#endif
#ifndef GW_TILE_WAVES_PER_EU
#define GW_TILE_WAVES_PER_EU 0
#endif
#if GW_TILE_WAVES_PER_EU > 0
#define GW_TILE_ATTR __attribute__((amdgpu_waves_per_eu(GW_TILE_WAVES_PER_EU)))
#else
#define GW_TILE_ATTR
#endif

namespace gw {

constexpr int kTileUnroll = GW_TILE_UNROLL;

// ---------------------------------------------------------------- event tables
// Tables of bin k: u = f^(1/3), u^2, u^-5, ln u, f and the amplitude f^-7/6.
__device__ __forceinline__ void bin_tables(double f_low, double df, int64_t k, Tab1 *tab1, Tab2 *tab2)
{
    const double f = __dadd_rn(f_low, __dmul_rn((double)k, df));
    const double u = cbrt(f);
    Tab1 t1;
    t1.u = u;
    t1.u2 = u * u;
    t1.um5 = pow(f, -5.0 / 3.0);
    t1.lnu = log(f) / 3.0;
    tab1[k] = t1;
    Tab2 t2;
    t2.f = f;
    t2.amp = pow(f, -7.0 / 6.0);
    tab2[k] = t2;
}

// D_det,k = 4 df a_k conj(d) / S for bin k, accumulating |d|^2/S and a^2/S.
// A PSD value that is not positive and finite makes its weight NaN, which
// turns <d,d> and hence every lnL of the event into NaN.
__device__ __forceinline__ void bin_data(int64_t n_bins, int n_det, double df, int64_t k, double amp,
                                         const double2 *__restrict__ data, const double *__restrict__ psd,
                                         double2 *__restrict__ dcoef, double dd[kMaxDet], double qq[kMaxDet])
{
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) {
        if (d < n_det) {
            const double s = psd[(int64_t)d * n_bins + k];
            const double w = (s > 0.0 && s < INFINITY) ? 1.0 / s : NAN;
            const double2 v = data[(int64_t)d * n_bins + k];
            const double scale = 4.0 * df * amp * w;
            dcoef[(int64_t)d * n_bins + k] = make_double2(scale * v.x, -scale * v.y);
            dd[d] += (v.x * v.x + v.y * v.y) * w;
            qq[d] += amp * amp * w;
        }
    }
}

// Fixed-order tree reduction over the block of (dd[d], qq[d]) for d < n_det;
// thread 0 writes out[2 d] = sum dd[d], out[2 d + 1] = sum qq[d].
__device__ __forceinline__ void block_reduce_pairs(int n_det, const double dd[kMaxDet], const double qq[kMaxDet],
                                                   double *red, double *out)
{
    for (int j = 0; j < 2 * n_det; ++j) {
        double x = 0.0;
#pragma unroll
        for (int d = 0; d < kMaxDet; ++d) {
            if (j == 2 * d) x = dd[d];
            if (j == 2 * d + 1) x = qq[d];
        }
        red[threadIdx.x] = x;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[j] = red[0];
        __syncthreads();
    }
}

// Sums the per-block partials of one event in a fixed order:
// event_sums[0] = <d,d> summed over detectors, event_sums[1 + det] = Q_det.
__device__ __forceinline__ void sum_event_partials(int n_blocks, int n_det, double df,
                                                   const double *__restrict__ partials, double *red,
                                                   double *__restrict__ event_sums)
{
    double total_dd = 0.0;
    for (int j = 0; j < 2 * n_det; ++j) {
        double x = 0.0;
        for (int b = threadIdx.x; b < n_blocks; b += kBlock) x += partials[(int64_t)b * 2 * n_det + j];
        red[threadIdx.x] = x;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (j % 2 == 0) total_dd += 4.0 * df * red[0];
            else event_sums[1 + j / 2] = 4.0 * df * red[0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) event_sums[0] = total_dd;
}

__global__ __launch_bounds__(kBlock) void event_tables_kernel(double f_low, double df, int64_t n_bins,
                                                               Tab1 *__restrict__ tab1, Tab2 *__restrict__ tab2)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_bins; k += stride)
        bin_tables(f_low, df, k, tab1, tab2);
}

__global__ __launch_bounds__(kBlock) void event_data_kernel(int64_t n_bins, int n_det, double df,
                                                             const double2 *__restrict__ data,
                                                             const double *__restrict__ psd,
                                                             const Tab2 *__restrict__ tab2,
                                                             double2 *__restrict__ dcoef,
                                                             double *__restrict__ partials)
{
    __shared__ double red[kBlock];
    double dd[kMaxDet], qq[kMaxDet];
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) { dd[d] = 0.0; qq[d] = 0.0; }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_bins; k += stride)
        bin_data(n_bins, n_det, df, k, tab2[k].amp, data, psd, dcoef, dd, qq);
    block_reduce_pairs(n_det, dd, qq, red, partials + (int64_t)blockIdx.x * 2 * n_det);
}

__global__ __launch_bounds__(kBlock) void event_sums_kernel(int n_blocks, int n_det, double df,
                                                             const double *__restrict__ partials,
                                                             double *__restrict__ event_sums)
{
    __shared__ double red[kBlock];
    sum_event_partials(n_blocks, n_det, df, partials, red, event_sums);
}

// Ragged batch, all events at once: block b handles bins
// [256 local, 256 local + 256) of event e, (e, local) = block_map[b].
__global__ __launch_bounds__(kBlock) void ragged_event_prep_kernel(const RaggedEvent *__restrict__ events,
                                                                    const int2 *__restrict__ block_map)
{
    __shared__ double red[kBlock];
    const int2 em = block_map[blockIdx.x];
    const RaggedEvent &re = events[em.x];
    double dd[kMaxDet], qq[kMaxDet];
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) { dd[d] = 0.0; qq[d] = 0.0; }
    const int64_t k = (int64_t)em.y * kBlock + threadIdx.x;
    if (k < re.n_bins) {
        bin_tables(re.f_low, re.df, k, re.tab1, re.tab2);
        bin_data(re.n_bins, re.n_det, re.df, k, re.tab2[k].amp, re.data, re.psd, re.dcoef, dd, qq);
    }
    block_reduce_pairs(re.n_det, dd, qq, red, re.prep + (int64_t)em.y * 2 * re.n_det);
}

// Ragged batch: block e sums event e's per-block partials.
__global__ __launch_bounds__(kBlock) void ragged_event_sums_kernel(const RaggedEvent *__restrict__ events)
{
    __shared__ double red[kBlock];
    const RaggedEvent &re = events[blockIdx.x];
    sum_event_partials(re.prep_blocks, re.n_det, re.df, re.prep, red, re.sums);
}

// ---------------------------------------------------------------- per-sample preparation
// Row s: mass ratios, the phase polynomial coefficients (in turns), antenna
// patterns F = D : e, delays -n.r/c, and the complex amplitudes
//   P_det = A0 [F+ (1 + cos^2 iota)/2 - i Fx cos iota] e^{i (phi_c + pi/4)}.
// In polarisation mode (n_out == 2, no detectors) channel 0 is h_plus and
// channel 1 is h_cross.
__device__ __forceinline__ void prep_sample(int64_t s, int64_t n_samples, int n_param, int n_out, bool polarisations,
                                            const DetGeom &geom, const double *__restrict__ theta,
                                            double *__restrict__ rec)
{
    double t[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) t[i] = i < n_param ? theta[s * n_param + i] : 0.0;
    int status = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (i < n_param && !isfinite(t[i])) status = 2;
    if (status == 0 && (!(t[0] > 0.0) || !(t[1] > 0.0 && t[1] <= 1.0) || !(t[2] > 0.0))) status = 1;

    const double mc = t[0], q = t[1], dl = t[2], phic = t[3], tc = t[4];
    const double eta = q / ((1.0 + q) * (1.0 + q));
    const double mtot_s = mc * pow(eta, -0.6) * GW_MSUN_S;
    const double alpha = cbrt(GW_PI * mtot_s);          // v = alpha u
    const double ln_alpha = log(alpha);
    double phi[8], phil[8];
    gw_pn_coefficients(eta, phi, phil);
    const double pref = 3.0 / (128.0 * eta) / GW_TWO_PI;   // phase in turns
    double apow[8];
    {
        const double a2 = alpha * alpha;
        apow[5] = 1.0;
        apow[6] = alpha;
        apow[7] = a2;
        apow[0] = 1.0 / (a2 * a2 * alpha);
        apow[1] = apow[0] * alpha;
        apow[2] = apow[1] * alpha;
        apow[3] = apow[2] * alpha;
        apow[4] = apow[3] * alpha;
    }
    double cj[8], cjl[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        cj[j] = pref * apow[j] * (phi[j] + phil[j] * ln_alpha);
        cjl[j] = pref * apow[j] * phil[j];
    }

    // detector geometry
    const double ci = n_param == 9 ? cos(t[8]) : 1.0;
    double fp[kMaxDet], fx[kMaxDet], dt[kMaxDet];
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) { fp[d] = 1.0; fx[d] = 0.0; dt[d] = 0.0; }
    if (n_param == 9 && !polarisations) {
        const double ra = t[5], dec = t[6], psi = t[7];
        const double cra = cos(ra), sra = sin(ra), cde = cos(dec), sde = sin(dec), cps = cos(psi), sps = sin(psi);
        const double n[3] = {cde * cra, cde * sra, sde};
        const double ea[3] = {-sra, cra, 0.0};
        const double ed[3] = {-sde * cra, -sde * sra, cde};
        double x[3], y[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] = cps * ea[i] + sps * ed[i];
            y[i] = -sps * ea[i] + cps * ed[i];
        }
#pragma unroll
        for (int d = 0; d < kMaxDet; ++d) {
            if (d < n_out) {
                double p = 0.0, c = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const double dij = geom.tensor[d][3 * i + j];
                        p += dij * (x[i] * x[j] - y[i] * y[j]);
                        c += dij * (x[i] * y[j] + y[i] * x[j]);
                    }
                fp[d] = p;
                fx[d] = c;
                dt[d] = -(n[0] * geom.vertex[d][0] + n[1] * geom.vertex[d][1] + n[2] * geom.vertex[d][2]) / GW_C_SI;
            }
        }
    }
    const double tau0 = tc + dt[0];

    const double amp0 = sqrt(5.0 / 24.0) * pow(GW_PI, -2.0 / 3.0) * pow(mc * GW_MSUN_S, 5.0 / 6.0) / (dl * GW_MPC_S);
    const double rot_re = cos(phic + 0.25 * GW_PI), rot_im = sin(phic + 0.25 * GW_PI);
    const double plus = 0.5 * (1.0 + ci * ci);

    const int64_t ns = n_samples;
    rec[kRecC8 * ns + s] = tau0;                            // 2 pi f tau0 in turns: tau0 u^3
    rec[kRecC7 * ns + s] = cj[7];
    rec[kRecC6 * ns + s] = cj[6];
    rec[kRecC6L * ns + s] = cjl[6];
    rec[kRecC5 * ns + s] = cj[5];
    rec[kRecC5L * ns + s] = cjl[5];
    rec[kRecC4 * ns + s] = cj[4];
    rec[kRecC3 * ns + s] = cj[3];
    rec[kRecC2 * ns + s] = cj[2];
    rec[kRecC0 * ns + s] = cj[0];
    rec[kRecStatus * ns + s] = (double)status;
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) {
        if (d < n_out) {
            double pre, pim;   // P before the e^{i(phi_c + pi/4)} rotation
            if (polarisations) {
                pre = d == 0 ? amp0 * plus : 0.0;
                pim = d == 0 ? 0.0 : -amp0 * ci;
            } else {
                pre = amp0 * fp[d] * plus;
                pim = -amp0 * fx[d] * ci;
            }
            rec[(kRecDet + kRecFieldsPerDet * d) * ns + s] = pre * rot_re - pim * rot_im;
            rec[(kRecDet + kRecFieldsPerDet * d + 1) * ns + s] = pre * rot_im + pim * rot_re;
            rec[(kRecDet + kRecFieldsPerDet * d + 2) * ns + s] = dt[d] - dt[0];
        }
    }
}

__global__ __launch_bounds__(kBlock) void sample_prep_kernel(int64_t n_samples, int n_param, int n_out,
                                                              int polarisations, DetGeom geom,
                                                              const double *__restrict__ theta,
                                                              double *__restrict__ rec)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_samples) return;
    prep_sample(s, n_samples, n_param, n_out, polarisations != 0, geom, theta, rec);
}

// Ragged batch: block (event, group) prepares the group's rows.
__global__ __launch_bounds__(kBlock) void ragged_sample_prep_kernel(const RaggedEvent *__restrict__ events,
                                                                     const int2 *__restrict__ groups,
                                                                     const DetGeom *__restrict__ geoms, int n_param)
{
    const int2 eg = groups[blockIdx.x];
    const RaggedEvent &re = events[eg.x];
    const int64_t s = (int64_t)eg.y * kBlock + threadIdx.x;
    if (s >= re.n_samples) return;
    prep_sample(s, re.n_samples, n_param, re.n_det, false, geoms[eg.x], re.theta, re.rec);
}

// Sets n counters to zero (a kernel rather than a memset, so that it can be
// captured in a graph).
__global__ void zero_counters_kernel(unsigned *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- the hot loop
// Phase at detector 0 for one bin, in turns (Horner in u, see RecordField).
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

// One event seen by the tile loop.
struct EventView {
    int64_t n_bins, n_samples;
    double f_low, df;
    const Tab1 *tab1;
    const double2 *dcoef;
    const double *rec;
    double2 *partials;     // [chunk][n_samples][NDET]
};

// The 256 samples of `group` (one per thread) against bins [k_begin, k_end)
// of one event, staged through LDS tile by tile and shared by all the
// block's samples; writes Z_det of every sample for chunk `chunk`.
// MIXED selects the mixed-precision path: the phase polynomial and its
// reduction to a fractional turn stay FP64 (the phase reaches ~1e4 rad), the
// phasor e^{-i Phi_0} comes from the FP32 hardware sine/cosine, and the
// projection, accumulation and all sums stay FP64.
// All threads of the block must call this with the same arguments.
template <int NDET, bool MIXED>
__device__ __forceinline__ void tile_chunk(const EventView &ev, int group, int64_t chunk, int64_t k_begin,
                                           int64_t k_end, int tile_bins, Tab1 *lt, double2 *ld)
{
    const int64_t n_bins = ev.n_bins, n_samples = ev.n_samples;
    const double f_low = ev.f_low, df = ev.df;
    const Tab1 *__restrict__ tab1 = ev.tab1;
    const double2 *__restrict__ dcoef = ev.dcoef;
    const double *__restrict__ rec = ev.rec;
    const int64_t s = (int64_t)group * kBlock + threadIdx.x;
    const int64_t sr = s < n_samples ? s : n_samples - 1;

    const PhaseCoef cf = load_coef(rec, n_samples, sr);
    double rho_re[NDET], rho_im[NDET], delta[NDET];
#pragma unroll
    for (int d = 1; d < NDET; ++d) {
        delta[d] = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + sr];
        gw_phasor_turns(df * delta[d], rho_re[d], rho_im[d]);
    }
    double zr[NDET], zi[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { zr[d] = 0.0; zi[d] = 0.0; }

    for (int64_t t0 = k_begin; t0 < k_end; t0 += tile_bins) {
        const int nk = (int)min((int64_t)tile_bins, k_end - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < nk; i += kBlock) {
            lt[i] = tab1[t0 + i];
#pragma unroll
            for (int d = 0; d < NDET; ++d) ld[d * tile_bins + i] = dcoef[(int64_t)d * n_bins + t0 + i];
        }
        __syncthreads();
        double sr_[NDET], si_[NDET];
#pragma unroll
        for (int d = 1; d < NDET; ++d) { sr_[d] = 0.0; si_[d] = 0.0; }
#pragma unroll kTileUnroll
        for (int j = 0; j < nk; ++j) {
            const Tab1 tb = lt[j];
            double er, ei;
            if constexpr (MIXED) {
                // FP64 phase and exact reduction to a fractional turn, then the
                // hardware sine and cosine (inputs in turns) in FP32
                const double x = turns_phase(cf, tb);
                const float r = (float)(x - __builtin_rint(x));
                er = (double)__builtin_amdgcn_cosf(r);
                ei = -(double)__builtin_amdgcn_sinf(r);
            } else {
                gw_phasor_turns(turns_phase(cf, tb), er, ei);
            }
            const double2 d0 = ld[j];
            zr[0] = __builtin_fma(d0.x, er, zr[0]);
            zr[0] = __builtin_fma(-d0.y, ei, zr[0]);
            zi[0] = __builtin_fma(d0.x, ei, zi[0]);
            zi[0] = __builtin_fma(d0.y, er, zi[0]);
#pragma unroll
            for (int d = 1; d < NDET; ++d) {
                const double2 dv = ld[d * tile_bins + j];
                double tr = dv.x * er;
                tr = __builtin_fma(-dv.y, ei, tr);
                tr = __builtin_fma(sr_[d], rho_re[d], tr);
                tr = __builtin_fma(si_[d], rho_im[d], tr);
                double ti = dv.x * ei;
                ti = __builtin_fma(dv.y, er, ti);
                ti = __builtin_fma(si_[d], rho_re[d], ti);
                ti = __builtin_fma(-sr_[d], rho_im[d], ti);
                sr_[d] = tr;
                si_[d] = ti;
            }
        }
        if (NDET > 1) {
            const double f_last = __dadd_rn(f_low, __dmul_rn((double)(t0 + nk - 1), df));
#pragma unroll
            for (int d = 1; d < NDET; ++d) {
                double rr, ri;
                gw_phasor_turns(f_last * delta[d], rr, ri);
                zr[d] = __builtin_fma(rr, sr_[d], zr[d]);
                zr[d] = __builtin_fma(-ri, si_[d], zr[d]);
                zi[d] = __builtin_fma(rr, si_[d], zi[d]);
                zi[d] = __builtin_fma(ri, sr_[d], zi[d]);
            }
        }
    }
    if (s < n_samples) {
#pragma unroll
        for (int d = 0; d < NDET; ++d)
            ev.partials[(chunk * n_samples + s) * NDET + d] = make_double2(zr[d], zi[d]);
    }
}

// One event: block (chunk, group).  Blocks are dispatched round-robin over the
// 8 XCDs; when the grid is a multiple of 8 the linear work index is remapped
// so that the blocks of one XCD cover consecutive chunks (and all sample
// groups of each), keeping their bin data in that XCD's L2.
template <int NDET, bool MIXED>
__global__ __launch_bounds__(kBlock) GW_TILE_ATTR void lnl_tile_kernel(EventView ev, int n_groups, int64_t chunk_bins,
                                                                       int tile_bins)
{
    extern __shared__ double4 lds_raw[];
    Tab1 *lt = reinterpret_cast<Tab1 *>(lds_raw);
    double2 *ld = reinterpret_cast<double2 *>(lt + tile_bins);
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned w = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const int group = (int)(w % (unsigned)n_groups);
    const int64_t chunk = (int64_t)(w / (unsigned)n_groups);
    const int64_t k_begin = chunk * chunk_bins;
    const int64_t k_end = min(ev.n_bins, k_begin + chunk_bins);
    tile_chunk<NDET, MIXED>(ev, group, chunk, k_begin, k_end, tile_bins, lt, ld);
}

// Many events: a persistent grid.  Every block repeatedly takes the next work
// item (event, sample group, bin chunk) from a device counter until the list
// is exhausted; the list is sorted by decreasing cost, so the large items go
// first and the small ones fill the tail.  The counter must be zero at launch.
template <int NDET, bool MIXED>
__global__ __launch_bounds__(kBlock) GW_TILE_ATTR void lnl_ragged_kernel(const RaggedEvent *__restrict__ events,
                                                                         const WorkItem *__restrict__ items,
                                                                         int n_items, unsigned *__restrict__ counter,
                                                                         int tile_bins)
{
    extern __shared__ double4 lds_raw[];
    __shared__ int next;
    Tab1 *lt = reinterpret_cast<Tab1 *>(lds_raw);
    double2 *ld = reinterpret_cast<double2 *>(lt + tile_bins);
    for (;;) {
        __syncthreads();                 // every thread has read `next` and left the LDS
        if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = next;
        if (it >= n_items) break;
        const WorkItem wi = items[it];
        const RaggedEvent &re = events[wi.event];
        EventView ev;
        ev.n_bins = re.n_bins;
        ev.n_samples = re.n_samples;
        ev.f_low = re.f_low;
        ev.df = re.df;
        ev.tab1 = re.tab1;
        ev.dcoef = re.dcoef;
        ev.rec = re.rec;
        ev.partials = re.partials;
        const int64_t k_begin = (int64_t)wi.chunk * re.chunk_bins;
        const int64_t k_end = min(re.n_bins, k_begin + re.chunk_bins);
        tile_chunk<NDET, MIXED>(ev, wi.group, wi.chunk, k_begin, k_end, tile_bins, lt, ld);
    }
}

// lnL = -1/2 <d,d> + sum_det [Re(P Z) - 1/2 |P|^2 Q], chunks summed in order.
__device__ __forceinline__ double finalize_row(int64_t s, int64_t n_samples, int n_det, int n_chunks,
                                               const double2 *__restrict__ partials, const double *__restrict__ rec,
                                               const double *__restrict__ event_sums)
{
    const double dd = event_sums[0];
    double acc = -0.5 * dd;
    for (int d = 0; d < n_det; ++d) {
        double zr = 0.0, zi = 0.0;
        for (int c = 0; c < n_chunks; ++c) {
            const double2 z = partials[((int64_t)c * n_samples + s) * n_det + d];
            zr += z.x;
            zi += z.y;
        }
        const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + s];
        const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + s];
        acc += (pr * zr - pi * zi) - 0.5 * (pr * pr + pi * pi) * event_sums[1 + d];
    }
    const int status = (int)rec[kRecStatus * n_samples + s];
    double out = acc;
    if (status == 1) out = -INFINITY;
    if (status == 2 || isnan(dd)) out = NAN;
    return out;
}

__global__ __launch_bounds__(kBlock) void lnl_finalize_kernel(int64_t n_samples, int n_det, int n_chunks,
                                                               const double2 *__restrict__ partials,
                                                               const double *__restrict__ rec,
                                                               const double *__restrict__ event_sums,
                                                               double *__restrict__ lnl)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_samples) return;
    lnl[s] = finalize_row(s, n_samples, n_det, n_chunks, partials, rec, event_sums);
}

// Ragged batch: block (event, group) finalizes the group's rows.
__global__ __launch_bounds__(kBlock) void ragged_finalize_kernel(const RaggedEvent *__restrict__ events,
                                                                  const int2 *__restrict__ groups)
{
    const int2 eg = groups[blockIdx.x];
    const RaggedEvent &re = events[eg.x];
    const int64_t s = (int64_t)eg.y * kBlock + threadIdx.x;
    if (s >= re.n_samples) return;
    re.lnl[s] = finalize_row(s, re.n_samples, re.n_det, re.n_chunks, re.partials, re.rec, re.sums);
}

// ---------------------------------------------------------------- waveform materialisation
// h[s][ch][k] = a_k P_ch e^{-i Phi_0,k} e^{-2 pi i f_k delta_ch}; one thread per bin,
// consecutive bins in consecutive lanes for coalesced 16-byte stores.
__global__ __launch_bounds__(kBlock) void waveform_kernel(int64_t n_bins, int n_out, int64_t n_samples,
                                                           int64_t blocks_per_sample,
                                                           const Tab1 *__restrict__ tab1,
                                                           const Tab2 *__restrict__ tab2,
                                                           const double *__restrict__ rec,
                                                           double2 *__restrict__ h_out)
{
    const int64_t s = (int64_t)blockIdx.x / blocks_per_sample;
    const int64_t k = ((int64_t)blockIdx.x % blocks_per_sample) * kBlock + threadIdx.x;
    if (k >= n_bins) return;
    const int status = (int)rec[kRecStatus * n_samples + s];
    const PhaseCoef cf = load_coef(rec, n_samples, s);
    const Tab1 tb = tab1[k];
    const Tab2 t2 = tab2[k];
    double er, ei;
    gw_phasor_turns(turns_phase(cf, tb), er, ei);
    for (int d = 0; d < n_out; ++d) {
        const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + s];
        const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + s];
        const double delta = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + s];
        double gr = er, gi = ei;
        if (delta != 0.0) {
            double rr, ri;
            gw_phasor_turns(t2.f * delta, rr, ri);
            gr = er * rr - ei * ri;
            gi = er * ri + ei * rr;
        }
        double2 h;
        h.x = t2.amp * (pr * gr - pi * gi);
        h.y = t2.amp * (pr * gi + pi * gr);
        if (status != 0) h = make_double2(NAN, NAN);
        h_out[((int64_t)s * n_out + d) * n_bins + k] = h;
    }
}

// ---------------------------------------------------------------- launchers
static int grid_blocks(int64_t n, int cap)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t launch_event_tables(const gw_grid &grid, Tab1 *tab1, Tab2 *tab2, hipStream_t stream)
{
    hipLaunchKernelGGL(event_tables_kernel, dim3(grid_blocks(grid.n_bins, 4096)), dim3(kBlock), 0, stream,
                       grid.f_low, grid.delta_f, grid.n_bins, tab1, tab2);
    return hipGetLastError();
}

hipError_t launch_event_data(const gw_grid &grid, int n_det, const gw_c128 *data, const double *psd,
                             const Tab2 *tab2, double2 *dcoef, double *prep_partials, int prep_blocks,
                             double *event_sums, hipStream_t stream)
{
    hipLaunchKernelGGL(event_data_kernel, dim3(prep_blocks), dim3(kBlock), 0, stream, grid.n_bins, n_det,
                       grid.delta_f, reinterpret_cast<const double2 *>(data), psd, tab2, dcoef, prep_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(event_sums_kernel, dim3(1), dim3(kBlock), 0, stream, prep_blocks, n_det, grid.delta_f,
                       prep_partials, event_sums);
    return hipGetLastError();
}

hipError_t launch_sample_prep(int64_t n_samples, int n_param, int n_out, bool polarisations, const DetGeom &geom,
                              const double *theta, double *records, hipStream_t stream)
{
    hipLaunchKernelGGL(sample_prep_kernel, dim3(grid_blocks(n_samples, 1 << 30)), dim3(kBlock), 0, stream,
                       n_samples, n_param, n_out, polarisations ? 1 : 0, geom, theta, records);
    return hipGetLastError();
}

size_t lnl_tile_lds_bytes(int n_det, int tile_bins)
{
    return (size_t)tile_bins * (sizeof(Tab1) + (size_t)n_det * sizeof(double2));
}

template <int NDET>
static const void *tile_kernel_ptr(bool mixed)
{
    return mixed ? reinterpret_cast<const void *>(&lnl_tile_kernel<NDET, true>)
                 : reinterpret_cast<const void *>(&lnl_tile_kernel<NDET, false>);
}

static const void *tile_kernel_for(int n_det, bool mixed)
{
    switch (n_det) {
    case 1: return tile_kernel_ptr<1>(mixed);
    case 2: return tile_kernel_ptr<2>(mixed);
    case 3: return tile_kernel_ptr<3>(mixed);
    case 4: return tile_kernel_ptr<4>(mixed);
    case 5: return tile_kernel_ptr<5>(mixed);
    case 6: return tile_kernel_ptr<6>(mixed);
    case 7: return tile_kernel_ptr<7>(mixed);
    default: return tile_kernel_ptr<8>(mixed);
    }
}

int lnl_tile_blocks_per_cu(int n_det, int tile_bins, bool mixed)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tile_kernel_for(n_det, mixed), kBlock,
                                                     lnl_tile_lds_bytes(n_det, tile_bins)) != hipSuccess)
        return 1;
    return n < 1 ? 1 : n;
}

template <int NDET>
static void launch_tiles_t(const EventView &ev, const TilePlan &plan, bool mixed, hipStream_t stream)
{
    const unsigned blocks = (unsigned)plan.n_groups * (unsigned)plan.n_chunks;
    const size_t lds = lnl_tile_lds_bytes(NDET, plan.tile_bins);
    if (mixed)
        hipLaunchKernelGGL((lnl_tile_kernel<NDET, true>), dim3(blocks), dim3(kBlock), lds, stream, ev, plan.n_groups,
                           plan.chunk_bins, plan.tile_bins);
    else
        hipLaunchKernelGGL((lnl_tile_kernel<NDET, false>), dim3(blocks), dim3(kBlock), lds, stream, ev, plan.n_groups,
                           plan.chunk_bins, plan.tile_bins);
}

hipError_t launch_lnl_tiles(const gw_grid &grid, int n_det, int64_t n_samples, const TilePlan &plan, bool mixed,
                            const Tab1 *tab1, const double2 *dcoef, const double *records,
                            double2 *partials, hipStream_t stream)
{
    EventView ev;
    ev.n_bins = grid.n_bins;
    ev.n_samples = n_samples;
    ev.f_low = grid.f_low;
    ev.df = grid.delta_f;
    ev.tab1 = tab1;
    ev.dcoef = dcoef;
    ev.rec = records;
    ev.partials = partials;
    switch (n_det) {
    case 1: launch_tiles_t<1>(ev, plan, mixed, stream); break;
    case 2: launch_tiles_t<2>(ev, plan, mixed, stream); break;
    case 3: launch_tiles_t<3>(ev, plan, mixed, stream); break;
    case 4: launch_tiles_t<4>(ev, plan, mixed, stream); break;
    case 5: launch_tiles_t<5>(ev, plan, mixed, stream); break;
    case 6: launch_tiles_t<6>(ev, plan, mixed, stream); break;
    case 7: launch_tiles_t<7>(ev, plan, mixed, stream); break;
    case 8: launch_tiles_t<8>(ev, plan, mixed, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NDET>
static void launch_ragged_t(const RaggedClass &c, const RaggedEvent *events, bool mixed, int tile_bins,
                            hipStream_t stream)
{
    const size_t lds = lnl_tile_lds_bytes(NDET, tile_bins);
    if (mixed)
        hipLaunchKernelGGL((lnl_ragged_kernel<NDET, true>), dim3(c.grid), dim3(kBlock), lds, stream, events, c.items,
                           c.n_items, c.counter, tile_bins);
    else
        hipLaunchKernelGGL((lnl_ragged_kernel<NDET, false>), dim3(c.grid), dim3(kBlock), lds, stream, events, c.items,
                           c.n_items, c.counter, tile_bins);
}

hipError_t launch_ragged(const RaggedLaunch &r, hipStream_t stream)
{
    hipLaunchKernelGGL(ragged_event_prep_kernel, dim3(r.n_prep_blocks), dim3(kBlock), 0, stream, r.events,
                       r.block_map);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ragged_event_sums_kernel, dim3(r.n_events), dim3(kBlock), 0, stream, r.events);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(ragged_sample_prep_kernel, dim3(r.n_groups), dim3(kBlock), 0, stream, r.events, r.groups,
                       r.geoms, r.n_param);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, stream, r.counters, kMaxDet);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int i = 0; i < r.n_classes; ++i) {
        const RaggedClass &c = r.classes[i];
        switch (c.n_det) {
        case 1: launch_ragged_t<1>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 2: launch_ragged_t<2>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 3: launch_ragged_t<3>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 4: launch_ragged_t<4>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 5: launch_ragged_t<5>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 6: launch_ragged_t<6>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 7: launch_ragged_t<7>(c, r.events, r.mixed, r.tile_bins, stream); break;
        case 8: launch_ragged_t<8>(c, r.events, r.mixed, r.tile_bins, stream); break;
        default: return hipErrorInvalidValue;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ragged_finalize_kernel, dim3(r.n_groups), dim3(kBlock), 0, stream, r.events, r.groups);
    return hipGetLastError();
}

template <int NDET>
static const void *ragged_kernel_ptr(bool mixed)
{
    return mixed ? reinterpret_cast<const void *>(&lnl_ragged_kernel<NDET, true>)
                 : reinterpret_cast<const void *>(&lnl_ragged_kernel<NDET, false>);
}

int lnl_ragged_blocks_per_cu(int n_det, int tile_bins, bool mixed)
{
    const void *fn = nullptr;
    switch (n_det) {
    case 1: fn = ragged_kernel_ptr<1>(mixed); break;
    case 2: fn = ragged_kernel_ptr<2>(mixed); break;
    case 3: fn = ragged_kernel_ptr<3>(mixed); break;
    case 4: fn = ragged_kernel_ptr<4>(mixed); break;
    case 5: fn = ragged_kernel_ptr<5>(mixed); break;
    case 6: fn = ragged_kernel_ptr<6>(mixed); break;
    case 7: fn = ragged_kernel_ptr<7>(mixed); break;
    default: fn = ragged_kernel_ptr<8>(mixed); break;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kBlock, lnl_tile_lds_bytes(n_det, tile_bins)) !=
        hipSuccess)
        return 1;
    return n < 1 ? 1 : n;
}

hipError_t launch_lnl_finalize(int64_t n_samples, int n_det, const TilePlan &plan, const double2 *partials,
                               const double *records, const double *event_sums, double *lnl_out,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(lnl_finalize_kernel, dim3(grid_blocks(n_samples, 1 << 30)), dim3(kBlock), 0, stream,
                       n_samples, n_det, plan.n_chunks, partials, records, event_sums, lnl_out);
    return hipGetLastError();
}

hipError_t launch_waveform(const gw_grid &grid, int n_out, int64_t n_samples, const Tab1 *tab1, const Tab2 *tab2,
                           const double *records, gw_c128 *h_out, hipStream_t stream)
{
    const int64_t per = (grid.n_bins + kBlock - 1) / kBlock;
    const int64_t blocks = per * n_samples;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(waveform_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, grid.n_bins, n_out,
                       n_samples, per, tab1, tab2, records, reinterpret_cast<double2 *>(h_out));
    return hipGetLastError();
}

}  // namespace gw
