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
// phasor of gw_device_math.h and the other detectors follow from complex
// rotations R_det,k+1 = R_det,k e^{-2 pi i df delta_det}, re-anchored exactly at
// the start of every LDS tile.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gw_device_math.h"
#include "gw_internal.h"

namespace gw {

// ---------------------------------------------------------------- event tables
__global__ __launch_bounds__(kBlock) void event_tables_kernel(double f_low, double df, int64_t n_bins,
                                                               Tab1 *__restrict__ tab1, Tab2 *__restrict__ tab2)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_bins; k += stride) {
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
}

// D_det,k = 4 df a_k conj(d) / S and per-block partial sums of |d|^2/S and a^2/S.
// A PSD value that is not positive and finite makes its weight NaN, which
// turns <d,d> and hence every lnL of the call into NaN.
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
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_bins; k += stride) {
        const double a = tab2[k].amp;
#pragma unroll
        for (int d = 0; d < kMaxDet; ++d) {
            if (d < n_det) {
                const double s = psd[(int64_t)d * n_bins + k];
                const double w = (s > 0.0 && s < INFINITY) ? 1.0 / s : NAN;
                const double2 v = data[(int64_t)d * n_bins + k];
                const double scale = 4.0 * df * a * w;
                dcoef[(int64_t)d * n_bins + k] = make_double2(scale * v.x, -scale * v.y);
                dd[d] += (v.x * v.x + v.y * v.y) * w;
                qq[d] += a * a * w;
            }
        }
    }
    // fixed-order tree reduction of each quantity over the block
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
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 2 * n_det + j] = red[0];
        __syncthreads();
    }
}

// event_sums[0] = <d,d> summed over detectors, event_sums[1 + det] = Q_det.
__global__ __launch_bounds__(kBlock) void event_sums_kernel(int n_blocks, int n_det, double df,
                                                             const double *__restrict__ partials,
                                                             double *__restrict__ event_sums)
{
    __shared__ double red[kBlock];
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

// ---------------------------------------------------------------- per-sample preparation
// One thread per sample: mass ratios, the half-phase polynomial coefficients,
// antenna patterns F = D : e, delays -n.r/c, and the complex amplitudes
//   P_det = A0 [F+ (1 + cos^2 iota)/2 - i Fx cos iota] e^{i (phi_c + pi/4)}.
// In polarisation mode (n_out == 2, no detectors) channel 0 is h_plus and
// channel 1 is h_cross.
__global__ __launch_bounds__(kBlock) void sample_prep_kernel(int64_t n_samples, int n_param, int n_out,
                                                              int polarisations, DetGeom geom,
                                                              const double *__restrict__ theta,
                                                              double *__restrict__ rec)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_samples) return;
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
    const double pref = 0.5 * 3.0 / (128.0 * eta);       // half phase
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
    rec[kRecC8 * ns + s] = GW_PI * tau0;
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

// ---------------------------------------------------------------- the hot loop
// Half phase at detector 0 for one bin (Horner in u, see RecordField).
struct PhaseCoef {
    double c8, c7, c6, c6l, c5, c5l, c4, c3, c2, c0;
};

__device__ __forceinline__ double half_phase(const PhaseCoef &c, const Tab1 &t)
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

// Block (chunk, group): the 256 samples of `group` (one per thread) against
// the bins of `chunk`, staged through LDS tile by tile and shared by all the
// block's samples.  Writes Z_det of every sample for this chunk.
// Block-to-work mapping: blocks are dispatched round-robin over the 8 XCDs;
// when the grid is a multiple of 8 the linear work index is remapped so that
// the blocks of one XCD cover consecutive chunks (and all sample groups of
// each), keeping their bin data in that XCD's L2.
template <int NDET>
__global__ __launch_bounds__(kBlock) void lnl_tile_kernel(int64_t n_bins, int64_t n_samples, double f_low,
                                                          double df, int n_groups, int64_t chunk_bins,
                                                          int tile_bins, const Tab1 *__restrict__ tab1,
                                                          const double2 *__restrict__ dcoef,
                                                          const double *__restrict__ rec,
                                                          double2 *__restrict__ partials)
{
    extern __shared__ double4 lds_raw[];
    Tab1 *lt = reinterpret_cast<Tab1 *>(lds_raw);
    double2 *ld = reinterpret_cast<double2 *>(lt + tile_bins);

    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned w = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const int group = (int)(w % (unsigned)n_groups);
    const int64_t chunk = (int64_t)(w / (unsigned)n_groups);
    const int64_t s = (int64_t)group * kBlock + threadIdx.x;
    const int64_t sr = s < n_samples ? s : n_samples - 1;

    const PhaseCoef cf = load_coef(rec, n_samples, sr);
    double rho_re[NDET], rho_im[NDET], delta[NDET];
#pragma unroll
    for (int d = 1; d < NDET; ++d) {
        delta[d] = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + sr];
        gw_phasor_half(GW_PI * df * delta[d], rho_re[d], rho_im[d]);
    }
    double zr[NDET], zi[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { zr[d] = 0.0; zi[d] = 0.0; }

    const int64_t k_begin = chunk * chunk_bins;
    const int64_t k_end = min(n_bins, k_begin + chunk_bins);
    for (int64_t t0 = k_begin; t0 < k_end; t0 += tile_bins) {
        const int nk = (int)min((int64_t)tile_bins, k_end - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < nk; i += kBlock) {
            lt[i] = tab1[t0 + i];
#pragma unroll
            for (int d = 0; d < NDET; ++d) ld[d * tile_bins + i] = dcoef[(int64_t)d * n_bins + t0 + i];
        }
        __syncthreads();
        double rr[NDET], ri[NDET];
        {
            const double f0 = __dadd_rn(f_low, __dmul_rn((double)t0, df));
#pragma unroll
            for (int d = 1; d < NDET; ++d) gw_phasor_half(GW_PI * f0 * delta[d], rr[d], ri[d]);
        }
        for (int j = 0; j < nk; ++j) {
            const Tab1 tb = lt[j];
            double er, ei;
            gw_phasor_half(half_phase(cf, tb), er, ei);
            const double2 d0 = ld[j];
            zr[0] = __builtin_fma(d0.x, er, zr[0]);
            zr[0] = __builtin_fma(-d0.y, ei, zr[0]);
            zi[0] = __builtin_fma(d0.x, ei, zi[0]);
            zi[0] = __builtin_fma(d0.y, er, zi[0]);
#pragma unroll
            for (int d = 1; d < NDET; ++d) {
                const double gr = er * rr[d] - ei * ri[d];
                const double gi = er * ri[d] + ei * rr[d];
                const double2 dv = ld[d * tile_bins + j];
                zr[d] = __builtin_fma(dv.x, gr, zr[d]);
                zr[d] = __builtin_fma(-dv.y, gi, zr[d]);
                zi[d] = __builtin_fma(dv.x, gi, zi[d]);
                zi[d] = __builtin_fma(dv.y, gr, zi[d]);
                const double nr = rr[d] * rho_re[d] - ri[d] * rho_im[d];
                const double ni = rr[d] * rho_im[d] + ri[d] * rho_re[d];
                rr[d] = nr;
                ri[d] = ni;
            }
        }
    }
    if (s < n_samples) {
#pragma unroll
        for (int d = 0; d < NDET; ++d)
            partials[(chunk * n_samples + s) * NDET + d] = make_double2(zr[d], zi[d]);
    }
}

// lnL = -1/2 <d,d> + sum_det [Re(P Z) - 1/2 |P|^2 Q], chunks summed in order.
__global__ __launch_bounds__(kBlock) void lnl_finalize_kernel(int64_t n_samples, int n_det, int n_chunks,
                                                               const double2 *__restrict__ partials,
                                                               const double *__restrict__ rec,
                                                               const double *__restrict__ event_sums,
                                                               double *__restrict__ lnl)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_samples) return;
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
    lnl[s] = out;
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
    gw_phasor_half(half_phase(cf, tb), er, ei);
    for (int d = 0; d < n_out; ++d) {
        const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + s];
        const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + s];
        const double delta = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + s];
        double gr = er, gi = ei;
        if (delta != 0.0) {
            double rr, ri;
            gw_phasor_half(GW_PI * t2.f * delta, rr, ri);
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
static const void *tile_kernel_ptr()
{
    return reinterpret_cast<const void *>(&lnl_tile_kernel<NDET>);
}

static const void *tile_kernel_for(int n_det)
{
    switch (n_det) {
    case 1: return tile_kernel_ptr<1>();
    case 2: return tile_kernel_ptr<2>();
    case 3: return tile_kernel_ptr<3>();
    case 4: return tile_kernel_ptr<4>();
    case 5: return tile_kernel_ptr<5>();
    case 6: return tile_kernel_ptr<6>();
    case 7: return tile_kernel_ptr<7>();
    default: return tile_kernel_ptr<8>();
    }
}

int lnl_tile_blocks_per_cu(int n_det, int tile_bins)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tile_kernel_for(n_det), kBlock,
                                                     lnl_tile_lds_bytes(n_det, tile_bins)) != hipSuccess)
        return 1;
    return n < 1 ? 1 : n;
}

template <int NDET>
static void launch_tiles_t(const gw_grid &grid, int64_t n_samples, const TilePlan &plan, const Tab1 *tab1,
                           const double2 *dcoef, const double *records, double2 *partials, hipStream_t stream)
{
    const unsigned blocks = (unsigned)plan.n_groups * (unsigned)plan.n_chunks;
    hipLaunchKernelGGL(lnl_tile_kernel<NDET>, dim3(blocks), dim3(kBlock), lnl_tile_lds_bytes(NDET, plan.tile_bins),
                       stream, grid.n_bins, n_samples, grid.f_low, grid.delta_f, plan.n_groups, plan.chunk_bins,
                       plan.tile_bins, tab1, dcoef, records, partials);
}

hipError_t launch_lnl_tiles(const gw_grid &grid, int n_det, int64_t n_samples, const TilePlan &plan,
                            const Tab1 *tab1, const double2 *dcoef, const double *records,
                            double2 *partials, hipStream_t stream)
{
    switch (n_det) {
    case 1: launch_tiles_t<1>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 2: launch_tiles_t<2>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 3: launch_tiles_t<3>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 4: launch_tiles_t<4>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 5: launch_tiles_t<5>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 6: launch_tiles_t<6>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 7: launch_tiles_t<7>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    case 8: launch_tiles_t<8>(grid, n_samples, plan, tab1, dcoef, records, partials, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
