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

#include "gw_build_id.h"
#include "gw_device_math.h"
#include "gw_internal.h"
#include "gw_plan.h"
#include "gw_template.h"

// Tuning of the tile kernel's inner loop: bins per unrolled step (FP64 and
// mixed paths), and the number of waves per SIMD the register allocation
// must leave room for.  The FP64 kernels run two blocks per CU (their LDS
// holds the phasor table), so 8 bins per step fit their registers; the mixed
// kernels run three, and 4 bins keep them within 168 VGPRs.
#ifndef GW_TILE_UNROLL
#define GW_TILE_UNROLL 8
#endif
#ifndef GW_TILE_UNROLL_MIXED
#define GW_TILE_UNROLL_MIXED 4
#endif
#ifndef GW_TILE_WAVES_PER_EU
#define GW_TILE_WAVES_PER_EU 0
#endif
// 1: the FP64 tile loops take e^{-i Phi} from the LDS table (gw_phasor_table);
// 0: from the polynomial phasor (gw_phasor_turns).
#ifndef GW_PHASOR_TABLE
#define GW_PHASOR_TABLE 1
#endif
#if GW_TILE_WAVES_PER_EU > 0
#define GW_TILE_ATTR __attribute__((amdgpu_waves_per_eu(GW_TILE_WAVES_PER_EU)))
#else
#define GW_TILE_ATTR
#endif

namespace gw {

constexpr int kTileUnroll = GW_TILE_UNROLL, kTileUnrollMixed = GW_TILE_UNROLL_MIXED;

// ---------------------------------------------------------------- event tables
__device__ __forceinline__ void bin_tables(double f_low, double df, int64_t k, Tab1 *tab1, Tab2 *tab2)
{
    freq_tables(bin_frequency(f_low, df, k), tab1[k], tab2[k]);
}

// One event's device arrays as the preparation kernels see them.
struct PrepView {
    int64_t n_bins;
    int n_det;
    double df;
    const double2 *data;
    const double *psd;
    const Tab2 *tab2;
    double2 *dcoef;
    double2 *edir;
    double *vdir;
};

// Bin k of every detector: D = 4 df a conj(d) / S (split form) and, for the
// direct form, d / a and a^2 / S; adds |d|^2/S, a^2/S and (with `norm`)
// ln(2 pi S) to acc[3 d + 0, 1, 2].  A PSD value that is not positive and
// finite makes its weight NaN, which turns <d,d> and hence every lnL of the
// event into NaN.
__device__ __forceinline__ void bin_data(const PrepView &v, int64_t k, bool direct, bool norm,
                                         double acc[kPrepPerDet * kMaxDet])
{
    const double amp = v.tab2[k].amp;
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) {
        if (d < v.n_det) {
            const double s = v.psd[(int64_t)d * v.n_bins + k];
            const double w = (s > 0.0 && s < INFINITY) ? 1.0 / s : NAN;
            const double2 x = v.data[(int64_t)d * v.n_bins + k];
            const double scale = 4.0 * v.df * amp * w;
            v.dcoef[(int64_t)d * v.n_bins + k] = make_double2(scale * x.x, -scale * x.y);
            if (direct) {
                v.edir[(int64_t)d * v.n_bins + k] = make_double2(x.x / amp, x.y / amp);
                v.vdir[(int64_t)d * v.n_bins + k] = amp * amp * w;
            }
            acc[kPrepPerDet * d] = (x.x * x.x + x.y * x.y) * w;
            acc[kPrepPerDet * d + 1] = amp * amp * w;
            acc[kPrepPerDet * d + 2] = norm ? log(2.0 * GW_PI * s) : 0.0;
        }
    }
}

// Fixed-order tree sum of x over the block; every thread gets the total.
// `red` is kBlock doubles of LDS.  All threads must call it.
__device__ __forceinline__ double block_sum(double x, double *red)
{
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double total = red[0];
    __syncthreads();
    return total;
}

// Sum over the 64 lanes of a wave by a fixed butterfly (lane 0's value is
// the one used).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Block b of an event's preparation: bins [256 b, 256 b + 256); writes the
// block's sums out[kPrepPerDet d + j] (wave sums, then the 4 waves in order).
// `red` holds at least 4 kPrepPerDet kMaxDet doubles of LDS.
__device__ __forceinline__ void prep_block(const PrepView &v, int64_t b, bool direct, bool norm, double *red,
                                           double *__restrict__ out)
{
    constexpr int kQ = kPrepPerDet * kMaxDet;
    double acc[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) acc[i] = 0.0;
    const int64_t k = b * kBlock + threadIdx.x;
    if (k < v.n_bins) bin_data(v, k, direct, norm, acc);
    const int nq = kPrepPerDet * v.n_det, lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
        if (j < nq) {
            const double t = wave_sum(acc[j]);
            if (lane == 0) red[wave * kQ + j] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nq)
        out[threadIdx.x] = ((red[threadIdx.x] + red[kQ + threadIdx.x]) + red[2 * kQ + threadIdx.x]) +
                           red[3 * kQ + threadIdx.x];
    __syncthreads();
}

// Column j of an event's per-block partials summed over its n_blocks blocks
// (strided per thread, then a fixed tree): the event-wide sum of quantity j.
__device__ __forceinline__ double column_total(int n_blocks, int per, int j, const double *__restrict__ partials,
                                               double *red)
{
    double x = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += kBlock) x += partials[(int64_t)b * per + j];
    return block_sum(x, red);
}

// Inclusive Hillis-Steele scan of x over the block (fixed order); `red` is
// kBlock doubles of LDS.  All threads must call it.
__device__ __forceinline__ double block_scan(double x, double *red)
{
    red[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const double add = (int)threadIdx.x >= off ? red[threadIdx.x - off] : 0.0;
        __syncthreads();
        red[threadIdx.x] += add;
        __syncthreads();
    }
    const double total = red[threadIdx.x];
    __syncthreads();
    return total;
}

// offsets[b] = sum over blocks b' < b of column j of an event's per-block
// partials, for every b < n_blocks (one block: each thread scans a
// contiguous segment of blocks on top of the preceding segments' totals).
__device__ __forceinline__ void block_offsets(int64_t n_blocks, int per, int j, const double *__restrict__ partials,
                                              double *red, double *__restrict__ offsets)
{
    const int64_t seg = (n_blocks + kBlock - 1) / kBlock;
    const int64_t b0 = (int64_t)threadIdx.x * seg, b1 = min(n_blocks, b0 + seg);
    double mine = 0.0;
    for (int64_t b = b0; b < b1; ++b) mine += partials[b * per + j];
    double run = block_scan(mine, red) - mine;      // exclusive: the preceding segments
    for (int64_t b = b0; b < b1; ++b) {
        offsets[b] = run;
        run += partials[b * per + j];
    }
}

// Prefix sums of a^2/S for the ISCO end: block b of the event writes
// qprefix[d][k] = sum_{j <= k} a_j^2 / S_d,j for its 256 bins, from the
// preceding blocks' total qoffsets[d][b] and a scan of its own bins.
__device__ __forceinline__ void prefix_block(const PrepView &v, int64_t b, int64_t n_blocks,
                                             const double *__restrict__ qoffsets, double *red,
                                             double *__restrict__ qprefix)
{
    const int64_t k = b * kBlock + threadIdx.x;
    const double amp = k < v.n_bins ? v.tab2[k].amp : 0.0;
    for (int d = 0; d < v.n_det; ++d) {
        const double offset = qoffsets[(int64_t)d * n_blocks + b];
        double q = 0.0;
        if (k < v.n_bins) {
            const double s = v.psd[(int64_t)d * v.n_bins + k];
            const double w = (s > 0.0 && s < INFINITY) ? 1.0 / s : NAN;
            q = amp * amp * w;
        }
        const double incl = block_scan(q, red);
        if (k < v.n_bins) qprefix[(int64_t)d * v.n_bins + k] = offset + incl;
    }
}

__global__ __launch_bounds__(kBlock) void event_tables_kernel(double f_low, double df, int64_t n_bins,
                                                               Tab1 *__restrict__ tab1, Tab2 *__restrict__ tab2)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_bins; k += stride)
        bin_tables(f_low, df, k, tab1, tab2);
}

// Block j: sums[j] = the event-wide sum of quantity j (kPrepPerDet n_det blocks).
// Also zeroes the tile kernel's work-queue counters when there are any.
__global__ __launch_bounds__(kBlock) void event_sums_kernel(int n_blocks, int n_det,
                                                             const double *__restrict__ partials,
                                                             double *__restrict__ sums, unsigned *__restrict__ queue)
{
    __shared__ double red[kBlock];
    const double t = column_total(n_blocks, kPrepPerDet * n_det, blockIdx.x, partials, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = t;
    if (queue && blockIdx.x == 0 && threadIdx.x < kQueues) queue[threadIdx.x] = 0u;
}

// Block d: qoffsets[d][b], the a^2/S total of the blocks before b.
__global__ __launch_bounds__(kBlock) void event_offsets_kernel(int64_t n_blocks, int n_det,
                                                                const double *__restrict__ partials,
                                                                double *__restrict__ qoffsets)
{
    __shared__ double red[kBlock];
    const int d = blockIdx.x;
    block_offsets(n_blocks, kPrepPerDet * n_det, kPrepPerDet * d + 1, partials, red, qoffsets + (int64_t)d * n_blocks);
}

__global__ __launch_bounds__(kBlock) void event_prefix_kernel(PrepView v, int64_t n_blocks,
                                                               const double *__restrict__ qoffsets,
                                                               double *__restrict__ qprefix)
{
    __shared__ double red[kBlock];
    prefix_block(v, blockIdx.x, n_blocks, qoffsets, red, qprefix);
}

__device__ __forceinline__ PrepView prep_view(const RaggedEvent &re)
{
    PrepView v;
    v.n_bins = re.n_bins;
    v.n_det = re.n_det;
    v.df = re.df;
    v.data = re.data;
    v.psd = re.psd;
    v.tab2 = re.tab2;
    v.dcoef = re.dcoef;
    v.edir = re.edir;
    v.vdir = re.vdir;
    return v;
}

// Ragged batch, all events at once: block b handles bins
// [256 local, 256 local + 256) of event e, (e, local) = block_map[b].
__global__ __launch_bounds__(kBlock) void ragged_event_prep_kernel(const RaggedEvent *__restrict__ events,
                                                                    const int2 *__restrict__ block_map,
                                                                    int direct, int norm)
{
    __shared__ double red[kBlock];
    const int2 em = block_map[blockIdx.x];
    const RaggedEvent &re = events[em.x];
    const int64_t k = (int64_t)em.y * kBlock + threadIdx.x;
    if (k < re.n_bins) bin_tables(re.f_low, re.df, k, re.tab1, re.tab2);
    __syncthreads();
    prep_block(prep_view(re), em.y, direct != 0, norm != 0, red,
               re.prep + (int64_t)em.y * kPrepPerDet * re.n_det);
}

// Ragged batch: block e sums event e's per-block partials.
__global__ __launch_bounds__(kBlock) void ragged_event_sums_kernel(const RaggedEvent *__restrict__ events)
{
    __shared__ double red[kBlock];
    const RaggedEvent &re = events[blockIdx.x];
    for (int j = 0; j < kPrepPerDet * re.n_det; ++j) {
        const double t = column_total(re.prep_blocks, kPrepPerDet * re.n_det, j, re.prep, red);
        if (threadIdx.x == 0) re.sums[j] = t;
    }
}

// Ragged batch: block e computes event e's qoffsets for every detector.
__global__ __launch_bounds__(kBlock) void ragged_offsets_kernel(const RaggedEvent *__restrict__ events)
{
    __shared__ double red[kBlock];
    const RaggedEvent &re = events[blockIdx.x];
    for (int d = 0; d < re.n_det; ++d)
        block_offsets(re.prep_blocks, kPrepPerDet * re.n_det, kPrepPerDet * d + 1, re.prep, red,
                      re.qoffsets + (int64_t)d * re.prep_blocks);
}

// Ragged batch: prefix sums of a^2/S, blocks as in ragged_event_prep_kernel.
__global__ __launch_bounds__(kBlock) void ragged_prefix_kernel(const RaggedEvent *__restrict__ events,
                                                                const int2 *__restrict__ block_map)
{
    __shared__ double red[kBlock];
    const int2 em = block_map[blockIdx.x];
    const RaggedEvent &re = events[em.x];
    prefix_block(prep_view(re), em.y, re.prep_blocks, re.qoffsets, red, re.qprefix);
}

// ---------------------------------------------------------------- per-sample preparation
// Row s: mass ratios, the phase polynomial coefficients (in turns), antenna
// patterns F = D : e, delays -n.r/c, and the complex amplitudes
//   P_det = A0 [F+ (1 + cos^2 iota)/2 - i Fx cos iota] e^{i (phi_c + pi/4)}.
// In polarisation mode (n_out == 2, no detectors) channel 0 is h_plus and
// channel 1 is h_cross.  The template's last bin K_s is n_bins - 1, or with
// the ISCO end the last bin with f_k <= f_isco = 1 / (6^(3/2) pi M) (-1 when
// there is none, and for samples that are not evaluated).
__device__ __forceinline__ void prep_sample(double f_low, double df, int64_t n_bins, int64_t s, int64_t n_samples,
                                            int n_param, int n_out, bool polarisations, bool isco,
                                            const DetGeom &geom, const double *__restrict__ theta,
                                            double *__restrict__ rec)
{
    double t[kMaxParam];
#pragma unroll
    for (int i = 0; i < kMaxParam; ++i) t[i] = i < n_param ? theta[s * n_param + i] : 0.0;
    int status = 0;
#pragma unroll
    for (int i = 0; i < kMaxParam; ++i)
        if (i < n_param && !isfinite(t[i])) status = 2;
    if (status == 0 && (!(t[0] > 0.0) || !(t[1] > 0.0 && t[1] <= 1.0) || !(t[2] > 0.0))) status = 1;
    const bool spins = param_has_spins(n_param);
    const double chi1 = spins ? t[n_param - 2] : 0.0, chi2 = spins ? t[n_param - 1] : 0.0;
    if (status == 0 && spins && (fabs(chi1) > 1.0 || fabs(chi2) > 1.0)) status = 1;

    const double mc = t[0], q = t[1], dl = t[2], phic = t[3], tc = t[4];
    const double eta = q / ((1.0 + q) * (1.0 + q));
    const double mtot_s = mc * pow(eta, -0.6) * GW_MSUN_S;
    const double alpha = cbrt(GW_PI * mtot_s);          // v = alpha u
    const double ln_alpha = log(alpha);
    double phi[8], phil[8];
    gw_pn_coefficients(eta, phi, phil);
    if (spins) gw_pn_spin_terms(1.0 / (1.0 + q), q / (1.0 + q), chi1, chi2, phi, phil);
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
    const double ci = param_has_sky(n_param) ? cos(t[8]) : 1.0;
    double fp[kMaxDet], fx[kMaxDet], dt[kMaxDet];
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) { fp[d] = 1.0; fx[d] = 0.0; dt[d] = 0.0; }
    if (param_has_sky(n_param) && !polarisations) {
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
    double kcut = (double)(n_bins - 1);
    if (isco) {
        kcut = -1.0;
        if (status == 0) {
            const double f_isco = 1.0 / (pow(6.0, 1.5) * GW_PI * mtot_s);
            const double kf = fmin(fmax(floor((f_isco - f_low) / df), -1.0), (double)(n_bins - 1));
            int64_t k = (int64_t)kf;
            // settle the rounding: the same f_k = f_low + k df as every table
            while (k + 1 < n_bins && __dadd_rn(f_low, __dmul_rn((double)(k + 1), df)) <= f_isco) ++k;
            while (k >= 0 && __dadd_rn(f_low, __dmul_rn((double)k, df)) > f_isco) --k;
            kcut = (double)k;
        }
    }
    rec[kRecKcut * ns + s] = kcut;
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

__global__ __launch_bounds__(kBlock) void sample_prep_kernel(double f_low, double df, int64_t n_bins,
                                                              int64_t n_samples, int n_param, int n_out,
                                                              int polarisations, int isco, DetGeom geom,
                                                              const double *__restrict__ theta,
                                                              double *__restrict__ rec)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_samples) return;
    prep_sample(f_low, df, n_bins, s, n_samples, n_param, n_out, polarisations != 0, isco != 0, geom, theta, rec);
}

// One block per 256 consecutive bins, after sample_blocks blocks of 256
// samples each (sample records, when sample_blocks > 0).  The two parts share
// no data, so one launch runs them side by side; the sample blocks come
// first, since each of their threads has the longer serial work.
__global__ __launch_bounds__(kBlock) void event_data_kernel(PrepView v, int direct, int norm,
                                                             double *__restrict__ partials, int sample_blocks,
                                                             double f_low, SamplePrep sp)
{
    if ((int)blockIdx.x < sample_blocks) {
        const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (s < sp.n_samples)
            prep_sample(f_low, v.df, v.n_bins, s, sp.n_samples, sp.n_param, v.n_det, false, sp.isco != 0, sp.geom,
                        sp.theta, sp.records);
        return;
    }
    __shared__ double red[kBlock];
    const int64_t b = (int64_t)blockIdx.x - sample_blocks;
    prep_block(v, b, direct != 0, norm != 0, red, partials + b * kPrepPerDet * v.n_det);
}

// *k_limit = 1 + the largest K_s of the batch (one block).
__global__ __launch_bounds__(kBlock) void isco_limit_kernel(int64_t n_samples, const double *__restrict__ rec,
                                                             int64_t *__restrict__ k_limit)
{
    __shared__ double red[kBlock];
    double m = -1.0;
    for (int64_t s = threadIdx.x; s < n_samples; s += kBlock) m = fmax(m, rec[kRecKcut * n_samples + s]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *k_limit = (int64_t)red[0] + 1;
}

// Ragged batch: block (event, group) prepares the group's rows.
__global__ __launch_bounds__(kBlock) void ragged_sample_prep_kernel(const RaggedEvent *__restrict__ events,
                                                                     const int2 *__restrict__ groups,
                                                                     const DetGeom *__restrict__ geoms, int n_param,
                                                                     int isco)
{
    const int2 eg = groups[blockIdx.x];
    const RaggedEvent &re = events[eg.x];
    const int64_t s = (int64_t)eg.y * kBlock + threadIdx.x;
    if (s >= re.n_samples) return;
    prep_sample(re.f_low, re.df, re.n_bins, s, re.n_samples, n_param, re.n_det, false, isco != 0, geoms[eg.x],
                re.theta, re.rec);
}

// Sets n counters to zero (a kernel rather than a memset, so that it can be
// captured in a graph).
__global__ void zero_counters_kernel(unsigned *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- the hot loop
// One event seen by the tile loop.
struct EventView {
    int64_t n_bins, n_samples;
    double f_low, df;
    const Tab1 *tab1;
    const double2 *dcoef;      // split forms: D [n_det][n_bins]
    const double2 *edir;       // direct form: d / a [n_det][n_bins]
    const double *vdir;        // direct form: a^2 / S [n_det][n_bins]
    const double *rec;
    const int64_t *k_limit;    // split form with the ISCO end: 1 + max K_s (device)
    double2 *partials;         // double [chunk][n_samples]: sum_det Re(P_det Z_det) (split), residual sum (direct)
};

// LDS layout of a tile: tab1 [tile], then per detector D (split) or d/a
// (direct) [NDET][tile] double2, then for the direct form a^2/S [NDET][tile].
// LDS of one tile block: the phasor table (FP64 path) and the tiles.
__host__ __device__ constexpr size_t phasor_table_lds(bool mixed)
{
    return (GW_PHASOR_TABLE && !mixed) ? (size_t)GW_PHTAB_N * sizeof(double2) : 0;
}
__host__ __device__ constexpr size_t tile_lds_bytes(int n_det, int tile_bins, int form, bool mixed)
{
    return phasor_table_lds(mixed) +
           (size_t)tile_bins * (sizeof(Tab1) + (size_t)n_det * sizeof(double2) +
                                (form == kFormDirect ? (size_t)n_det * sizeof(double) : 0));
}

// Copies the phasor table into the head of the block's LDS (FP64 path) and
// returns where the tiles begin.  The tile loop's first barrier publishes it.
template <bool MIXED>
__device__ __forceinline__ double *stage_phasor_table(double4 *lds_raw)
{
    if constexpr (GW_PHASOR_TABLE && !MIXED) {
        double2 *tab = reinterpret_cast<double2 *>(lds_raw);
        gw_stage_phasor_table(tab, kBlock);
        return reinterpret_cast<double *>(tab + GW_PHTAB_N);
    }
    return reinterpret_cast<double *>(lds_raw);
}

// The 256 samples of `group` (one per thread) against bins [k_begin, k_end)
// of one event, staged through LDS tile by tile and shared by all the
// block's samples; writes the chunk's partial sums of every sample.
// MIXED selects the mixed-precision path: the phase polynomial and its
// reduction to a fractional turn stay FP64 (the phase reaches ~1e4 rad), the
// phasor e^{-i Phi_0} comes from the FP32 hardware sine/cosine, and the
// projection, accumulation and all sums stay FP64.
// FORM (TileForm): the split forms accumulate Z_det (kFormSplitIsco only
// over bins k <= K_s of each sample); the direct form accumulates
// sum_det a^2/S |d/a - P_det e^{-i Phi_det}|^2 with the template zero above K_s.
// All threads of the block must call this with the same arguments.
template <int NDET, bool MIXED, int FORM>
__device__ __forceinline__ void tile_chunk(const EventView &ev, int group, int64_t chunk, int64_t k_begin,
                                           int64_t k_end, int tile_bins, double *lds)
{
    // the phasor table sits just below the tiles (FP64 path; the mixed path has none)
    const double2 *ptab =
        (GW_PHASOR_TABLE && !MIXED) ? reinterpret_cast<const double2 *>(lds) - GW_PHTAB_N : nullptr;
    constexpr bool kDirect = FORM == kFormDirect;
    constexpr bool kMasked = FORM != kFormSplit;
    const int64_t n_bins = ev.n_bins, n_samples = ev.n_samples;
    const double f_low = ev.f_low, df = ev.df;
    const Tab1 *__restrict__ tab1 = ev.tab1;
    const double2 *__restrict__ dsrc = kDirect ? ev.edir : ev.dcoef;
    const double *__restrict__ vdir = ev.vdir;
    const double *__restrict__ rec = ev.rec;
    const int64_t s = (int64_t)group * kBlock + threadIdx.x;
    const int64_t sr = s < n_samples ? s : n_samples - 1;
    Tab1 *lt = reinterpret_cast<Tab1 *>(lds);
    double2 *ld = reinterpret_cast<double2 *>(lt + tile_bins);
    double *lv = reinterpret_cast<double *>(ld + NDET * tile_bins);

    PhaseCoef cf = load_coef(rec, n_samples, sr);
#if GW_PHASOR_TABLE
    // the table phasor takes the phase in units of 1/N turn (exact: N is a power of two)
    if constexpr (!MIXED) cf = scale_coef(cf, (double)GW_PHTAB_N);
#endif
    const int64_t kcut = kMasked ? (int64_t)rec[kRecKcut * n_samples + sr] : n_bins - 1;
    double rho_re[NDET], rho_im[NDET], delta[NDET], p_re[NDET], p_im[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        if (kDirect) {
            p_re[d] = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + sr];
            p_im[d] = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + sr];
        }
        if (d == 0) continue;
        delta[d] = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + sr];
        gw_phasor_turns(df * delta[d], rho_re[d], rho_im[d]);
    }
    double zr[NDET], zi[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { zr[d] = 0.0; zi[d] = 0.0; }
    double acc = 0.0;

    for (int64_t t0 = k_begin; t0 < k_end; t0 += tile_bins) {
        const int nk = (int)min((int64_t)tile_bins, k_end - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < nk; i += kBlock) {
            lt[i] = tab1[t0 + i];
#pragma unroll
            for (int d = 0; d < NDET; ++d) {
                ld[d * tile_bins + i] = dsrc[(int64_t)d * n_bins + t0 + i];
                if (kDirect) lv[d * tile_bins + i] = vdir[(int64_t)d * n_bins + t0 + i];
            }
        }
        __syncthreads();
        // last live bin of this lane within the tile (template end)
        const int jcut = kMasked ? (int)max((int64_t)-1, min(kcut - t0, (int64_t)nk - 1)) : nk - 1;
        // split: Horner sums S_d over the tile; direct: T_d = P_d e^{-2 pi i f delta_d} at the current bin
        double sr_[NDET], si_[NDET];
#pragma unroll
        for (int d = 0; d < NDET; ++d) { sr_[d] = 0.0; si_[d] = 0.0; }
        if (kDirect) {
            const double f_first = __dadd_rn(f_low, __dmul_rn((double)t0, df));
#pragma unroll
            for (int d = 0; d < NDET; ++d) {
                if (d == 0) {
                    sr_[0] = p_re[0];
                    si_[0] = p_im[0];
                    continue;
                }
                double rr, ri;
                gw_phasor_turns(f_first * delta[d], rr, ri);
                sr_[d] = p_re[d] * rr - p_im[d] * ri;
                si_[d] = p_re[d] * ri + p_im[d] * rr;
            }
        }
#pragma unroll(MIXED ? kTileUnrollMixed : kTileUnroll)
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
#if GW_PHASOR_TABLE
                gw_phasor_table(turns_phase(cf, tb), ptab, er, ei);
#else
                gw_phasor_turns(turns_phase(cf, tb), er, ei);
#endif
            }
            if (kMasked && j > jcut) {
                er = 0.0;
                ei = 0.0;
            }
            if constexpr (kDirect) {
#pragma unroll
                for (int d = 0; d < NDET; ++d) {
                    const double2 e = ld[d * tile_bins + j];
                    const double v = lv[d * tile_bins + j];
                    // residual d/a - P_d e^{-i Phi_d}
                    double rr = __builtin_fma(-er, sr_[d], e.x);
                    rr = __builtin_fma(ei, si_[d], rr);
                    double ri = __builtin_fma(-er, si_[d], e.y);
                    ri = __builtin_fma(-ei, sr_[d], ri);
                    acc = __builtin_fma(v, __builtin_fma(rr, rr, ri * ri), acc);
                    if (d > 0) {
                        const double tr = sr_[d] * rho_re[d] - si_[d] * rho_im[d];
                        si_[d] = sr_[d] * rho_im[d] + si_[d] * rho_re[d];
                        sr_[d] = tr;
                    }
                }
            } else {
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
        }
        if (!kDirect && NDET > 1) {
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
        if (!kDirect) {
            // the chunk's share of sum_det Re(P_det Z_det), linear in Z
            acc = 0.0;
#pragma unroll
            for (int d = 0; d < NDET; ++d) {
                const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + s];
                const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + s];
                acc = __builtin_fma(pr, zr[d], acc);
                acc = __builtin_fma(-pi, zi[d], acc);
            }
        }
        reinterpret_cast<double *>(ev.partials)[chunk * n_samples + s] = acc;
    }
}

// One event.  queue == null: one block per work item (chunk, group), the grid
// being about one wave of resident blocks; blocks are dispatched round-robin
// over the 8 XCDs, and when the grid is a multiple of 8 the linear work index
// is remapped so that the blocks of one XCD cover consecutive chunks.
// queue != null: a persistent grid over kQueues work queues (counters zero
// at launch), so that blocks the wave arbiter favours, or CUs that clock
// higher, take more items and every SIMD keeps its waves until the end.
// Queue x holds the chunks c = x (mod kQueues) in index order, all sample
// groups of a chunk together; block b starts on queue b mod kQueues, which
// under round-robin dispatch is the queue of its own XCD, so a chunk's bins
// are fetched into one L2, and when its queue is empty takes items from the
// others in turn.  With the ISCO end (split form) the chunks cover only the
// bins below 1 + max K_s, read from the device, so that no block works on
// bins every template has left.
template <int NDET, bool MIXED, int FORM>
__global__ __launch_bounds__(kBlock) GW_TILE_ATTR void lnl_tile_kernel(EventView ev, int n_groups, int n_chunks,
                                                                       int rounds, int tile_bins,
                                                                       unsigned *__restrict__ queue)
{
    extern __shared__ double4 lds_raw[];
    __shared__ int next_chunk, next_group;
    const int64_t n_eff =
        FORM == kFormSplitIsco ? min(ev.n_bins, max((int64_t)0, *ev.k_limit)) : ev.n_bins;
    double *const tiles = stage_phasor_table<MIXED>(lds_raw);
    if (queue == nullptr) {
        const unsigned nb = gridDim.x, b = blockIdx.x;
        const unsigned w = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
        int64_t k_begin, k_end;
        chunk_range(n_eff, (int64_t)(w / (unsigned)n_groups), n_chunks, rounds, k_begin, k_end);
        tile_chunk<NDET, MIXED, FORM>(ev, (int)(w % (unsigned)n_groups), (int64_t)(w / (unsigned)n_groups), k_begin,
                                      k_end, tile_bins, tiles);
        return;
    }
    const unsigned home = blockIdx.x % kQueues;
    unsigned visited = 0;                // queues found empty (thread 0)
    for (;;) {
        __syncthreads();                 // every thread has read the item and left the LDS tiles
        if (threadIdx.x == 0) {
            int chunk = -1, group = 0;
            while (visited < kQueues) {
                const unsigned x = (home + visited) % kQueues;
                const int k = (int)atomicAdd(queue + x, 1u);
                if (queue_item((int)x, k, n_groups, n_chunks, chunk, group)) break;
                ++visited;
            }
            next_chunk = chunk;
            next_group = group;
        }
        __syncthreads();
        const int chunk = next_chunk;
        if (chunk < 0) break;
        int64_t k_begin, k_end;
        chunk_range(n_eff, chunk, n_chunks, rounds, k_begin, k_end);
        tile_chunk<NDET, MIXED, FORM>(ev, next_group, chunk, k_begin, k_end, tile_bins, tiles);
    }
}

// Many events: a persistent grid.  Every block repeatedly takes the next work
// item (event, sample group, bin chunk) from a device counter until the list
// is exhausted; the list is sorted by decreasing cost, so the large items go
// first and the small ones fill the tail.  The counter must be zero at launch.
template <int NDET, bool MIXED, int FORM>
__global__ __launch_bounds__(kBlock) GW_TILE_ATTR void lnl_ragged_kernel(const RaggedEvent *__restrict__ events,
                                                                         const WorkItem *__restrict__ items,
                                                                         int n_items, unsigned *__restrict__ counter,
                                                                         int tile_bins)
{
    extern __shared__ double4 lds_raw[];
    __shared__ int next;
    double *const tiles = stage_phasor_table<MIXED>(lds_raw);
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
        ev.edir = re.edir;
        ev.vdir = re.vdir;
        ev.rec = re.rec;
        ev.k_limit = nullptr;
        ev.partials = re.partials;
        const int64_t k_begin = (int64_t)wi.chunk * re.chunk_bins;
        const int64_t k_end = min(re.n_bins, k_begin + re.chunk_bins);
        tile_chunk<NDET, MIXED, FORM>(ev, wi.group, wi.chunk, k_begin, k_end, tile_bins, tiles);
    }
}

// lnL of row s from its chunk totals: split forms -1/2 <d,d> + sum_det
// [Re(P Z_det) - 1/2 |P|^2 Q_det], Q_det from the event sums or, with the
// ISCO end, 4 df times the prefix sum of a^2/S up to K_s; direct form -2 df
// times the residual sum.  GW_FLAG_ADD_NORM subtracts sum ln(2 pi S).
// sums: the event-wide totals of |d|^2/S, a^2/S, ln(2 pi S) per detector.
__device__ __forceinline__ double assemble_row(int64_t s, int64_t n_samples, int n_det, int64_t n_bins, double df,
                                               unsigned flags, double total, const double *__restrict__ rec,
                                               const double *__restrict__ sums, const double *__restrict__ qprefix)
{
    double dd = 0.0, norm = 0.0;
    for (int d = 0; d < n_det; ++d) {
        dd += sums[kPrepPerDet * d];
        norm += sums[kPrepPerDet * d + 2];
    }
    dd *= 4.0 * df;
    double out;
    if (flags & GW_FLAG_DIRECT) {
        out = -2.0 * df * total;
    } else {
        const bool isco = (flags & GW_FLAG_TERM_ISCO) != 0;
        const int64_t kcut = (int64_t)rec[kRecKcut * n_samples + s];
        double acc = -0.5 * dd + total;
        for (int d = 0; d < n_det; ++d) {
            const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + s];
            const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + s];
            double q = 4.0 * df * sums[kPrepPerDet * d + 1];
            if (isco) q = kcut >= 0 ? 4.0 * df * qprefix[(int64_t)d * n_bins + kcut] : 0.0;
            acc -= 0.5 * (pr * pr + pi * pi) * q;
        }
        out = acc;
    }
    if (flags & GW_FLAG_ADD_NORM) out -= norm;
    const int status = (int)rec[kRecStatus * n_samples + s];
    if (status == 1) out = -INFINITY;
    if (status == 2 || isnan(dd)) out = NAN;
    return out;
}

// Row s with its chunks summed in order (one thread per row).
__device__ __forceinline__ double finalize_row(int64_t s, int64_t n_samples, int n_det, int n_chunks,
                                               int64_t n_bins, double df, unsigned flags,
                                               const double2 *__restrict__ partials, const double *__restrict__ rec,
                                               const double *__restrict__ sums, const double *__restrict__ qprefix)
{
    const double *pd = reinterpret_cast<const double *>(partials);
    double total = 0.0;
    for (int c = 0; c < n_chunks; ++c) total += pd[(int64_t)c * n_samples + s];
    return assemble_row(s, n_samples, n_det, n_bins, df, flags, total, rec, sums, qprefix);
}

// One event: 16 rows per block, 16 threads per row; thread part p sums the
// chunk totals p, p + 16, ... in order, then the parts are added in order
// 0..15.
constexpr int kFinRows = 16, kFinParts = kBlock / kFinRows;

__global__ __launch_bounds__(kBlock) void lnl_finalize_kernel(int64_t n_samples, int n_det, int n_chunks,
                                                               int64_t n_bins, double df, unsigned flags,
                                                               const double2 *__restrict__ partials,
                                                               const double *__restrict__ rec,
                                                               const double *__restrict__ sums,
                                                               const double *__restrict__ qprefix,
                                                               double *__restrict__ lnl)
{
    __shared__ double red[kFinParts][kFinRows];
    const int r = threadIdx.x % kFinRows, part = threadIdx.x / kFinRows;
    const int64_t s = (int64_t)blockIdx.x * kFinRows + r;
    if (s < n_samples) {
        const double *pd = reinterpret_cast<const double *>(partials);
        double acc = 0.0;
        for (int c = part; c < n_chunks; c += kFinParts) acc += pd[(int64_t)c * n_samples + s];
        red[part][r] = acc;
    }
    __syncthreads();
    if (part != 0 || s >= n_samples) return;
    double total = 0.0;
    for (int p = 0; p < kFinParts; ++p) total += red[p][r];
    lnl[s] = assemble_row(s, n_samples, n_det, n_bins, df, flags, total, rec, sums, qprefix);
}

// Ragged batch: block (event, group) finalizes the group's rows.
__global__ __launch_bounds__(kBlock) void ragged_finalize_kernel(const RaggedEvent *__restrict__ events,
                                                                  const int2 *__restrict__ groups, unsigned flags)
{
    const int2 eg = groups[blockIdx.x];
    const RaggedEvent &re = events[eg.x];
    const int64_t s = (int64_t)eg.y * kBlock + threadIdx.x;
    if (s >= re.n_samples) return;
    re.lnl[s] = finalize_row(s, re.n_samples, re.n_det, re.n_chunks, re.n_bins, re.df, flags, re.partials, re.rec,
                             re.sums, re.qprefix);
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
                             const EventBuffers &eb, unsigned flags, const SamplePrep *sp, hipStream_t stream)
{
    PrepView v;
    v.n_bins = grid.n_bins;
    v.n_det = n_det;
    v.df = grid.delta_f;
    v.data = reinterpret_cast<const double2 *>(data);
    v.psd = psd;
    v.tab2 = eb.tab2;
    v.dcoef = eb.dcoef;
    v.edir = eb.edir;
    v.vdir = eb.vdir;
    const int direct = (flags & GW_FLAG_DIRECT) ? 1 : 0, norm = (flags & GW_FLAG_ADD_NORM) ? 1 : 0;
    SamplePrep none{};
    const int sample_blocks = sp ? (int)grid_blocks(sp->n_samples, 1 << 30) : 0;
    hipLaunchKernelGGL(event_data_kernel, dim3(eb.prep_blocks + sample_blocks), dim3(kBlock), 0, stream, v, direct,
                       norm, eb.prep, sample_blocks, grid.f_low, sp ? *sp : none);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(event_sums_kernel, dim3(kPrepPerDet * n_det), dim3(kBlock), 0, stream, eb.prep_blocks, n_det,
                       eb.prep, eb.sums, eb.queue);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (flags & GW_FLAG_TERM_ISCO) {
        hipLaunchKernelGGL(event_offsets_kernel, dim3(n_det), dim3(kBlock), 0, stream, (int64_t)eb.prep_blocks, n_det,
                           eb.prep, eb.qoffsets);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(event_prefix_kernel, dim3(eb.prep_blocks), dim3(kBlock), 0, stream, v,
                           (int64_t)eb.prep_blocks, eb.qoffsets, eb.qprefix);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_sample_prep(const gw_grid &grid, int64_t n_samples, int n_param, int n_out, bool polarisations,
                              bool isco, const DetGeom &geom, const double *theta, double *records,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(sample_prep_kernel, dim3(grid_blocks(n_samples, 1 << 30)), dim3(kBlock), 0, stream,
                       grid.f_low, grid.delta_f, grid.n_bins, n_samples, n_param, n_out, polarisations ? 1 : 0,
                       isco ? 1 : 0, geom, theta, records);
    return hipGetLastError();
}

hipError_t launch_isco_limit(int64_t n_samples, const double *records, int64_t *k_limit, hipStream_t stream)
{
    hipLaunchKernelGGL(isco_limit_kernel, dim3(1), dim3(kBlock), 0, stream, n_samples, records, k_limit);
    return hipGetLastError();
}

size_t lnl_tile_lds_bytes(int n_det, int tile_bins, int form, bool mixed)
{
    return tile_lds_bytes(n_det, tile_bins, form, mixed);
}

template <int NDET, bool MIXED>
static const void *tile_kernel_form(int form)
{
    switch (form) {
    case kFormSplit: return reinterpret_cast<const void *>(&lnl_tile_kernel<NDET, MIXED, kFormSplit>);
    case kFormSplitIsco: return reinterpret_cast<const void *>(&lnl_tile_kernel<NDET, MIXED, kFormSplitIsco>);
    default: return reinterpret_cast<const void *>(&lnl_tile_kernel<NDET, MIXED, kFormDirect>);
    }
}

template <int NDET, bool MIXED>
static const void *ragged_kernel_form(int form)
{
    switch (form) {
    case kFormSplit: return reinterpret_cast<const void *>(&lnl_ragged_kernel<NDET, MIXED, kFormSplit>);
    case kFormSplitIsco: return reinterpret_cast<const void *>(&lnl_ragged_kernel<NDET, MIXED, kFormSplitIsco>);
    default: return reinterpret_cast<const void *>(&lnl_ragged_kernel<NDET, MIXED, kFormDirect>);
    }
}

// The kernel (tile or ragged) for a detector count, precision and form.
static const void *kernel_for(bool ragged, int n_det, bool mixed, int form)
{
#define GW_KERNEL_CASE(N)                                                                                        \
    case N:                                                                                                    \
        if (ragged) return mixed ? ragged_kernel_form<N, true>(form) : ragged_kernel_form<N, false>(form);      \
        return mixed ? tile_kernel_form<N, true>(form) : tile_kernel_form<N, false>(form);
    switch (n_det) {
        GW_KERNEL_CASE(1)
        GW_KERNEL_CASE(2)
        GW_KERNEL_CASE(3)
        GW_KERNEL_CASE(4)
        GW_KERNEL_CASE(5)
        GW_KERNEL_CASE(6)
        GW_KERNEL_CASE(7)
        GW_KERNEL_CASE(8)
    default: return nullptr;
    }
#undef GW_KERNEL_CASE
}

static int occupancy(const void *fn, size_t lds)
{
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kBlock, lds) != hipSuccess) return 1;
    return n < 1 ? 1 : n;
}

int lnl_tile_blocks_per_cu(int n_det, int tile_bins, bool mixed, int form)
{
    return occupancy(kernel_for(false, n_det, mixed, form), tile_lds_bytes(n_det, tile_bins, form, mixed));
}

int lnl_ragged_blocks_per_cu(int n_det, int tile_bins, bool mixed, int form)
{
    return occupancy(kernel_for(true, n_det, mixed, form), tile_lds_bytes(n_det, tile_bins, form, mixed));
}

hipError_t launch_lnl_tiles(const gw_grid &grid, int n_det, int64_t n_samples, const TilePlan &plan, bool mixed,
                            int form, const EventBuffers &eb, const double *records, double2 *partials,
                            hipStream_t stream)
{
    EventView ev;
    ev.n_bins = grid.n_bins;
    ev.n_samples = n_samples;
    ev.f_low = grid.f_low;
    ev.df = grid.delta_f;
    ev.tab1 = eb.tab1;
    ev.dcoef = eb.dcoef;
    ev.edir = eb.edir;
    ev.vdir = eb.vdir;
    ev.rec = records;
    ev.k_limit = eb.k_limit;
    ev.partials = partials;
    const void *fn = kernel_for(false, n_det, mixed, form);
    if (!fn) return hipErrorInvalidValue;
    int n_groups = plan.n_groups, n_chunks = plan.n_chunks, rounds = plan.rounds, tile_bins = plan.tile_bins;
    unsigned *queue = plan.rounds > 0 ? eb.queue : nullptr;
    if (plan.rounds > 0 && !queue) return hipErrorInvalidValue;
    void *args[] = {&ev, &n_groups, &n_chunks, &rounds, &tile_bins, &queue};
    return hipLaunchKernel(fn, dim3((unsigned)plan.blocks), dim3(kBlock), args,
                           tile_lds_bytes(n_det, plan.tile_bins, form, mixed), stream);
}

hipError_t launch_ragged(const RaggedLaunch &r, hipStream_t stream)
{
    const int direct = (r.flags & GW_FLAG_DIRECT) ? 1 : 0, norm = (r.flags & GW_FLAG_ADD_NORM) ? 1 : 0;
    const int form = tile_form(r.flags);
    hipLaunchKernelGGL(ragged_event_prep_kernel, dim3(r.n_prep_blocks), dim3(kBlock), 0, stream, r.events,
                       r.block_map, direct, norm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ragged_event_sums_kernel, dim3(r.n_events), dim3(kBlock), 0, stream, r.events);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (r.flags & GW_FLAG_TERM_ISCO) {
        hipLaunchKernelGGL(ragged_offsets_kernel, dim3(r.n_events), dim3(kBlock), 0, stream, r.events);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(ragged_prefix_kernel, dim3(r.n_prep_blocks), dim3(kBlock), 0, stream, r.events,
                           r.block_map);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ragged_sample_prep_kernel, dim3(r.n_groups), dim3(kBlock), 0, stream, r.events, r.groups,
                       r.geoms, r.n_param, (r.flags & GW_FLAG_TERM_ISCO) ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, stream, r.counters, kMaxDet);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int i = 0; i < r.n_classes; ++i) {
        const RaggedClass &c = r.classes[i];
        const void *fn = kernel_for(true, c.n_det, r.mixed, form);
        if (!fn) return hipErrorInvalidValue;
        const RaggedEvent *events = r.events;
        const WorkItem *items = c.items;
        int n_items = c.n_items, tile_bins = r.tile_bins;
        unsigned *counter = c.counter;
        void *args[] = {&events, &items, &n_items, &counter, &tile_bins};
        e = hipLaunchKernel(fn, dim3(c.grid), dim3(kBlock), args,
                            tile_lds_bytes(c.n_det, r.tile_bins, form, r.mixed), stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ragged_finalize_kernel, dim3(r.n_groups), dim3(kBlock), 0, stream, r.events, r.groups,
                       r.flags);
    return hipGetLastError();
}

hipError_t launch_lnl_finalize(const gw_grid &grid, int64_t n_samples, int n_det, const TilePlan &plan,
                               const double2 *partials, const double *records, const EventBuffers &eb,
                               unsigned flags, double *lnl_out, hipStream_t stream)
{
    const int64_t blocks = (n_samples + kFinRows - 1) / kFinRows;
    hipLaunchKernelGGL(lnl_finalize_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, n_samples, n_det,
                       plan.n_chunks, grid.n_bins, grid.delta_f, flags, partials, records, eb.sums, eb.qprefix,
                       lnl_out);
    return hipGetLastError();
}


}  // namespace gw

GW_DEFINE_SOURCE_HASH(kernels)
