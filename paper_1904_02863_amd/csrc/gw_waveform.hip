// The waveform kernel of gw_waveform_batch (the template of Sec. II of
// arXiv:1904.02863 written out for every sample, detector and bin), kept in
// its own translation unit: it shares the tables, records and phase
// evaluation of the likelihood kernels (gw_template.h) but none of their
// launch planning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gw_build_id.h"
#include "gw_device_math.h"
#include "gw_internal.h"
#include "gw_template.h"

namespace gw {

// ---------------------------------------------------------------- waveform materialisation
// h[s][ch][k] = a_k P_ch e^{-i Phi_0,k} e^{-2 pi i f_k delta_ch} for k <= K_s
// (zero above the template end).  Block (span of kWaveBins bins, group of
// kWaveSamples samples): thread t holds the tables of bins span + t + kBlock j,
// j < kWaveSteps, in registers and writes them for every sample of the group,
// so the tables are read once per group rather than once per sample (read
// per sample they cost as many bytes as the output at 256 samples), and
// every store instruction of a wave covers 64 consecutive bins.  A sample's
// record is the same for the whole block (scalar loads).  The delay phasor of
// each channel is evaluated exactly at the thread's first bin and advanced by
// the fixed rotation e^{-2 pi i kBlock df delta} to its next bins.
// Work items (span, group) are ordered span-major, every group of a span
// after the other, and dealt to the XCDs in contiguous runs: the grid is a
// multiple of 8 and block b, which the dispatcher places on XCD b mod 8,
// takes item (b mod 8) (grid / 8) + b / 8.  The groups of one span then run
// one after the other on one XCD and read the span's tables from its L2, so
// the tables come from memory about once per launch instead of once per group.
constexpr int kWaveSteps = 4;
constexpr int kWaveBins = kBlock * kWaveSteps;
#ifndef GW_WAVE_SAMPLES
#define GW_WAVE_SAMPLES 4
#endif
constexpr int kWaveSamples = GW_WAVE_SAMPLES;

__global__ __launch_bounds__(kBlock) void waveform_kernel(int64_t n_bins, int n_out, int64_t n_samples,
                                                           int64_t n_spans, int64_t n_groups, double df,
                                                           const Tab1 *__restrict__ tab1,
                                                           const Tab2 *__restrict__ tab2,
                                                           const double *__restrict__ rec,
                                                           double2 *__restrict__ h_out)
{
    const int64_t per_xcd = (int64_t)gridDim.x / 8;
    const int64_t item = (int64_t)(blockIdx.x % 8u) * per_xcd + (int64_t)(blockIdx.x / 8u);
    if (item >= n_spans * n_groups) return;
    const int64_t span = item / n_groups;
    const int64_t s0 = (item % n_groups) * kWaveSamples;
    const int64_t k0 = span * kWaveBins + threadIdx.x;
    if (k0 >= n_bins) return;
    Tab1 t[kWaveSteps];
    double amp[kWaveSteps];
#pragma unroll
    for (int j = 0; j < kWaveSteps; ++j) {
        const int64_t k = min(k0 + (int64_t)kBlock * j, n_bins - 1);
        t[j] = tab1[k];
        amp[j] = tab2[k].amp;
    }
    const double f0 = tab2[k0].f;
    const int64_t s_end = min(s0 + (int64_t)kWaveSamples, n_samples);
    for (int64_t s = s0; s < s_end; ++s) {
        const int status = (int)rec[kRecStatus * n_samples + s];
        const int64_t kcut = (int64_t)rec[kRecKcut * n_samples + s];
        const PhaseCoef cf = load_coef(rec, n_samples, s);
        double er[kWaveSteps], ei[kWaveSteps];
#pragma unroll
        for (int j = 0; j < kWaveSteps; ++j) gw_phasor_turns(turns_phase(cf, t[j]), er[j], ei[j]);
        for (int d = 0; d < n_out; ++d) {
            const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + s];
            const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + s];
            const double delta = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + s];
            // T = P e^{-2 pi i f delta} at the thread's first bin; step rotation
            double rr = 1.0, ri = 0.0, sr = 1.0, si = 0.0;
            if (delta != 0.0) {
                gw_phasor_turns(f0 * delta, rr, ri);
                gw_phasor_turns((double)kBlock * df * delta, sr, si);
            }
            double tr = pr * rr - pi * ri, ti = pr * ri + pi * rr;
            double2 *out = h_out + ((int64_t)s * n_out + d) * n_bins;
#pragma unroll
            for (int j = 0; j < kWaveSteps; ++j) {
                const int64_t k = k0 + (int64_t)kBlock * j;
                if (k < n_bins) {
                    double2 h;
                    h.x = amp[j] * (tr * er[j] - ti * ei[j]);
                    h.y = amp[j] * (tr * ei[j] + ti * er[j]);
                    if (k > kcut) h = make_double2(0.0, 0.0);
                    if (status != 0) h = make_double2(NAN, NAN);
                    out[k] = h;
                }
                const double nr = tr * sr - ti * si;
                ti = tr * si + ti * sr;
                tr = nr;
            }
        }
    }
}

hipError_t launch_waveform(const gw_grid &grid, int n_out, int64_t n_samples, const Tab1 *tab1, const Tab2 *tab2,
                           const double *records, gw_c128 *h_out, hipStream_t stream)
{
    const int64_t spans = (grid.n_bins + kWaveBins - 1) / kWaveBins;
    const int64_t groups = (n_samples + kWaveSamples - 1) / kWaveSamples;
    const int64_t blocks = (spans * groups + 7) / 8 * 8;     // a multiple of the 8 XCDs
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(waveform_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, grid.n_bins, n_out,
                       n_samples, spans, groups, grid.delta_f, tab1, tab2, records,
                       reinterpret_cast<double2 *>(h_out));
    return hipGetLastError();
}

// out[i] = v for i < n: a plain store stream with the waveform kernel's
// pattern (16-byte stores, a wave covering 64 consecutive elements), the
// write ceiling the waveform kernel is measured against.
__global__ __launch_bounds__(kBlock) void fill_c128_kernel(int64_t n, double2 v, double2 *__restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) out[i] = v;
}

hipError_t launch_fill_c128(int64_t n, double re, double im, gw_c128 *out, int n_cu, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)n_cu * 16);
    hipLaunchKernelGGL(fill_c128_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, n, make_double2(re, im),
                       reinterpret_cast<double2 *>(out));
    return hipGetLastError();
}

}  // namespace gw

GW_DEFINE_SOURCE_HASH(waveform)
