// Relative binning (Zackay, Dai & Venumadhav 2018) for the likelihood of
// Eq. (cbclike): the route to long signals that Secs. I and V of
// arXiv:1904.02863 name beside GPU waveforms.  About 10^3 unevenly spaced
// frequencies stand for the whole grid, and no exponential over the grid is
// evaluated per sample.
//
// With the fiducial template h0 (parameters theta0) the ratio on detector d,
//     r_d(f) = h_d(f; theta) / h0_d(f)
//            = (P_d / P0_d) e^{-2 pi i [dPhi_0(f) + f (delta_d - delta0_d)]},
// needs no amplitude (f^-7/6 cancels) and only the phase difference at
// detector 0, dPhi_0 = Phi_0(theta) - Phi_0(theta0).  Phi_0 is linear in the
// record's coefficients, so dPhi_0 is the same Horner polynomial evaluated
// with the differences of the two records' coefficients: a small number of
// turns near the fiducial, evaluated with the same absolute accuracy.
// Within a bin r is taken as linear between its values at the two edges, and
// the bin's share of <d, h> - <h, h>/2 is a quadratic form in those two
// values whose coefficients come from the summary data A0, A1, B0, B1, B2
// (sums over the fiducial template, formed once per event by
// summary_kernel).  Written per edge (coef_kernel), the two bins that meet at
// an edge share one linear and one squared term, so a sample pays, per edge
// and detector, one phasor and eight more floating-point operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gw_build_id.h"
#include "gw_device_math.h"
#include "gw_internal.h"
#include "gw_template.h"

// Blocks per compute unit the per-sample pass is sized for; 0 asks the
// runtime for the kernel's occupancy limit.
#ifndef GW_RB_BLOCKS_PER_CU
#define GW_RB_BLOCKS_PER_CU 0
#endif

namespace gw {
namespace rb {

namespace {

// Sums v[0..N-1] over the block: wave butterflies, then the four waves in a
// fixed order.  The totals are valid in thread 0; `red` holds 4 N doubles.
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double *red)
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) red[wave * N + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = ((red[i] + red[N + i]) + red[2 * N + i]) + red[3 * N + i];
    __syncthreads();
}

// ---------------------------------------------------------------- event preparation
__global__ __launch_bounds__(kBlock) void edges_kernel(double f_low, double df, int64_t n_edges,
                                                        const int64_t *__restrict__ idx, RbEdge *__restrict__ edges)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_edges) return;
    RbEdge e;
    Tab2 t2;
    freq_tables(bin_frequency(f_low, df, idx[i]), e.t1, t2);
    e.f = t2.f;
    e.pad[0] = e.pad[1] = e.pad[2] = 0.0;
    edges[i] = e;
}

// One block per bin b: the summary data of every detector over the grid bins
// k in [e_b, e_{b+1}) (the last bin also e_B), with w = 4 df / S and the
// fiducial h0 = a P0 e^{-2 pi i (Phi_0 + f delta0)}:
//   A0 = sum w d conj(h0), A1 = sum w d conj(h0) (f - fm), B0 = sum w |h0|^2,
//   B1 = sum w |h0|^2 (f - fm), B2 = sum w |h0|^2 (f - fm)^2,   fm = (f_lo + f_hi)/2,
// and, over all detectors, sum w |d|^2 and sum ln(2 pi S).  A PSD value <= 0
// or non-finite makes w NaN.
__global__ __launch_bounds__(kBlock) void summary_kernel(int n_det, int64_t n_rb, int64_t n_bins, double f_low,
                                                          double df, const int64_t *__restrict__ idx,
                                                          const Tab1 *__restrict__ tab1, const Tab2 *__restrict__ tab2,
                                                          const double *__restrict__ fid,
                                                          const double2 *__restrict__ data,
                                                          const double *__restrict__ psd, double *__restrict__ raw,
                                                          double *__restrict__ bin_dd)
{
    __shared__ double red[4 * kRawPerDet];
    const int64_t b = blockIdx.x;
    const int64_t lo = idx[b], up = idx[b + 1];
    const int64_t last = b == n_rb - 1 ? up : up - 1;
    const double fm = 0.5 * (bin_frequency(f_low, df, lo) + bin_frequency(f_low, df, up));
    const PhaseCoef cf = load_coef(fid, 1, 0);
    const double wscale = 4.0 * df;
    double dd = 0.0, nrm = 0.0;
    for (int d = 0; d < n_det; ++d) {
        const double pr = fid[kRecDet + kRecFieldsPerDet * d];
        const double pi = fid[kRecDet + kRecFieldsPerDet * d + 1];
        const double delta = fid[kRecDet + kRecFieldsPerDet * d + 2];
        const double2 *__restrict__ dd_row = data + (int64_t)d * n_bins;
        const double *__restrict__ s_row = psd + (int64_t)d * n_bins;
        double v[kRawPerDet] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t k = lo + threadIdx.x; k <= last; k += kBlock) {
            const Tab1 t1 = tab1[k];
            const Tab2 t2 = tab2[k];
            double er, ei;
            gw_phasor_turns(__builtin_fma(t2.f, delta, turns_phase(cf, t1)), er, ei);
            const double hr = t2.amp * (pr * er - pi * ei);
            const double hi = t2.amp * (pr * ei + pi * er);
            const double s = s_row[k];
            const double w = (s > 0.0 && s < INFINITY) ? wscale / s : NAN;
            const double2 dk = dd_row[k];
            const double xr = w * (dk.x * hr + dk.y * hi);
            const double xi = w * (dk.y * hr - dk.x * hi);
            const double y = w * (hr * hr + hi * hi);
            const double x = t2.f - fm;
            v[0] += xr;
            v[1] += xi;
            v[2] += xr * x;
            v[3] += xi * x;
            v[4] += y;
            v[5] += y * x;
            v[6] += y * x * x;
            dd += w * (dk.x * dk.x + dk.y * dk.y);
            nrm += log(2.0 * GW_PI * s);
        }
        block_reduce(v, red);
        if (threadIdx.x == 0) {
            double *r = raw + (b * n_det + d) * kRawPerDet;
#pragma unroll
            for (int i = 0; i < kRawPerDet; ++i) r[i] = v[i];
        }
    }
    double t[2] = {dd, nrm};
    block_reduce(t, red);
    if (threadIdx.x == 0) {
        bin_dd[2 * b] = t[0];
        bin_dd[2 * b + 1] = t[1];
    }
}

// One thread per (edge e, detector): the coefficients of the ratio at e from
// the summary data of the bins that end (e - 1) and start (e) there; see
// RbCoef.  Edge 0 has no bin below it and edge B none above.
__global__ __launch_bounds__(kBlock) void coef_kernel(int n_det, int64_t n_rb, const RbEdge *__restrict__ edges,
                                                       const double *__restrict__ raw, RbCoef *__restrict__ coef,
                                                       RbEnds *__restrict__ ends)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (n_rb + 1) * n_det) return;
    const int64_t e = i / n_det;
    const int d = (int)(i % n_det);
    RbEnds x;
    x.hi_r = x.hi_i = x.hi_q = x.lo_r = x.lo_i = x.lo_q = x.qcum = x.pad1 = 0.0;
    double xb = 0.0;
    if (e >= 1) {          // bin e - 1 ends at e
        const double *v = raw + ((e - 1) * n_det + d) * kRawPerDet;
        const double w = edges[e].f - edges[e - 1].f;
        x.hi_r = __builtin_fma(0.5, v[0], v[2] / w);
        x.hi_i = __builtin_fma(0.5, v[1], v[3] / w);
        x.hi_q = -0.125 * v[4] - 0.5 * v[6] / (w * w) - 0.5 * v[5] / w;
        xb = -0.25 * v[4] + v[6] / (w * w);
    }
    if (e < n_rb) {        // bin e starts at e
        const double *v = raw + (e * n_det + d) * kRawPerDet;
        const double w = edges[e + 1].f - edges[e].f;
        x.lo_r = __builtin_fma(0.5, v[0], -v[2] / w);
        x.lo_i = __builtin_fma(0.5, v[1], -v[3] / w);
        x.lo_q = -0.125 * v[4] - 0.5 * v[6] / (w * w) + 0.5 * v[5] / w;
    }
    RbCoef c;
    c.lr = x.hi_r + x.lo_r;
    c.li = x.hi_i + x.lo_i;
    c.q = x.hi_q + x.lo_q;
    c.xb = xb;
    coef[i] = c;
    ends[i] = x;
}

// One block per detector d: ends[e].qcum = sum of coef[e'].q over e' < e, in
// a fixed order (each thread a contiguous run of edges, then the runs' sums
// in thread order), for e = 0 .. n_rb.
__global__ __launch_bounds__(kBlock) void qcum_kernel(int n_det, int64_t n_rb, const RbCoef *__restrict__ coef,
                                                       RbEnds *__restrict__ ends)
{
    __shared__ double run[kBlock];
    const int d = blockIdx.x;
    const int64_t n = n_rb + 1;
    const int64_t per = (n + kBlock - 1) / kBlock;
    const int64_t e0 = min(n, (int64_t)threadIdx.x * per), e1 = min(n, e0 + per);
    double acc = 0.0;
    for (int64_t e = e0; e < e1; ++e) acc += coef[e * n_det + d].q;
    run[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int t = 0; t < kBlock; ++t) {
            const double v = run[t];
            run[t] = sum;
            sum += v;
        }
    }
    __syncthreads();
    double prefix = run[threadIdx.x];
    for (int64_t e = e0; e < e1; ++e) {
        ends[e * n_det + d].qcum = prefix;
        prefix += coef[e * n_det + d].q;
    }
}

// One block: totals[0] = <d, d>, totals[1] = sum ln(2 pi S) from the per-bin
// sums (each thread a strided set of bins, then the fixed block tree).
__global__ __launch_bounds__(kBlock) void totals_kernel(int64_t n_rb, const double *__restrict__ bin_dd,
                                                         double *__restrict__ totals)
{
    __shared__ double red[4 * 2];
    double t[2] = {0.0, 0.0};
    for (int64_t b = threadIdx.x; b < n_rb; b += kBlock) {
        t[0] += bin_dd[2 * b];
        t[1] += bin_dd[2 * b + 1];
    }
    block_reduce(t, red);
    if (threadIdx.x == 0) {
        totals[0] = t[0];
        totals[1] = t[1];
    }
}

// ---------------------------------------------------------------- per-sample pass
// Block (sample group g, chunk c): thread t takes sample 256 g + t over the
// bins [b0, b1) of chunk c, i.e. the edges b0 .. b1.  The items (g, c) are
// dealt to the XCDs in contiguous runs, the chunks of a group one after the
// other: the grid is a multiple of 8 and block b, which the dispatcher places
// on XCD b mod 8, takes item (b mod 8) (grid / 8) + b / 8, so the chunk blocks
// of a group share one L2 and read the group's sample records from memory
// once.  The ratio is formed
// once per edge; each edge adds its linear and squared terms (one-sided at
// the chunk's two end edges, whose other bin belongs to the next chunk) and
// the cross term of the bin below it.  The squared terms need no per-edge
// work: r_d = q_d e^{-2 pi i x} has |r_d|^2 = |q_d|^2 at every edge, so they
// add |q_d|^2 times the chunk's sum of the squared-term coefficients (from
// the prefix sums qcum and the one-sided end coefficients).  The edge tables
// and coefficients are
// the same for every lane of a wave (the loop index is uniform), so they come
// through the scalar cache.  Writes the chunk's partial sum of
// <d, h> - <h, h>/2 for every sample.
// MIXED: the phase difference and its reduction to a fractional turn stay
// FP64, the phasor comes from the FP32 hardware sine and cosine (inputs in
// turns), and the ratio and every sum stay FP64.
// FP64: the phase comes in scaled by GW_PHTAB_N (coefficients and delay
// differences scaled at load) and the phasor from the LDS table tab.
// The template's phasor e_d = e^{-2 pi i x_d} at edge e for every detector:
// x_0 the phase difference from the fiducial waveform at the edge, x_d =
// x_0 + f_e (delta_d - delta_d^0) for the others (in turns, scaled by the
// table size on the FP64 path).  The ratio to the fiducial waveform is
// r_d = q_d e_d, q_d = P_d / P_d^0.
template <int NDET, bool MIXED>
__device__ __forceinline__ void edge_phasor(const PhaseCoef &c, const RbEdge &e, const double (&dl)[NDET],
                                            double (&er)[NDET], double (&ei)[NDET], const double2 *tab)
{
    const double dphi = turns_phase(c, e.t1);
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const double x = d == 0 ? dphi : __builtin_fma(e.f, dl[d], dphi);
        if constexpr (MIXED) {
            const float r = (float)(x - __builtin_rint(x));
            er[d] = (double)__builtin_amdgcn_cosf(r);
            ei[d] = -(double)__builtin_amdgcn_sinf(r);
        } else {
            gw_phasor_table(x, tab, er[d], ei[d]);
        }
    }
}

// Edges per unrolled step of the relative-binning edge loop.
#ifndef GW_RB_UNROLL
#define GW_RB_UNROLL 4
#endif

template <int NDET, bool MIXED>
__global__ __launch_bounds__(kBlock) void lnl_kernel(int64_t n_samples, int64_t n_rb, int n_chunks,
                                                      const RbEdge *__restrict__ edges,
                                                      const RbCoef *__restrict__ coef, const RbEnds *__restrict__ ends,
                                                      const double *__restrict__ fid, const double *__restrict__ rec,
                                                      double *__restrict__ partials)
{
    const int64_t per_xcd = (int64_t)gridDim.x / 8;
    const int64_t item = (int64_t)(blockIdx.x % 8u) * per_xcd + (int64_t)(blockIdx.x / 8u);
    const int64_t n_groups = (n_samples + kBlock - 1) / kBlock;
    if (item >= n_groups * n_chunks) return;
    const int64_t group = item / n_chunks;
    const int chunk = (int)(item % n_chunks);
    const int64_t s = group * kBlock + threadIdx.x;
    const int64_t sr = s < n_samples ? s : n_samples - 1;
    const int64_t b0 = n_rb * chunk / n_chunks, b1 = n_rb * (chunk + 1) / n_chunks;
    __shared__ double2 tab[MIXED ? 1 : GW_PHTAB_N];
    if constexpr (!MIXED) {
        gw_stage_phasor_table(tab, kBlock);
        __syncthreads();
    }

    PhaseCoef c = load_coef(rec, n_samples, sr);
    const PhaseCoef c0 = load_coef(fid, 1, 0);
    c.c8 -= c0.c8;
    c.c7 -= c0.c7;
    c.c6 -= c0.c6;
    c.c6l -= c0.c6l;
    c.c5 -= c0.c5;
    c.c5l -= c0.c5l;
    c.c4 -= c0.c4;
    c.c3 -= c0.c3;
    c.c2 -= c0.c2;
    c.c0 -= c0.c0;
    // FP64: phase in units of 1/N turn for the table phasor (exact: N is a power of two)
    const double scale = MIXED ? 1.0 : (double)GW_PHTAB_N;
    if constexpr (!MIXED) c = scale_coef(c, scale);
    double qr[NDET], qi[NDET], dl[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const double pr = rec[(kRecDet + kRecFieldsPerDet * d) * n_samples + sr];
        const double pi = rec[(kRecDet + kRecFieldsPerDet * d + 1) * n_samples + sr];
        const double delta = rec[(kRecDet + kRecFieldsPerDet * d + 2) * n_samples + sr];
        const double p0r = fid[kRecDet + kRecFieldsPerDet * d];
        const double p0i = fid[kRecDet + kRecFieldsPerDet * d + 1];
        const double inv = 1.0 / (p0r * p0r + p0i * p0i);
        qr[d] = (pr * p0r + pi * p0i) * inv;     // P / P0
        qi[d] = (pi * p0r - pr * p0i) * inv;
        dl[d] = (delta - fid[kRecDet + kRecFieldsPerDet * d + 2]) * scale;   // zero for detector 0
    }
    // With r = q e, the linear terms Re(conj(l) r) = qr U + qi V for
    // U = sum (l_r e_r + l_i e_i), V = sum (l_i e_r - l_r e_i), and the cross
    // terms x_b Re(r_prev conj(r_next)) = |q|^2 x_b Re(e_prev conj(e_next)):
    // the sums run over the template's phasors alone and q enters once, at
    // the end.
    double er[NDET], ei[NDET], pr[NDET], pi[NDET], U[NDET], V[NDET], X[NDET];
    // first edge: the lower side of bin b0 only
    edge_phasor<NDET, MIXED>(c, edges[b0], dl, pr, pi, tab);
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const RbEnds k = ends[b0 * NDET + d];
        U[d] = __builtin_fma(k.lo_r, pr[d], k.lo_i * pi[d]);
        V[d] = __builtin_fma(k.lo_i, pr[d], -(k.lo_r * pi[d]));
        X[d] = 0.0;
    }
    // edges inside the chunk: both bins that meet there
#pragma unroll GW_RB_UNROLL
    for (int64_t e = b0 + 1; e < b1; ++e) {
        edge_phasor<NDET, MIXED>(c, edges[e], dl, er, ei, tab);
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            const RbCoef k = coef[e * NDET + d];
            X[d] = __builtin_fma(k.xb, __builtin_fma(pr[d], er[d], pi[d] * ei[d]), X[d]);
            U[d] = __builtin_fma(k.lr, er[d], __builtin_fma(k.li, ei[d], U[d]));
            V[d] = __builtin_fma(k.li, er[d], __builtin_fma(-k.lr, ei[d], V[d]));
            pr[d] = er[d];
            pi[d] = ei[d];
        }
    }
    // last edge: the upper side of bin b1 - 1 only; then the squared terms
    edge_phasor<NDET, MIXED>(c, edges[b1], dl, er, ei, tab);
    double total = 0.0;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const RbEnds k = ends[b1 * NDET + d];
        const RbEnds k0 = ends[b0 * NDET + d];
        const double xb = coef[b1 * NDET + d].xb;
        const double x = __builtin_fma(xb, __builtin_fma(pr[d], er[d], pi[d] * ei[d]), X[d]);
        const double u = __builtin_fma(k.hi_r, er[d], __builtin_fma(k.hi_i, ei[d], U[d]));
        const double v = __builtin_fma(k.hi_i, er[d], __builtin_fma(-k.hi_r, ei[d], V[d]));
        // squared-term coefficients of the chunk: the lower side of its first
        // edge, both sides of every inner edge, the upper side of its last edge
        const double qsum = (k0.lo_q + (k.qcum - ends[(b0 + 1) * NDET + d].qcum)) + k.hi_q;
        const double q2 = __builtin_fma(qr[d], qr[d], qi[d] * qi[d]);
        total += __builtin_fma(q2, qsum + x, __builtin_fma(qr[d], u, qi[d] * v));
    }
    if (s < n_samples) partials[(int64_t)chunk * n_samples + s] = total;
}

// lnL[s] = sum over chunks of the partials - <d, d>/2 (- sum ln 2 pi S), with
// the record's domain status applied.
__global__ __launch_bounds__(kBlock) void finalize_kernel(int64_t n_samples, int n_chunks,
                                                           const double *__restrict__ partials,
                                                           const double *__restrict__ rec,
                                                           const double *__restrict__ totals, int add_norm,
                                                           double *__restrict__ lnl)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_samples) return;
    double sum = 0.0;
    for (int c = 0; c < n_chunks; ++c) sum += partials[(int64_t)c * n_samples + s];
    double v = sum - 0.5 * totals[0];
    if (add_norm) v -= totals[1];
    const int status = (int)rec[kRecStatus * n_samples + s];
    if (status == 1) v = -INFINITY;
    if (status == 2) v = NAN;
    lnl[s] = v;
}

template <int NDET>
void *lnl_kernel_ptr(bool mixed)
{
    return mixed ? reinterpret_cast<void *>(&lnl_kernel<NDET, true>) : reinterpret_cast<void *>(&lnl_kernel<NDET, false>);
}

void *lnl_kernel_for(int n_det, bool mixed)
{
    switch (n_det) {
    case 1: return lnl_kernel_ptr<1>(mixed);
    case 2: return lnl_kernel_ptr<2>(mixed);
    case 3: return lnl_kernel_ptr<3>(mixed);
    case 4: return lnl_kernel_ptr<4>(mixed);
    case 5: return lnl_kernel_ptr<5>(mixed);
    case 6: return lnl_kernel_ptr<6>(mixed);
    case 7: return lnl_kernel_ptr<7>(mixed);
    default: return lnl_kernel_ptr<8>(mixed);
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_edges(const gw_grid &grid, int64_t n_edges, const int64_t *edge_idx, RbEdge *edges,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(edges_kernel, dim3((unsigned)((n_edges + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream,
                       grid.f_low, grid.delta_f, n_edges, edge_idx, edges);
    return hipGetLastError();
}

hipError_t launch_summary(const gw_grid &grid, int n_det, int64_t n_rb, const int64_t *edge_idx, const Tab1 *tab1,
                          const Tab2 *tab2, const double *fid, const gw_c128 *data, const double *psd,
                          const RbEdge *edges, double *raw, RbCoef *coef, RbEnds *ends, double *bin_dd,
                          double *totals, hipStream_t stream)
{
    hipLaunchKernelGGL(summary_kernel, dim3((unsigned)n_rb), dim3(kBlock), 0, stream, n_det, n_rb, grid.n_bins,
                       grid.f_low, grid.delta_f, edge_idx, tab1, tab2, fid,
                       reinterpret_cast<const double2 *>(data), psd, raw, bin_dd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(kBlock), 0, stream, n_rb, bin_dd, totals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t n = (n_rb + 1) * n_det;
    hipLaunchKernelGGL(coef_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, n_det, n_rb,
                       edges, raw, coef, ends);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(qcum_kernel, dim3((unsigned)n_det), dim3(kBlock), 0, stream, n_det, n_rb, coef, ends);
    return hipGetLastError();
}

int lnl_blocks_per_cu(int n_det, bool mixed)
{
    static int cache[2][kMaxDet] = {};
    if (GW_RB_BLOCKS_PER_CU > 0) return GW_RB_BLOCKS_PER_CU;
    if (n_det < 1 || n_det > kMaxDet) return 1;
    int &c = cache[mixed ? 1 : 0][n_det - 1];
    if (c == 0) {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, lnl_kernel_for(n_det, mixed), kBlock, 0) !=
                hipSuccess ||
            blocks < 1)
            blocks = 4;
        c = blocks;
    }
    return c;
}

int lnl_chunks(int64_t n_samples, int64_t n_rb, int n_det, bool mixed, int n_cu)
{
    const int64_t groups = (n_samples + kBlock - 1) / kBlock;
    // enough blocks to fill every compute unit to its occupancy limit in one
    // wave of blocks (more resident waves hide the latency of the long
    // dependent chains of the phasor polynomials), chunks of at least 16 bins
    const int64_t target = (int64_t)lnl_blocks_per_cu(n_det, mixed) * (n_cu > 0 ? n_cu : 256);
    int64_t chunks = (target + groups - 1) / groups;
    chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, n_rb / 16));
    chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, 4096));
    return (int)chunks;
}

hipError_t launch_lnl(int n_det, bool mixed, int64_t n_samples, int64_t n_rb, int n_chunks, const RbEdge *edges,
                      const RbCoef *coef, const RbEnds *ends, const double *fid, const double *rec,
                      double *partials, hipEvent_t t_start, hipEvent_t t_stop, hipStream_t stream)
{
    if (n_det < 1 || n_det > kMaxDet) return hipErrorInvalidValue;
    const int64_t groups = (n_samples + kBlock - 1) / kBlock;
    const int64_t blocks = (groups * n_chunks + 7) / 8 * 8;     // a multiple of the 8 XCDs
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    void *args[] = {&n_samples, &n_rb, &n_chunks, &edges, &coef, &ends, &fid, &rec, &partials};
    hipError_t e;
    if (t_start && (e = hipEventRecord(t_start, stream)) != hipSuccess) return e;
    e = hipLaunchKernel(lnl_kernel_for(n_det, mixed), dim3((unsigned)blocks), dim3(kBlock), args, 0, stream);
    if (e != hipSuccess) return e;
    if (t_stop && (e = hipEventRecord(t_stop, stream)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_finalize(int64_t n_samples, int n_chunks, const double *partials, const double *rec,
                           const double *totals, bool add_norm, double *lnl_out, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((n_samples + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream,
                       n_samples, n_chunks, partials, rec, totals, add_norm ? 1 : 0, lnl_out);
    return hipGetLastError();
}

}  // namespace rb
}  // namespace gw

GW_DEFINE_SOURCE_HASH(relbin)
