// Population likelihood of Eq. (poplike), Sec. IV of arXiv:1904.02863, for
// gfx950: the recycled hierarchical likelihood
//     ln L(Lambda) = sum_i ln[ (1/n) sum_j p(theta_ij | Lambda) / p(theta_ij | 0) ]
// for a batch of hyper-parameter points Lambda over the posterior samples of
// N events (n samples each), without the rate and selection factors.
//
// The population model (the paper names its three components without
// printing them): a power law plus a Gaussian peak in the primary mass on
// [m_min, m_max]; a power law in q = m2/m1 on [m_min/m1, 1]; independent Beta
// spin magnitudes; spin tilt cosines from a mixture of isotropic and two
// Gaussians centred on aligned spins, truncated to [-1, 1].  Every
// normalisation is closed-form and computed once per Lambda.
//
// Layout: samples field-major [7][N][n] (m1, q, a1, a2, cos t1, cos t2,
// ln p(theta | 0)), or prepared once into [8][N][n] (prepare_kernel: the
// logarithms and offsets that do not depend on Lambda, so that a call with
// one Lambda evaluates no per-sample logarithm).  Each block keeps 4 samples
// per thread of one event in registers and loops over every Lambda,
// whose constants it reads with wave-uniform loads; each wave writes its own
// partial sum, so the weights kernel has no barrier.  One wave per (Lambda,
// event) then sums that event's partials and takes the log of the mean, and
// a last kernel adds the events of each Lambda by a fixed tree.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "gw_build_id.h"
#include "gw_internal.h"

namespace gw {
namespace pop {

constexpr int kThreads = 256;
#ifndef GW_POP_PER_THREAD
#define GW_POP_PER_THREAD 4
#endif
constexpr int kPerThread = GW_POP_PER_THREAD;     // samples per thread, held in registers
constexpr int kPerBlock = kThreads * kPerThread;   // samples of one event per block
constexpr int kWaves = kThreads / 64;
static_assert(kThreads == 256, "the weights kernel fills its 256-entry exp table one entry per thread");

// Constants of one hyper-parameter point.
struct HyperC {
    double neg_alpha, ln_zpl;             // power law: m^-alpha / Z_pl
    double mu, inv_sigma, ln_zg;          // peak: exp(-((m - mu)/sigma)^2 / 2) / (sigma sqrt(2 pi) Z_g)
    double one_m_lam, lam;
    double mmin, mmax, ln_mmin, beta, one_p_beta;
    double ach_m1, bch_m1, ln_beta_fn;    // spin magnitudes
    double iso, xi, k1, k2, ln_zt;        // tilts
    int status;                           // 1 evaluate, 0 out of domain, -1 non-finite
    int beta_is_m1;                       // beta == -1: log normalisation of q
};

__device__ __forceinline__ double gauss_mass(double mu, double sigma, double lo, double hi)
{
    const double s = sigma * 1.4142135623730951;
    return 0.5 * (erf((hi - mu) / s) - erf((lo - mu) / s));
}

__global__ __launch_bounds__(kThreads) void hyper_kernel(int64_t n_hyper, const double *__restrict__ hyper,
                                                         HyperC *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n_hyper) return;
    const double *h = hyper + k * 12;
    const double alpha = h[0], beta = h[1], mmin = h[2], mmax = h[3], lam = h[4], mpp = h[5], sigpp = h[6];
    const double ach = h[7], bch = h[8], xi = h[9], s1 = h[10], s2 = h[11];
    HyperC c{};
    int status = 1;
    for (int i = 0; i < 12; ++i)
        if (!isfinite(h[i])) status = -1;
    if (status == 1 && (!(mmin > 0.0 && mmin < mmax) || !(sigpp > 0.0) || !(lam >= 0.0 && lam <= 1.0) ||
                        !(ach > 0.0) || !(bch > 0.0) || !(xi >= 0.0 && xi <= 1.0) || !(s1 > 0.0) || !(s2 > 0.0)))
        status = 0;
    c.status = status;
    if (status == 1) {
        // Z_pl = int m^-alpha dm over [m_min, m_max]
        const double L = log(mmax / mmin);
        const double e = 1.0 - alpha;
        const double zpl = alpha == 1.0 ? L : exp(e * log(mmin)) * expm1(e * L) / e;
        c.neg_alpha = -alpha;
        c.ln_zpl = log(zpl);
        c.mu = mpp;
        c.inv_sigma = 1.0 / sigpp;
        c.ln_zg = log(sigpp * 2.5066282746310002 * gauss_mass(mpp, sigpp, mmin, mmax));
        c.one_m_lam = 1.0 - lam;
        c.lam = lam;
        c.mmin = mmin;
        c.mmax = mmax;
        c.ln_mmin = log(mmin);
        c.beta = beta;
        c.one_p_beta = 1.0 + beta;
        c.beta_is_m1 = beta == -1.0 ? 1 : 0;
        c.ach_m1 = ach - 1.0;
        c.bch_m1 = bch - 1.0;
        c.ln_beta_fn = lgamma(ach) + lgamma(bch) - lgamma(ach + bch);
        c.iso = (1.0 - xi) / 4.0;
        c.xi = xi;
        c.k1 = 0.5 / (s1 * s1);
        c.k2 = 0.5 / (s2 * s2);
        c.ln_zt = log(s1 * 2.5066282746310002 * gauss_mass(1.0, s1, -1.0, 1.0)) +
                  log(s2 * 2.5066282746310002 * gauss_mass(1.0, s2, -1.0, 1.0));
    }
    out[k] = c;
}

// One sample's logarithms and flags, kept across the hyper-parameter loop.
struct Sample {
    double m1, ln_m1, ln_q, q, ln_a_sum, ln_1ma_sum, c1m, c2m, ln_prior;
    bool ok;   // inside every support that does not depend on Lambda
};

__device__ __forceinline__ Sample load_sample(const double *__restrict__ s, int64_t plane, int64_t idx, bool live)
{
    Sample x{};
    x.ok = false;
    if (!live) return x;
    const double m1 = s[idx], q = s[plane + idx], a1 = s[2 * plane + idx], a2 = s[3 * plane + idx];
    const double c1 = s[4 * plane + idx], c2 = s[5 * plane + idx];
    x.ln_prior = s[6 * plane + idx];
    x.ok = m1 > 0.0 && q > 0.0 && q <= 1.0 && a1 >= 0.0 && a1 <= 1.0 && a2 >= 0.0 && a2 <= 1.0 &&
           fabs(c1) <= 1.0 && fabs(c2) <= 1.0 && isfinite(x.ln_prior);
    if (!x.ok) return x;
    x.m1 = m1;
    x.ln_m1 = log(m1);
    x.q = q;
    x.ln_q = log(q);
    x.ln_a_sum = log(a1) + log(a2);
    x.ln_1ma_sum = log1p(-a1) + log1p(-a2);
    x.c1m = c1 - 1.0;
    x.c2m = c2 - 1.0;
    return x;
}

// Prepared samples, field-major [kPrepFields][N][n]: the part of load_sample
// that does not depend on Lambda, computed once (gw_pop_prepare).  A sample
// outside the Lambda-independent supports carries m1 = -1, which every
// population's mass support rejects.
constexpr int kPrepFields = 8;   // m1, ln m1, ln q, ln a1 + ln a2, ln(1-a1) + ln(1-a2), c1 - 1, c2 - 1, ln prior

__device__ __forceinline__ Sample load_prepared(const double *__restrict__ p, int64_t plane, int64_t idx, bool live)
{
    Sample x{};
    x.ok = false;
    if (!live) return x;
    x.m1 = p[idx];
    x.ok = x.m1 > 0.0;
    x.ln_m1 = p[plane + idx];
    x.ln_q = p[2 * plane + idx];
    x.ln_a_sum = p[3 * plane + idx];
    x.ln_1ma_sum = p[4 * plane + idx];
    x.c1m = p[5 * plane + idx];
    x.c2m = p[6 * plane + idx];
    x.ln_prior = p[7 * plane + idx];
    return x;
}

__global__ __launch_bounds__(kThreads) void prepare_kernel(int64_t plane, const double *__restrict__ s,
                                                           double *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= plane) return;
    const Sample x = load_sample(s, plane, i, true);
    p[i] = x.ok ? x.m1 : -1.0;
    p[plane + i] = x.ok ? x.ln_m1 : 0.0;
    p[2 * plane + i] = x.ok ? x.ln_q : 0.0;
    p[3 * plane + i] = x.ok ? x.ln_a_sum : 0.0;
    p[4 * plane + i] = x.ok ? x.ln_1ma_sum : 0.0;
    p[5 * plane + i] = x.ok ? x.c1m : 0.0;
    p[6 * plane + i] = x.ok ? x.c2m : 0.0;
    p[7 * plane + i] = x.ok ? x.ln_prior : 0.0;
}

// e^x for finite x from the table t[j] = 2^(j/256) (LDS, 256 entries): with
// k = rint(256 x / ln 2) (the round-to-integer of adding 1.5 * 2^52, whose low
// bits are k in two's complement) and r = x - k ln 2 / 256 (two-constant
// Cody-Waite reduction, |r| <= ln 2 / 512), e^x = 2^(k >> 8) t[k & 255] e^r,
// e^r by its Taylor polynomial of degree 4 (next term below 4e-17).  x is
// clamped to [-746, 710] first (below, e^x underflows to 0; above, the
// result overflows to inf), which keeps |k| < 2^19.  14 operations and one
// LDS read against ~30 for the library's exp.
__device__ __forceinline__ double table_exp(double x, const double *__restrict__ t)
{
    constexpr double kRound = 6755399441055744.0;          // 1.5 * 2^52
    constexpr double kInvStep = 369.3299304675746;          // 256 / ln 2
    constexpr double kStepHi = 0.002707604318857193;        // ln 2 / 256, 21 leading bits
    constexpr double kStepLo = 1.855205093371747e-09;       // the rest of ln 2 / 256
    x = fmin(fmax(x, -746.0), 710.0);
    const double tt = __builtin_fma(x, kInvStep, kRound);
    const double kf = tt - kRound;
    double r = __builtin_fma(-kf, kStepHi, x);
    r = __builtin_fma(-kf, kStepLo, r);
    const int k = __double2loint(tt);
    double p = __builtin_fma(r, 1.0 / 24.0, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(t[k & 255] * p, k >> 8);
}

// p(theta | Lambda) / p(theta | 0) of one sample; t: the table of table_exp.
__device__ __forceinline__ double weight(const Sample &x, const HyperC &c, const double *__restrict__ t)
{
    if (!x.ok || x.m1 < c.mmin || x.m1 > c.mmax) return 0.0;
    const double ln_qmin = c.ln_mmin - x.ln_m1;          // q_min = m_min / m1
    if (x.m1 <= c.mmin || x.ln_q < ln_qmin) return 0.0;
    // q^beta, the two spin magnitudes and the prior: the log of every factor
    // but the primary mass, tilts and q normalisation
    double e = __builtin_fma(c.beta, x.ln_q, -x.ln_prior);
    e = __builtin_fma(c.ach_m1, x.ln_a_sum, e);
    e = __builtin_fma(c.bch_m1, x.ln_1ma_sum, e);
    e -= 2.0 * c.ln_beta_fn;
    // primary mass times exp(e): both mixture components carry it
    const double a_pl = __builtin_fma(c.neg_alpha, x.ln_m1, e - c.ln_zpl);
    const double z = (x.m1 - c.mu) * c.inv_sigma;
    const double a_g = __builtin_fma(-0.5 * z, z, e - c.ln_zg);
    const double p_me = __builtin_fma(c.one_m_lam, table_exp(a_pl, t), c.lam * table_exp(a_g, t));
    // 1 / the mass ratio normalisation int_{q_min}^1 x^beta dx (one division
    // whichever form the point takes)
    const double num = c.beta_is_m1 ? -1.0 : -c.one_p_beta;
    const double den = c.beta_is_m1 ? ln_qmin : expm1(c.one_p_beta * ln_qmin);
    const double inv_zq = num / den;
    // tilts
    const double g = table_exp(-(c.k1 * x.c1m * x.c1m + c.k2 * x.c2m * x.c2m) - c.ln_zt, t);
    const double p_t = __builtin_fma(c.xi, g, c.iso);
    return p_me * p_t * inv_zq;
}

// Block b = event * chunks + chunk: kPerBlock samples of the event; for every
// Lambda each wave writes the sum of its samples' weights to
// partials[(k * n_events + event) * n_slots + chunk * kWaves + wave].
template <bool PREPARED>
__global__ __launch_bounds__(kThreads) void weights_kernel(int64_t n_events, int64_t n_per, int64_t chunks,
                                                           const double *__restrict__ s, int64_t n_hyper,
                                                           const HyperC *__restrict__ hc, int64_t n_slots,
                                                           double *__restrict__ partials)
{
    __shared__ double t_exp[256];
    t_exp[threadIdx.x] = exp2((double)threadIdx.x / 256.0);     // kThreads == 256
    __syncthreads();
    const int64_t event = (int64_t)blockIdx.x / chunks, chunk = (int64_t)blockIdx.x % chunks;
    const int64_t plane = n_events * n_per;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    Sample x[kPerThread];
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        // consecutive lanes read consecutive samples
        const int64_t j = chunk * kPerBlock + (int64_t)i * kThreads + threadIdx.x;
        x[i] = PREPARED ? load_prepared(s, plane, event * n_per + j, j < n_per)
                        : load_sample(s, plane, event * n_per + j, j < n_per);
    }
    for (int64_t k = 0; k < n_hyper; ++k) {
        const HyperC c = hc[k];
        double w = 0.0;
        if (c.status == 1) {
#pragma unroll
            for (int i = 0; i < kPerThread; ++i) w += weight(x[i], c, t_exp);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
        if (lane == 0) partials[(k * n_events + event) * n_slots + chunk * kWaves + wave] = w;
    }
}

// Wave w of block b handles (Lambda k, event i) with k * n_events + i =
// b * kWaves + w: its lanes sum the event's partials (strided, then a fixed
// butterfly) and lane 0 writes ln(mean) to lmean[k][i].
__global__ __launch_bounds__(kThreads) void event_means_kernel(int64_t n_events, int64_t n_per, int64_t n_slots,
                                                               int64_t n_pairs, const double *__restrict__ partials,
                                                               double *__restrict__ lmean)
{
    const int lane = threadIdx.x % 64;
    const int64_t pair = (int64_t)blockIdx.x * kWaves + threadIdx.x / 64;
    if (pair >= n_pairs) return;
    const double *p = partials + pair * n_slots;
    double sum = 0.0;
    for (int64_t t = lane; t < n_slots; t += 64) sum += p[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (lane == 0) lmean[pair] = log(sum / (double)n_per);
}

// Block k: ln L(Lambda_k) = sum over events of lmean[k][i] (strided per
// thread, then a fixed tree), or -inf / NaN for points outside the domain.
__global__ __launch_bounds__(kThreads) void finalize_kernel(int64_t n_events, const HyperC *__restrict__ hc,
                                                            const double *__restrict__ lmean,
                                                            double *__restrict__ lnl)
{
    __shared__ double red[kThreads];
    const int64_t k = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n_events; i += kThreads) acc += lmean[k * n_events + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int status = hc[k].status;
        lnl[k] = status == 1 ? red[0] : (status == 0 ? -INFINITY : NAN);
    }
}

int64_t slots_per_event(int64_t n_per) { return (n_per + kPerBlock - 1) / kPerBlock * kWaves; }

int64_t weight_blocks(int64_t n_events, int64_t n_per) { return (n_per + kPerBlock - 1) / kPerBlock * n_events; }

size_t workspace_bytes(int64_t n_events, int64_t n_per, int64_t n_hyper)
{
    return (size_t)n_hyper * sizeof(HyperC) + 512 + (size_t)n_hyper * (size_t)n_events * sizeof(double) +
           (size_t)n_hyper * (size_t)n_events * (size_t)slots_per_event(n_per) * sizeof(double);
}

hipError_t prepare(int64_t n_events, int64_t n_per, const double *samples, double *prepared, hipStream_t stream)
{
    const int64_t plane = n_events * n_per;
    hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)((plane + kThreads - 1) / kThreads)), dim3(kThreads), 0, stream,
                       plane, samples, prepared);
    return hipGetLastError();
}

hipError_t launch(int64_t n_events, int64_t n_per, const double *samples, bool prepared, int64_t n_hyper,
                  const double *hyper, void *work, double *lnl, hipEvent_t t_start, hipEvent_t t_stop,
                  hipStream_t stream)
{
    HyperC *hc = static_cast<HyperC *>(work);
    const size_t hc_bytes = ((size_t)n_hyper * sizeof(HyperC) + 255) / 256 * 256;
    const size_t lm_bytes = ((size_t)n_hyper * (size_t)n_events * sizeof(double) + 255) / 256 * 256;
    double *lmean = reinterpret_cast<double *>(static_cast<char *>(work) + hc_bytes);
    double *partials = reinterpret_cast<double *>(static_cast<char *>(work) + hc_bytes + lm_bytes);
    hipLaunchKernelGGL(hyper_kernel, dim3((unsigned)((n_hyper + kThreads - 1) / kThreads)), dim3(kThreads), 0, stream,
                       n_hyper, hyper, hc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t chunks = (n_per + kPerBlock - 1) / kPerBlock;
    const int64_t n_slots = slots_per_event(n_per);
    if (t_start && (e = hipEventRecord(t_start, stream)) != hipSuccess) return e;
    if (prepared)
        hipLaunchKernelGGL(weights_kernel<true>, dim3((unsigned)(chunks * n_events)), dim3(kThreads), 0, stream,
                           n_events, n_per, chunks, samples, n_hyper, hc, n_slots, partials);
    else
        hipLaunchKernelGGL(weights_kernel<false>, dim3((unsigned)(chunks * n_events)), dim3(kThreads), 0, stream,
                           n_events, n_per, chunks, samples, n_hyper, hc, n_slots, partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (t_stop && (e = hipEventRecord(t_stop, stream)) != hipSuccess) return e;
    const int64_t n_pairs = n_hyper * n_events;
    hipLaunchKernelGGL(event_means_kernel, dim3((unsigned)((n_pairs + kWaves - 1) / kWaves)), dim3(kThreads), 0,
                       stream, n_events, n_per, n_slots, n_pairs, partials, lmean);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)n_hyper), dim3(kThreads), 0, stream, n_events, hc, lmean, lnl);
    return hipGetLastError();
}

}  // namespace pop
}  // namespace gw

GW_DEFINE_SOURCE_HASH(pop)
