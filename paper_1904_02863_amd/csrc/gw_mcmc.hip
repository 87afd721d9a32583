// Counter-based random numbers and Metropolis-Hastings kernels for many
// parallel chains whose proposals are judged by the exact likelihood of
// gw_lnl_batch (Eq. (cbclike) of arXiv:1904.02863, Sec. III).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a 64-bit key
// go through ten rounds of two 32x32->64-bit multiplies, the key advanced by
// the Weyl constants between rounds.  Every number the sampler draws is a pure
// function of (seed, stream, step, index), so runs are reproducible, resumable
// from any step and independent of launch shapes.
//
// Sampler coordinates: x in R^dim, x_i = logit(u_i), u_i the position of
// parameter i in its prior box [lo_i, hi_i] (uniform priors in
// Mc, q, d_L, phi_c, t_c, RA, sin Dec, psi, cos iota and, when dim = 11, the
// two aligned spins, which the non-spinning waveform does not use).  The prior
// density in x is prod_i u_i (1 - u_i).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "gw_build_id.h"
#include "gw_mcmc_internal.h"
#include "gwlnl.h"

namespace gw {
namespace mcmc {

__host__ __device__ inline void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Block `index` of (seed, stream, step): counter (index lo, index hi, step, stream).
__device__ __forceinline__ void philox_block(uint64_t seed, uint32_t stream, uint32_t step, uint64_t index,
                                             uint32_t out[4])
{
    const uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), step, stream};
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

// Two uniforms in (0, 1) with 53 random bits each.
__device__ __forceinline__ void uniform_pair(const uint32_t a[4], double &u0, double &u1)
{
    const double scale = 1.0 / 9007199254740992.0;   // 2^-53
    u0 = ((double)(a[0] >> 5) * 67108864.0 + (double)(a[1] >> 6) + 0.5) * scale;
    u1 = ((double)(a[2] >> 5) * 67108864.0 + (double)(a[3] >> 6) + 0.5) * scale;
}

// Two standard normals by the Box-Muller transform of one uniform pair.
__device__ __forceinline__ void normal_pair(const uint32_t a[4], double &z0, double &z1)
{
    double u0, u1;
    uniform_pair(a, u0, u1);
    const double r = sqrt(-2.0 * log(u0));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
}

__global__ __launch_bounds__(256) void philox_raw_kernel(uint64_t seed, uint32_t stream, uint32_t step,
                                                         uint64_t first, int64_t n_blocks,
                                                         uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_blocks) return;
    uint32_t a[4];
    philox_block(seed, stream, step, first + (uint64_t)i, a);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = a[j];
}

// out[i], i < n: uniform (kind 0) or normal (kind 1) number i of (seed, stream, step).
__global__ __launch_bounds__(256) void philox_fill_kernel(uint64_t seed, uint32_t stream, uint32_t step, int kind,
                                                          int64_t n, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * i >= n) return;
    uint32_t a[4];
    philox_block(seed, stream, step, (uint64_t)i, a);
    double v0, v1;
    if (kind == 0) uniform_pair(a, v0, v1);
    else normal_pair(a, v0, v1);
    out[2 * i] = v0;
    if (2 * i + 1 < n) out[2 * i + 1] = v1;
}

// Normals for a [n][dim] block of chains: chain c uses blocks c ceil(dim/2) + j.
__device__ __forceinline__ double chain_normal(uint64_t seed, uint32_t stream, uint32_t step, int64_t c, int dim,
                                               int i)
{
    const int per = (dim + 1) / 2;
    uint32_t a[4];
    philox_block(seed, stream, step, (uint64_t)(c * per + i / 2), a);
    double z0, z1;
    normal_pair(a, z0, z1);
    return (i & 1) ? z1 : z0;
}

// z[c][i] = normal i of chain c (flow proposals draw their latent point here).
__global__ __launch_bounds__(256) void chain_normals_kernel(int dim, int64_t n, uint64_t seed, uint32_t stream,
                                                            uint32_t step, double *__restrict__ z)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int i = 0; i < dim; ++i) z[c * dim + i] = chain_normal(seed, stream, step, c, dim, i);
}

// ---------------------------------------------------------------- coordinates
__device__ __forceinline__ double sigmoid(double x) { return x >= 0 ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x)); }

// log u + log(1 - u) for u = sigmoid(x), computed without cancellation.
__device__ __forceinline__ double log_u_1mu(double x)
{
    const double ax = fabs(x);
    return -ax - 2.0 * log1p(exp(-ax));
}

// theta (9 columns, the layout of gw_lnl_batch) and the log prior density of x.
__global__ __launch_bounds__(256) void to_theta_kernel(int dim, int64_t n, Box box, const double *__restrict__ x,
                                                       int theta_cols, double *__restrict__ theta,
                                                       double *__restrict__ logprior)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double p[kMaxDim];
    double lp = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double xi = x[c * dim + i];
        p[i] = box.lo[i] + (box.hi[i] - box.lo[i]) * sigmoid(xi);
        lp += log_u_1mu(xi);
    }
    double *th = theta + c * theta_cols;
    th[0] = p[0];           // Mc
    th[1] = p[1];           // q
    th[2] = p[2];           // d_L
    th[3] = p[3];           // phi_c
    th[4] = p[4];           // t_c
    th[5] = p[5];           // RA
    th[6] = asin(p[6]);     // Dec from sin Dec
    th[7] = p[7];           // psi
    th[8] = acos(p[8]);     // iota from cos iota
    if (theta_cols == 11) {
        th[9] = p[9];       // chi1
        th[10] = p[10];     // chi2
    }
    if (logprior) logprior[c] = lp;
}

// Random-walk proposal x' = x + L z for chains in random-walk mode (all chains
// when mode is null); L is lower triangular [dim][dim].
__global__ __launch_bounds__(256) void rw_propose_kernel(int dim, int64_t n, const double *__restrict__ x,
                                                         const double *__restrict__ chol, uint64_t seed, uint32_t step,
                                                         const int *__restrict__ mode, double *__restrict__ x_prop)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (mode && mode[c] != kModeRandomWalk) return;
    double z[kMaxDim];
    for (int i = 0; i < dim; ++i) z[i] = chain_normal(seed, kStreamRandomWalk, step, c, dim, i);
    for (int i = 0; i < dim; ++i) {
        double v = x[c * dim + i];
        for (int j = 0; j <= i; ++j) v += chol[i * dim + j] * z[j];
        x_prop[c * dim + i] = v;
    }
}

// Metropolis-Hastings decision per chain:
//   log alpha = (lnL' + log pi') - lnp + [log q(x) - log q(x')]   (flow mode)
// with the bracket absent in random-walk mode (symmetric proposal).
// On acceptance x and lnp take the proposal's values, and in flow mode so does
// log q(x) (a random-walk move leaves it stale until the next mode update
// recomputes it).  Acceptances are added to the counters that are given.
__global__ __launch_bounds__(256) void accept_kernel(int dim, int64_t n, uint64_t seed, uint32_t step,
                                                     double *__restrict__ x, double *__restrict__ lnp,
                                                     double *__restrict__ logq, const double *__restrict__ x_prop,
                                                     const double *__restrict__ lnl_prop,
                                                     const double *__restrict__ lp_prop,
                                                     const double *__restrict__ logq_prop,
                                                     const int *__restrict__ mode, int *__restrict__ window_accepts,
                                                     int *__restrict__ total_accepts)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const bool flow = mode && mode[c] == kModeFlow;
    const double target = lnl_prop[c] + lp_prop[c];
    double log_alpha = target - lnp[c];
    if (flow) log_alpha += logq[c] - logq_prop[c];
    uint32_t a[4];
    philox_block(seed, kStreamAccept, step, (uint64_t)c, a);
    double u0, u1;
    uniform_pair(a, u0, u1);
    const bool ok = isfinite(target) && log(u0) < log_alpha;
    if (ok) {
        for (int i = 0; i < dim; ++i) x[c * dim + i] = x_prop[c * dim + i];
        lnp[c] = target;
        if (flow) logq[c] = logq_prop[c];
    }
    if (window_accepts) window_accepts[c] += ok ? 1 : 0;
    if (total_accepts) total_accepts[c] += ok ? 1 : 0;
}

// Per-chain proposal mode from the acceptance count of the last window:
// flow proposals while the rate is at least `threshold`, random walk below;
// the window counters restart at zero.
__global__ __launch_bounds__(256) void update_mode_kernel(int64_t n, int *__restrict__ window_accepts, int window,
                                                          double threshold, int *__restrict__ mode)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    mode[c] = (double)window_accepts[c] < threshold * window ? kModeRandomWalk : kModeFlow;
    window_accepts[c] = 0;
}

// ---------------------------------------------------------------- adaptation
// Fixed-order sum of v over the 256 threads of the block; thread 0 gets it.
__device__ __forceinline__ double block_sum256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double total = red[0];
    __syncthreads();
    return total;
}

// One block.  Sample mean and covariance of the n rows of x [n][dim] (two
// passes, fixed order) into mean_out [dim] and cov_out [dim][dim] when given;
// with chol given, C = (2.38^2 / dim) scale^2 Cov + eps I, eps = floor
// max(1, trace / dim), and its lower Cholesky factor into chol [dim][dim]
// (upper part zero).  A pivot that is not positive is replaced by sqrt(eps),
// which keeps the factor finite for degenerate chain sets.
__global__ __launch_bounds__(256) void adapt_chol_kernel(int dim, int64_t n, const double *__restrict__ x,
                                                         double scale, double floor, double *__restrict__ chol,
                                                         double *__restrict__ mean_out, double *__restrict__ cov_out)
{
    __shared__ double red[256];
    __shared__ double mean[kMaxDim];
    __shared__ double c[kMaxDim * kMaxDim];
    // every column's sum in one pass over the rows (each thread its rows
    // tid, tid + 256, ... in order), then the block sums column by column
    double acc[kMaxDim];
#pragma unroll
    for (int i = 0; i < kMaxDim; ++i) acc[i] = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256)
#pragma unroll
        for (int i = 0; i < kMaxDim; ++i)
            if (i < dim) acc[i] += x[r * dim + i];
#pragma unroll
    for (int i = 0; i < kMaxDim; ++i) {
        if (i >= dim) break;
        const double total = block_sum256(acc[i], red);
        if (threadIdx.x == 0) mean[i] = total / (double)n;
    }
    __syncthreads();
    // row i of the covariance (j <= i) in one pass over the rows, the same
    // per-thread order as the means
    for (int i = 0; i < dim; ++i) {
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) acc[j] = 0.0;
        const double mi = mean[i];
        for (int64_t r = threadIdx.x; r < n; r += 256) {
            const double di = x[r * dim + i] - mi;
#pragma unroll
            for (int j = 0; j < kMaxDim; ++j)
                if (j <= i) acc[j] += di * (x[r * dim + j] - mean[j]);
        }
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) {
            if (j > i) break;
            const double total = block_sum256(acc[j], red);
            if (threadIdx.x == 0) c[i * kMaxDim + j] = total / (double)(n > 1 ? n - 1 : 1);
        }
    }
    if (threadIdx.x != 0) return;
    if (mean_out)
        for (int i = 0; i < dim; ++i) mean_out[i] = mean[i];
    if (cov_out)
        for (int i = 0; i < dim; ++i)
            for (int j = 0; j <= i; ++j) cov_out[i * dim + j] = cov_out[j * dim + i] = c[i * kMaxDim + j];
    if (!chol) return;
    const double f = 2.38 * 2.38 / (double)dim * scale * scale;
    double tr = 0.0;
    for (int i = 0; i < dim; ++i) tr += f * c[i * kMaxDim + i];
    const double eps = floor * fmax(1.0, tr / (double)dim);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j <= i; ++j) c[i * kMaxDim + j] = f * c[i * kMaxDim + j] + (i == j ? eps : 0.0);
    // Cholesky-Banachiewicz, row by row
    for (int i = 0; i < dim; ++i) {
        for (int j = 0; j <= i; ++j) {
            double v = c[i * kMaxDim + j];
            for (int k = 0; k < j; ++k) v -= chol[i * dim + k] * chol[j * dim + k];
            if (i == j) chol[i * dim + i] = v > 0.0 ? sqrt(v) : sqrt(eps);
            else chol[i * dim + j] = v / chol[j * dim + j];
        }
        for (int j = i + 1; j < dim; ++j) chol[i * dim + j] = 0.0;
    }
}

// out[0] = sum of counts[0 .. n) (one block, fixed order).
__global__ __launch_bounds__(256) void count_sum_kernel(int64_t n, const int *__restrict__ counts,
                                                        int64_t *__restrict__ out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += (double)counts[i];
    const double total = block_sum256(acc, red);
    if (threadIdx.x == 0) out[0] = (int64_t)total;
}

// dst[i] = src[floor(u_i n_src)], u_i uniform number i of (seed, stream, step):
// rows drawn with replacement (training minibatches).
__global__ __launch_bounds__(256) void gather_rows_kernel(int dim, int64_t n_out, const double *__restrict__ src,
                                                          int64_t n_src, uint64_t seed, uint32_t stream, uint32_t step,
                                                          double *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    uint32_t a[4];
    philox_block(seed, stream, step, (uint64_t)(i >> 1), a);
    double u0, u1;
    uniform_pair(a, u0, u1);
    const double u = (i & 1) ? u1 : u0;
    int64_t r = (int64_t)(u * (double)n_src);
    r = r < n_src ? r : n_src - 1;
    for (int j = 0; j < dim; ++j) dst[i * dim + j] = src[r * dim + j];
}

// ---------------------------------------------------------------- launchers
static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t philox_raw(uint64_t seed, uint32_t stream, uint32_t step, uint64_t first, int64_t n_blocks, uint32_t *out,
                      hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_raw_kernel, dim3(blocks_for(n_blocks)), dim3(256), 0, s, seed, stream, step, first,
                       n_blocks, out);
    return hipGetLastError();
}

hipError_t philox_fill(uint64_t seed, uint32_t stream, uint32_t step, int kind, int64_t n, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_fill_kernel, dim3(blocks_for((n + 1) / 2)), dim3(256), 0, s, seed, stream, step, kind, n,
                       out);
    return hipGetLastError();
}

hipError_t normals_for_chains(int dim, int64_t n, uint64_t seed, uint32_t stream, uint32_t step, double *out,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(chain_normals_kernel, dim3(blocks_for(n)), dim3(256), 0, s, dim, n, seed, stream, step, out);
    return hipGetLastError();
}

hipError_t to_theta(int dim, int64_t n, const Box &box, const double *x, int theta_cols, double *theta,
                    double *logprior, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_theta_kernel, dim3(blocks_for(n)), dim3(256), 0, s, dim, n, box, x, theta_cols, theta,
                       logprior);
    return hipGetLastError();
}

hipError_t rw_propose(int dim, int64_t n, const double *x, const double *chol, uint64_t seed, uint32_t step,
                      const int *mode, double *x_prop, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rw_propose_kernel, dim3(blocks_for(n)), dim3(256), 0, s, dim, n, x, chol, seed, step, mode,
                       x_prop);
    return hipGetLastError();
}

hipError_t accept(int dim, int64_t n, uint64_t seed, uint32_t step, double *x, double *lnp, double *logq,
                  const double *x_prop, const double *lnl_prop, const double *lp_prop, const double *logq_prop,
                  const int *mode, int *window_accepts, int *total_accepts, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(accept_kernel, dim3(blocks_for(n)), dim3(256), 0, s, dim, n, seed, step, x, lnp, logq, x_prop,
                       lnl_prop, lp_prop, logq_prop, mode, window_accepts, total_accepts);
    return hipGetLastError();
}

hipError_t update_mode(int64_t n, int *window_accepts, int window, double threshold, int *mode, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(update_mode_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, window_accepts, window, threshold,
                       mode);
    return hipGetLastError();
}

hipError_t adapt_chol(int dim, int64_t n, const double *x, double scale, double floor, double *chol, double *mean,
                      double *cov, hipStream_t s)
{
    hipLaunchKernelGGL(adapt_chol_kernel, dim3(1), dim3(256), 0, s, dim, n, x, scale, floor, chol, mean, cov);
    return hipGetLastError();
}

hipError_t count_sum(int64_t n, const int *counts, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(count_sum_kernel, dim3(1), dim3(256), 0, s, n, counts, out);
    return hipGetLastError();
}

hipError_t gather_rows(int dim, int64_t n_out, const double *src, int64_t n_src, uint64_t seed, uint32_t stream,
                       uint32_t step, double *dst, hipStream_t s)
{
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(n_out)), dim3(256), 0, s, dim, n_out, src, n_src, seed,
                       stream, step, dst);
    return hipGetLastError();
}

}  // namespace mcmc
}  // namespace gw

// ================================================================ C ABI
namespace {
int fail(int code, const std::string &msg) { return gw::set_error(code, msg); }
int hip_fail(hipError_t e, const char *where) { return fail(GW_EDEVICE, std::string(where) + ": " + hipGetErrorString(e)); }
}  // namespace

extern "C" {

int gw_philox_raw(uint64_t seed, uint32_t stream_id, uint32_t step, uint64_t first, int64_t n_blocks,
                  uint32_t *out, hipStream_t stream)
{
    if (n_blocks < 0 || (n_blocks > 0 && !out)) return fail(GW_EINVAL, "bad philox arguments");
    hipError_t e = gw::mcmc::philox_raw(seed, stream_id, step, first, n_blocks, out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_philox_raw");
}

int gw_philox_fill(uint64_t seed, uint32_t stream_id, uint32_t step, int kind, int64_t n, double *out,
                   hipStream_t stream)
{
    if (n < 0 || (n > 0 && !out) || (kind != 0 && kind != 1)) return fail(GW_EINVAL, "bad philox arguments");
    hipError_t e = gw::mcmc::philox_fill(seed, stream_id, step, kind, n, out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_philox_fill");
}

int gw_philox_chain_normals(int dim, int64_t n_chains, uint64_t seed, uint32_t stream_id, uint32_t step,
                            double *out, hipStream_t stream)
{
    if (dim < 1 || dim > gw::mcmc::kMaxDim || n_chains < 0 || (n_chains > 0 && !out))
        return fail(GW_EINVAL, "bad arguments");
    hipError_t e = gw::mcmc::normals_for_chains(dim, n_chains, seed, stream_id, step, out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_philox_chain_normals");
}

int gw_mcmc_to_theta(int dim, int64_t n, const double *box_lo, const double *box_hi, const double *x,
                     int theta_cols, double *theta_out, double *logprior_out, hipStream_t stream)
{
    if ((dim != 9 && dim != 11) || n < 0 || !box_lo || !box_hi || (n > 0 && (!x || !theta_out)))
        return fail(GW_EINVAL, "bad arguments");
    if (theta_cols != 9 && !(theta_cols == 11 && dim == 11))
        return fail(GW_EINVAL, "theta_cols must be 9, or 11 with dim 11");
    gw::mcmc::Box box{};
    for (int i = 0; i < dim; ++i) {
        if (!(box_hi[i] > box_lo[i])) return fail(GW_EINVAL, "empty prior box");
        box.lo[i] = box_lo[i];
        box.hi[i] = box_hi[i];
    }
    if (box.lo[6] < -1.0 || box.hi[6] > 1.0 || box.lo[8] < -1.0 || box.hi[8] > 1.0)
        return fail(GW_EINVAL, "sin Dec and cos iota boxes must lie in [-1, 1]");
    if (theta_cols == 11 && (box.lo[9] < -1.0 || box.hi[9] > 1.0 || box.lo[10] < -1.0 || box.hi[10] > 1.0))
        return fail(GW_EINVAL, "spin boxes must lie in [-1, 1]");
    hipError_t e = gw::mcmc::to_theta(dim, n, box, x, theta_cols, theta_out, logprior_out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_to_theta");
}

int gw_mcmc_rw_propose(int dim, int64_t n, const double *x, const double *chol, uint64_t seed, uint32_t step,
                       const int *mode, double *x_prop, hipStream_t stream)
{
    if (dim < 1 || dim > gw::mcmc::kMaxDim || n < 0 || (n > 0 && (!x || !chol || !x_prop)))
        return fail(GW_EINVAL, "bad arguments");
    hipError_t e = gw::mcmc::rw_propose(dim, n, x, chol, seed, step, mode, x_prop, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_rw_propose");
}

int gw_mcmc_accept(int dim, int64_t n, uint64_t seed, uint32_t step, double *x, double *lnp, double *logq,
                   const double *x_prop, const double *lnl_prop, const double *lp_prop, const double *logq_prop,
                   const int *mode, int *window_accepts, int *total_accepts, hipStream_t stream)
{
    if (dim < 1 || dim > gw::mcmc::kMaxDim || n < 0 ||
        (n > 0 && (!x || !lnp || !x_prop || !lnl_prop || !lp_prop)))
        return fail(GW_EINVAL, "bad arguments");
    if (mode && (!logq || !logq_prop)) return fail(GW_EINVAL, "flow mode needs logq and logq_prop");
    hipError_t e = gw::mcmc::accept(dim, n, seed, step, x, lnp, logq, x_prop, lnl_prop, lp_prop, logq_prop, mode,
                                     window_accepts, total_accepts, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_accept");
}

int gw_mcmc_update_mode(int64_t n, int *window_accepts, int window, double threshold, int *mode,
                        hipStream_t stream)
{
    if (n < 0 || window < 1 || (n > 0 && (!window_accepts || !mode))) return fail(GW_EINVAL, "bad arguments");
    hipError_t e = gw::mcmc::update_mode(n, window_accepts, window, threshold, mode, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_update_mode");
}

int gw_mcmc_adapt_chol(int dim, int64_t n, const double *x, double scale, double floor, double *chol_out,
                       hipStream_t stream)
{
    if (dim < 1 || dim > gw::mcmc::kMaxDim || n < 2 || !x || !chol_out)
        return fail(GW_EINVAL, "gw_mcmc_adapt_chol needs dim in 1..16, at least 2 rows and device arrays");
    if (!(scale > 0.0) || !(floor >= 0.0)) return fail(GW_EINVAL, "scale must be > 0 and floor >= 0");
    hipError_t e = gw::mcmc::adapt_chol(dim, n, x, scale, floor, chol_out, nullptr, nullptr, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_adapt_chol");
}

int gw_mcmc_moments(int dim, int64_t n, const double *x, double *mean_out, double *cov_out, hipStream_t stream)
{
    if (dim < 1 || dim > gw::mcmc::kMaxDim || n < 2 || !x || (!mean_out && !cov_out))
        return fail(GW_EINVAL, "gw_mcmc_moments needs dim in 1..16, at least 2 rows and an output");
    hipError_t e = gw::mcmc::adapt_chol(dim, n, x, 1.0, 0.0, nullptr, mean_out, cov_out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_moments");
}

int gw_mcmc_count(int64_t n, const int *counts, int64_t *out, hipStream_t stream)
{
    if (n < 0 || (n > 0 && !counts) || !out) return fail(GW_EINVAL, "bad arguments");
    hipError_t e = gw::mcmc::count_sum(n, counts, out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_mcmc_count");
}

int gw_gather_rows(int dim, int64_t n_out, const double *src, int64_t n_src, uint64_t seed, uint32_t stream_id,
                   uint32_t step, double *dst, hipStream_t stream)
{
    if (dim < 1 || n_out < 0 || n_src < 1 || !src || (n_out > 0 && !dst)) return fail(GW_EINVAL, "bad arguments");
    hipError_t e = gw::mcmc::gather_rows(dim, n_out, src, n_src, seed, stream_id, step, dst, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_gather_rows");
}

}  // extern "C"

GW_DEFINE_SOURCE_HASH(mcmc)
