// Learned proposal for the sampler: an affine-coupling normalising flow
// trained and evaluated with BF16 matrix-core (MFMA) kernels on gfx950, plus
// the counter-based random numbers and Metropolis-Hastings kernels that use
// it.  The likelihood that judges every proposal is the exact one of
// gw_lnl_batch (Eq. (cbclike) of arXiv:1904.02863, Sec. III); the paper notes
// (Sec. I) that sampling algorithms themselves are hard to parallelise, which
// is what many chains with learned independence proposals address here.
//
// Flow (RealNVP-style affine coupling, Dinh, Sohl-Dickstein & Bengio 2017):
// generative direction x = f_{L-1}( ... f_0(z)), z ~ N(0, I).  Layer l keeps
// the dimensions of its conditioning set C_l and maps the others (T_l) as
//     x_T = a_T exp(s) + t,   (r, t) = MLP_l(m_l * a),   s = 3 tanh(r / 3),
// MLP_l = Linear(dim -> H) ReLU Linear(H -> H) ReLU Linear(H -> 2 dim).
// The MLPs run on MFMA in BF16 with FP32 accumulation; the coupling itself,
// the state x and every log-determinant are FP64, so the forward and inverse
// maps invert each other to FP64 rounding (both see bit-identical MLP inputs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "gw_build_id.h"
#include "gw_flow_internal.h"
#include "gwlnl.h"

namespace gw {
namespace flow {

// ---------------------------------------------------------------- BF16 helpers
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                               // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---------------------------------------------------------------- GEMM on MFMA
// C[M x N] = A[M x K] B[K x N] (+ bias[N]) (ReLU if relu), FP32 accumulation.
// A(i, k) = A[i sa_i + k sa_k], B(k, j) = B[k sb_k + j sb_j], both BF16.
// Block: 256 threads, 64 x 64 output tile (blockIdx.z: K slice when split),
// K in steps of 16 through LDS; each
// of the 4 waves owns a 32 x 32 quarter as 2 x 2 tiles of
// v_mfma_f32_16x16x16_bf16.  Operand layout of that instruction (wave64):
// lane l supplies A(row l%16, k = 4(l/16)+0..3) and B(k = 4(l/16)+0..3,
// col l%16) and receives D(row 4(l/16)+0..3, col l%16).
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ uint16_t as[64][16 + 2];
    __shared__ uint16_t bs[16][64 + 2];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    // K slice of this block (the whole range unless split)
    const int ks = ((g.K + g.split - 1) / g.split + 15) / 16 * 16;
    const int k_lo = (int)blockIdx.z * ks, k_hi = min(g.K, k_lo + ks);
    float4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};

    for (int k0 = k_lo; k0 < k_hi; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + 256 * e;          // 0 .. 1023
            {   // A tile 64 x 16
                const int i = idx >> 4, k = idx & 15;
                const int gi = row0 + i, gk = k0 + k;
                as[i][k] = (gi < g.M && gk < k_hi) ? g.A[(int64_t)gi * g.sa_i + (int64_t)gk * g.sa_k] : (uint16_t)0;
            }
            {   // B tile 16 x 64
                const int k = idx >> 6, j = idx & 63;
                const int gk = k0 + k, gj = col0 + j;
                bs[k][j] = (gk < k_hi && gj < g.N) ? g.B[(int64_t)gk * g.sb_k + (int64_t)gj * g.sb_j] : (uint16_t)0;
            }
        }
        __syncthreads();
        const int kq = 4 * (lane >> 4), lr = lane & 15;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            short4_t av;
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = (short)as[wr + 16 * a + lr][kq + r];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                short4_t bv;
#pragma unroll
                for (int r = 0; r < 4; ++r) bv[r] = (short)bs[kq + r][wc + 16 * b + lr];
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[a][b], 0, 0, 0);
            }
        }
    }
    const int rq = 4 * (lane >> 4), lc = lane & 15;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + wr + 16 * a + rq + r;
                const int j = col0 + wc + 16 * b + lc;
                if (i < g.M && j < g.N) {
                    float v = acc[a][b][r];
                    if (g.split > 1) {
                        g.partial[((int64_t)blockIdx.z * g.M + i) * g.N + j] = v;
                        continue;
                    }
                    if (g.bias) v += g.bias[j];
                    if (g.relu) v = v > 0.f ? v : 0.f;
                    if (g.C) g.C[(int64_t)i * g.ldc + j] = v;
                    if (g.Cb) g.Cb[(int64_t)i * g.ldcb + j] = f32_to_bf16(v);
                }
            }
}

// Sums the split-K slices in slice order, then bias, ReLU and the outputs.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.M * g.N) return;
    const int i = (int)(t / g.N), j = (int)(t % g.N);
    float v = 0.f;
    for (int z = 0; z < g.split; ++z) v += g.partial[(int64_t)z * g.M * g.N + t];
    if (g.bias) v += g.bias[j];
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.C) g.C[(int64_t)i * g.ldc + j] = v;
    if (g.Cb) g.Cb[(int64_t)i * g.ldcb + j] = f32_to_bf16(v);
}

hipError_t gemm_bf16(const GemmArgs &g, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.split < 1 || g.split > kMaxSplit || (g.split > 1 && !g.partial)) return hipErrorInvalidValue;
    const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, g.split);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, stream, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.split == 1) return e;
    const int64_t total = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- coupling layers
// Row b of a [n][dim] FP64 state.  `cond` has bit i set when dimension i is
// in the layer's conditioning set.

// MLP input: the conditioning dimensions of a, the others zero, as BF16 in a
// row of kInPad entries (the GEMM's K is dim; the padding stays zero).
__global__ __launch_bounds__(256) void mask_input_kernel(int n, int dim, unsigned cond, const double *__restrict__ a,
                                                         uint16_t *__restrict__ xm)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int i = 0; i < kInPad; ++i) {
        const bool on = i < dim && ((cond >> i) & 1u);
        xm[(int64_t)b * kInPad + i] = on ? f32_to_bf16((float)a[(int64_t)b * dim + i]) : (uint16_t)0;
    }
}

// Affine coupling given the MLP output (r, t) = out[b][0..dim), out[b][dim..2dim):
//   forward (dir > 0): y_T = a_T exp(s) + t;  inverse (dir < 0): y_T = (a_T - t) exp(-s);
// s = 3 tanh(r/3); conditioning dimensions are copied.  sum_s[b] += sum_T s in
// both directions (log q = log N(z) - sum_s); s is stored when s_out is set.
__global__ __launch_bounds__(256) void coupling_kernel(int n, int dim, unsigned cond, int dir,
                                                       const double *__restrict__ a, const float *__restrict__ out,
                                                       double *__restrict__ y, double *__restrict__ sum_s,
                                                       double *__restrict__ s_out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double acc = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double ai = a[(int64_t)b * dim + i];
        double yi = ai, s = 0.0;
        if (!((cond >> i) & 1u)) {
            const double r = (double)out[(int64_t)b * 2 * dim + i];
            const double t = (double)out[(int64_t)b * 2 * dim + dim + i];
            s = 3.0 * tanh(r / 3.0);
            yi = dir > 0 ? ai * exp(s) + t : (ai - t) * exp(-s);
            acc += s;
        }
        y[(int64_t)b * dim + i] = yi;
        if (s_out) s_out[(int64_t)b * dim + i] = s;
    }
    sum_s[b] += acc;
}

// Affine normalisation around the coupling stack: forward x = mu + sigma u,
// inverse u = (x - mu) / sigma; sum_s[b] += sum log sigma in both directions.
__global__ __launch_bounds__(256) void affine_kernel(int n, int dim, int dir, const double *__restrict__ mu,
                                                     const double *__restrict__ log_sigma,
                                                     const double *__restrict__ a, double *__restrict__ y,
                                                     double *__restrict__ sum_s)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double acc = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double v = a[(int64_t)b * dim + i];
        y[(int64_t)b * dim + i] = dir > 0 ? mu[i] + exp(log_sigma[i]) * v : (v - mu[i]) * exp(-log_sigma[i]);
        acc += log_sigma[i];
    }
    sum_s[b] += acc;
}

// log q = -|z|^2/2 - dim/2 log(2 pi) - sum_s; the per-row training loss is
// |z|^2/2 + sum_s (the negative log density up to the constant).
__global__ __launch_bounds__(256) void base_density_kernel(int n, int dim, const double *__restrict__ z,
                                                           const double *__restrict__ sum_s,
                                                           double *__restrict__ logq, double *__restrict__ loss)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double zz = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double v = z[(int64_t)b * dim + i];
        zz += v * v;
    }
    const double l = 0.5 * zz + sum_s[b];
    if (logq) logq[b] = -l - 0.5 * dim * 1.8378770664093453;   // log(2 pi)
    if (loss) loss[b] = l;
}

// ---------------------------------------------------------------- training backward
// g = d loss / d z for loss = mean_b(|z_b|^2/2 + sum_s_b): z / n.
__global__ __launch_bounds__(256) void grad_init_kernel(int n, int dim, const double *__restrict__ z,
                                                        double *__restrict__ g)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * dim) return;
    g[idx] = z[idx] / (double)n;
}

// Backward of one inverse coupling x = (y - t) e^{-s} (T dims), x_C = y_C, with
// the loss term sum_T s / n.  g = d loss / d x.  Writes d loss / d(r, t) as
// BF16 and FP32 rows of kOutPad, and the direct part of d loss / d y (the MLP's
// contribution to the conditioning dimensions is added later).
__global__ __launch_bounds__(256) void coupling_inv_backward_kernel(int n, int dim, unsigned cond,
                                                                    const double *__restrict__ g,
                                                                    const double *__restrict__ x,
                                                                    const double *__restrict__ s,
                                                                    uint16_t *__restrict__ dout_b,
                                                                    float *__restrict__ dout_f,
                                                                    double *__restrict__ gy)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double inv_n = 1.0 / (double)n;
    for (int i = 0; i < kOutPad; ++i) {
        dout_b[(int64_t)b * kOutPad + i] = 0;
        dout_f[(int64_t)b * kOutPad + i] = 0.f;
    }
    for (int i = 0; i < dim; ++i) {
        const int64_t o = (int64_t)b * dim + i;
        if ((cond >> i) & 1u) {
            gy[o] = g[o];
        } else {
            const double si = s[o], e = exp(-si);
            const double dt = -g[o] * e;
            const double ds = -g[o] * x[o] + inv_n;
            const double dr = ds * (1.0 - (si / 3.0) * (si / 3.0));
            gy[o] = g[o] * e;
            dout_f[(int64_t)b * kOutPad + i] = (float)dr;
            dout_f[(int64_t)b * kOutPad + dim + i] = (float)dt;
            dout_b[(int64_t)b * kOutPad + i] = f32_to_bf16((float)dr);
            dout_b[(int64_t)b * kOutPad + dim + i] = f32_to_bf16((float)dt);
        }
    }
}

// dpre = dh * (h > 0) in place (FP32) and as BF16.
__global__ __launch_bounds__(256) void relu_backward_kernel(int64_t count, float *__restrict__ dh,
                                                            const uint16_t *__restrict__ h, uint16_t *__restrict__ db)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    const float v = (h[idx] & 0x7fffu) != 0 && !(h[idx] & 0x8000u) ? dh[idx] : 0.f;
    dh[idx] = v;
    db[idx] = f32_to_bf16(v);
}

// out[j] = sum_b m[b][j] (fixed order over b), j < cols.
// Column sums of m [rows][cols] (leading dimension ld) in two passes: slice
// y of the rows into part[y][cols] (FP64), then the slices in order.
constexpr int kColSlices = 32;

__global__ __launch_bounds__(256) void column_partial_kernel(int rows, int cols, int ld, const float *__restrict__ m,
                                                             double *__restrict__ part)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    const int per = (rows + kColSlices - 1) / kColSlices;
    const int r0 = (int)blockIdx.y * per, r1 = min(rows, r0 + per);
    double acc = 0.0;
    for (int b = r0; b < r1; ++b) acc += (double)m[(int64_t)b * ld + j];
    part[(int64_t)blockIdx.y * cols + j] = acc;
}

__global__ __launch_bounds__(256) void column_finish_kernel(int cols, const double *__restrict__ part,
                                                            float *__restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    double acc = 0.0;
    for (int y = 0; y < kColSlices; ++y) acc += part[(int64_t)y * cols + j];
    out[j] = (float)acc;
}

// d loss / d y for the conditioning dimensions: add the MLP input gradient.
__global__ __launch_bounds__(256) void add_input_grad_kernel(int n, int dim, unsigned cond,
                                                             const float *__restrict__ dxm, double *__restrict__ gy)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * dim) return;
    const int i = idx % dim;
    if ((cond >> i) & 1u) gy[idx] += (double)dxm[idx];
}

// Adam (Kingma & Ba 2015) on FP32 master parameters.
__global__ __launch_bounds__(256) void adam_kernel(int64_t count, float *__restrict__ p, const float *__restrict__ grad,
                                                   float *__restrict__ m, float *__restrict__ v, float lr, float beta1,
                                                   float beta2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 copies of the weight matrices (FP32 master -> BF16).
__global__ __launch_bounds__(256) void to_bf16_kernel(int64_t count, const float *__restrict__ src,
                                                      uint16_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    dst[i] = f32_to_bf16(src[i]);
}

__global__ __launch_bounds__(256) void zero_kernel(int64_t n, double *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// mean of loss[0..n) into out[0] (one block, fixed order).
__global__ __launch_bounds__(256) void mean_kernel(int n, const double *__restrict__ loss, double *__restrict__ out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) acc += loss[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / (double)n;
}

}  // namespace flow
}  // namespace gw

// ================================================================ host side
struct gw_flow {
    int device = 0;
    int dim = 0, layers = 0, hidden = 0;
    std::vector<unsigned> cond;           // conditioning mask per layer
    int64_t per_layer = 0, n_params = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    uint16_t *wb = nullptr;               // BF16 copy of params
    double *mu = nullptr, *log_sigma = nullptr;
    int64_t adam_t = 0;
    // batch scratch, capacity `cap` rows
    int64_t cap = 0;
    double *bound = nullptr;              // [layers + 2][cap][dim]
    double *s_store = nullptr;            // [layers][cap][dim]
    double *sum_s = nullptr, *loss = nullptr, *g = nullptr, *gy = nullptr;
    uint16_t *xm_b = nullptr;             // [layers][cap][kInPad]
    uint16_t *h1_b = nullptr, *h2_b = nullptr;   // [layers][cap][hidden]
    float *out_f = nullptr;               // [cap][2 dim]
    float *dout_f = nullptr;              // [cap][kOutPad]
    uint16_t *dout_b = nullptr;           // [cap][kOutPad]
    float *dh = nullptr;                  // [cap][hidden]
    uint16_t *dpre_b = nullptr;           // [cap][hidden]
    float *dxm = nullptr;                 // [cap][dim]
    float *splitk = nullptr;              // split-K partials of the weight gradients
    double *colpart = nullptr;            // column-sum partials [kColSlices][max(hidden, 2 dim)]
};

namespace {

using gw::flow::GemmArgs;
using gw::flow::kInPad;
using gw::flow::kOutPad;

int fail(int code, const std::string &m) { return gw::set_error(code, m); }
int hip_fail(hipError_t e, const char *where)
{
    return fail(GW_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

struct DeviceGuard {
    int previous = -1;
    bool ok = true;
    explicit DeviceGuard(int device)
    {
        if (hipGetDevice(&previous) != hipSuccess) { ok = false; return; }
        if (previous != device && hipSetDevice(device) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int now = -1;
        if (previous >= 0 && hipGetDevice(&now) == hipSuccess && now != previous) (void)hipSetDevice(previous);
    }
};

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// offsets of one layer's parameters (floats)
struct LayerOff { int64_t w1, b1, w2, b2, w3, b3; };
LayerOff layer_off(const gw_flow *f, int l)
{
    const int64_t D = f->dim, H = f->hidden;
    LayerOff o;
    o.w1 = l * f->per_layer;
    o.b1 = o.w1 + H * D;
    o.w2 = o.b1 + H;
    o.b2 = o.w2 + H * H;
    o.w3 = o.b2 + H;
    o.b3 = o.w3 + 2 * D * H;
    return o;
}

template <typename T>
hipError_t alloc(T **p, int64_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)std::max<int64_t>(count, 1));
}

void free_batch(gw_flow *f)
{
    void *ptrs[] = {f->bound, f->s_store, f->sum_s, f->loss, f->g, f->gy, f->xm_b, f->h1_b, f->h2_b,
                    f->out_f, f->dout_f, f->dout_b, f->dh, f->dpre_b, f->dxm, f->splitk, f->colpart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    f->bound = f->s_store = f->sum_s = f->loss = f->g = f->gy = f->colpart = nullptr;
    f->xm_b = f->h1_b = f->h2_b = f->dout_b = f->dpre_b = nullptr;
    f->out_f = f->dout_f = f->dh = f->dxm = f->splitk = nullptr;
    f->cap = 0;
}

int ensure_batch(gw_flow *f, int64_t n)
{
    if (n <= f->cap) return GW_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    free_batch(f);
    const int64_t c = std::max<int64_t>(n, 256);
    const int64_t D = f->dim, H = f->hidden, L = f->layers;
    if (alloc(&f->bound, (L + 2) * c * D) || alloc(&f->s_store, L * c * D) || alloc(&f->sum_s, c) ||
        alloc(&f->loss, c) || alloc(&f->g, c * D) || alloc(&f->gy, c * D) || alloc(&f->xm_b, L * c * kInPad) ||
        alloc(&f->h1_b, L * c * H) || alloc(&f->h2_b, L * c * H) || alloc(&f->out_f, c * 2 * D) ||
        alloc(&f->dout_f, c * kOutPad) || alloc(&f->dout_b, c * kOutPad) || alloc(&f->dh, c * H) ||
        alloc(&f->dpre_b, c * H) || alloc(&f->dxm, c * D) ||
        alloc(&f->splitk, (int64_t)gw::flow::kMaxSplit * std::max<int64_t>(H, 2 * D) * H) ||
        alloc(&f->colpart, (int64_t)gw::flow::kColSlices * std::max<int64_t>(H, 2 * D))) {
        free_batch(f);
        return fail(GW_ENOMEM, "flow batch buffers");
    }
    f->cap = c;
    return GW_OK;
}

double *boundary(gw_flow *f, int i) { return f->bound + (int64_t)i * f->cap * f->dim; }

// The MLP of layer l on the masked input of rows [0, n): writes out_f (r, t)
// and keeps the BF16 activations of layer l for the backward pass.
hipError_t mlp_forward(gw_flow *f, int l, int n, const double *a, hipStream_t s)
{
    const int D = f->dim, H = f->hidden;
    const LayerOff o = layer_off(f, l);
    uint16_t *xm = f->xm_b + (int64_t)l * f->cap * kInPad;
    uint16_t *h1 = f->h1_b + (int64_t)l * f->cap * H;
    uint16_t *h2 = f->h2_b + (int64_t)l * f->cap * H;
    hipLaunchKernelGGL(gw::flow::mask_input_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, f->cond[l], a, xm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GemmArgs g1{n, H, D, xm, kInPad, 1, f->wb + o.w1, 1, D, nullptr, 0, h1, H, f->params + o.b1, 1};
    if ((e = gw::flow::gemm_bf16(g1, s)) != hipSuccess) return e;
    GemmArgs g2{n, H, H, h1, H, 1, f->wb + o.w2, 1, H, nullptr, 0, h2, H, f->params + o.b2, 1};
    if ((e = gw::flow::gemm_bf16(g2, s)) != hipSuccess) return e;
    GemmArgs g3{n, 2 * D, H, h2, H, 1, f->wb + o.w3, 1, H, f->out_f, 2 * D, nullptr, 0, f->params + o.b3, 0};
    return gw::flow::gemm_bf16(g3, s);
}

#define GW_TRY(expr)                         \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

hipError_t zero(int64_t n, double *p, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gw::flow::zero_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, p);
    return hipGetLastError();
}

// Inverse pass x -> z over rows [0, n): boundary L+1 = x, boundary L = the
// normalised x, then the couplings L-1 .. 0 invert down to boundary 0 = z;
// sum_s = sum log sigma + sum over layers of sum_T s.  Activations of every
// layer are kept for the backward pass.
hipError_t inverse_pass(gw_flow *f, int n, const double *x, hipStream_t s)
{
    const int D = f->dim, L = f->layers;
    GW_TRY(zero(n, f->sum_s, s));
    GW_TRY(hipMemcpyAsync(boundary(f, L + 1), x, sizeof(double) * (size_t)n * D, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(gw::flow::affine_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, -1, f->mu, f->log_sigma,
                       boundary(f, L + 1), boundary(f, L), f->sum_s);
    GW_TRY(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        GW_TRY(mlp_forward(f, l, n, boundary(f, l + 1), s));
        hipLaunchKernelGGL(gw::flow::coupling_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, f->cond[l], -1,
                           boundary(f, l + 1), f->out_f, boundary(f, l), f->sum_s,
                           f->s_store + (int64_t)l * f->cap * D);
        GW_TRY(hipGetLastError());
    }
    return hipSuccess;
}

// Forward pass z -> x over rows [0, n): boundary 0 = z, couplings 0 .. L-1,
// then the affine normalisation to boundary L+1 = x; sum_s as in the inverse.
hipError_t forward_pass(gw_flow *f, int n, const double *z, hipStream_t s)
{
    const int D = f->dim, L = f->layers;
    GW_TRY(zero(n, f->sum_s, s));
    GW_TRY(hipMemcpyAsync(boundary(f, 0), z, sizeof(double) * (size_t)n * D, hipMemcpyDeviceToDevice, s));
    for (int l = 0; l < L; ++l) {
        GW_TRY(mlp_forward(f, l, n, boundary(f, l), s));
        hipLaunchKernelGGL(gw::flow::coupling_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, f->cond[l], 1,
                           boundary(f, l), f->out_f, boundary(f, l + 1), f->sum_s, nullptr);
        GW_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(gw::flow::affine_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, 1, f->mu, f->log_sigma,
                       boundary(f, L), boundary(f, L + 1), f->sum_s);
    return hipGetLastError();
}

// Gradient of the mean negative log density of rows x[0, n) with respect to
// every parameter (into f->grads); the mean loss goes to loss_out (device).
// Column sums of m [n][cols] (leading dimension ld) into out [cols].
hipError_t column_sum(gw_flow *f, int n, int cols, int ld, const float *m, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(gw::flow::column_partial_kernel, dim3(blocks_for(cols), gw::flow::kColSlices), dim3(256), 0, s,
                       n, cols, ld, m, f->colpart);
    GW_TRY(hipGetLastError());
    hipLaunchKernelGGL(gw::flow::column_finish_kernel, dim3(blocks_for(cols)), dim3(256), 0, s, cols, f->colpart, out);
    return hipGetLastError();
}

hipError_t gradients(gw_flow *f, int n, const double *x, double *loss_out, hipStream_t s)
{
    const int D = f->dim, H = f->hidden, L = f->layers;
    // weight gradients sum over the n rows: split K = n into slices of >= 256 rows
    const int split = std::max(1, std::min(gw::flow::kMaxSplit, n / 256));
    GW_TRY(inverse_pass(f, n, x, s));
    hipLaunchKernelGGL(gw::flow::base_density_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, boundary(f, 0),
                       f->sum_s, nullptr, f->loss);
    GW_TRY(hipGetLastError());
    if (loss_out) {
        hipLaunchKernelGGL(gw::flow::mean_kernel, dim3(1), dim3(256), 0, s, n, f->loss, loss_out);
        GW_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(gw::flow::grad_init_kernel, dim3(blocks_for((int64_t)n * D)), dim3(256), 0, s, n, D,
                       boundary(f, 0), f->g);
    GW_TRY(hipGetLastError());
    // the inverse pass applied couplings L-1 .. 0; go back through 0 .. L-1
    for (int l = 0; l < L; ++l) {
        const LayerOff o = layer_off(f, l);
        const uint16_t *xm = f->xm_b + (int64_t)l * f->cap * kInPad;
        const uint16_t *h1 = f->h1_b + (int64_t)l * f->cap * H;
        const uint16_t *h2 = f->h2_b + (int64_t)l * f->cap * H;
        hipLaunchKernelGGL(gw::flow::coupling_inv_backward_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D,
                           f->cond[l], f->g, boundary(f, l), f->s_store + (int64_t)l * f->cap * D, f->dout_b,
                           f->dout_f, f->gy);
        GW_TRY(hipGetLastError());
        // layer 3: dW3 = dout^T h2, db3 = colsum(dout), dh2 = dout W3
        GemmArgs gw3{2 * D, H, n, f->dout_b, 1, kOutPad, h2, H, 1, f->grads + o.w3, H, nullptr, 0, nullptr, 0,
                     split, f->splitk};
        GW_TRY(gw::flow::gemm_bf16(gw3, s));
        GW_TRY(column_sum(f, n, 2 * D, kOutPad, f->dout_f, f->grads + o.b3, s));
        GemmArgs gh2{n, H, 2 * D, f->dout_b, kOutPad, 1, f->wb + o.w3, H, 1, f->dh, H, nullptr, 0, nullptr, 0};
        GW_TRY(gw::flow::gemm_bf16(gh2, s));
        hipLaunchKernelGGL(gw::flow::relu_backward_kernel, dim3(blocks_for((int64_t)n * H)), dim3(256), 0, s,
                           (int64_t)n * H, f->dh, h2, f->dpre_b);
        GW_TRY(hipGetLastError());
        // layer 2: dW2 = dpre2^T h1, db2 = colsum(dpre2), dh1 = dpre2 W2
        GemmArgs gw2{H, H, n, f->dpre_b, 1, H, h1, H, 1, f->grads + o.w2, H, nullptr, 0, nullptr, 0,
                     split, f->splitk};
        GW_TRY(gw::flow::gemm_bf16(gw2, s));
        GW_TRY(column_sum(f, n, H, H, f->dh, f->grads + o.b2, s));
        GemmArgs gh1{n, H, H, f->dpre_b, H, 1, f->wb + o.w2, H, 1, f->dh, H, nullptr, 0, nullptr, 0};
        // dh1 overwrites dh only after the two reads above have been enqueued before it (stream order)
        GW_TRY(gw::flow::gemm_bf16(gh1, s));
        hipLaunchKernelGGL(gw::flow::relu_backward_kernel, dim3(blocks_for((int64_t)n * H)), dim3(256), 0, s,
                           (int64_t)n * H, f->dh, h1, f->dpre_b);
        GW_TRY(hipGetLastError());
        // layer 1: dW1 = dpre1^T xm, db1 = colsum(dpre1), dxm = dpre1 W1
        GemmArgs gw1{H, D, n, f->dpre_b, 1, H, xm, kInPad, 1, f->grads + o.w1, D, nullptr, 0, nullptr, 0,
                     split, f->splitk};
        GW_TRY(gw::flow::gemm_bf16(gw1, s));
        GW_TRY(column_sum(f, n, H, H, f->dh, f->grads + o.b1, s));
        GemmArgs gx{n, D, H, f->dpre_b, H, 1, f->wb + o.w1, D, 1, f->dxm, D, nullptr, 0, nullptr, 0};
        GW_TRY(gw::flow::gemm_bf16(gx, s));
        hipLaunchKernelGGL(gw::flow::add_input_grad_kernel, dim3(blocks_for((int64_t)n * D)), dim3(256), 0, s, n, D,
                           f->cond[l], f->dxm, f->gy);
        GW_TRY(hipGetLastError());
        std::swap(f->g, f->gy);      // d loss / d(boundary l + 1)
    }
    return hipSuccess;
}

hipError_t refresh_bf16(gw_flow *f, hipStream_t s)
{
    hipLaunchKernelGGL(gw::flow::to_bf16_kernel, dim3(blocks_for(f->n_params)), dim3(256), 0, s, f->n_params,
                       f->params, f->wb);
    return hipGetLastError();
}

int check_flow_call(gw_flow *f, const void *a, int64_t n)
{
    if (!f) return fail(GW_EINVAL, "flow is NULL");
    if (n < 0 || n > 0x7fffffff) return fail(GW_EINVAL, "row count out of range");
    if (n > 0 && !a) return fail(GW_EINVAL, "NULL array");
    return GW_OK;
}

}  // namespace

extern "C" {

int gw_flow_create(gw_flow **out, int device, int dim, int n_layers, int hidden, const unsigned *cond_masks)
{
    if (!out) return fail(GW_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim < 2 || dim > kInPad || 2 * dim > kOutPad) return fail(GW_EINVAL, "dim must be in 2..16");
    if (n_layers < 1 || n_layers > 64 || hidden < 1 || hidden > 4096) return fail(GW_EINVAL, "bad flow shape");
    if (!cond_masks) return fail(GW_EINVAL, "cond_masks is NULL");
    if (int rc = gw::check_build()) return rc;
    int dev = device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(GW_EDEVICE, "hipGetDevice");
    DeviceGuard g(dev);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the device");
    auto *f = new gw_flow();
    f->device = dev;
    f->dim = dim;
    f->layers = n_layers;
    f->hidden = hidden;
    f->cond.assign(cond_masks, cond_masks + n_layers);
    const int64_t D = dim, H = hidden;
    f->per_layer = H * D + H + H * H + H + 2 * D * H + 2 * D;
    f->n_params = f->per_layer * n_layers;
    if (alloc(&f->params, f->n_params) || alloc(&f->grads, f->n_params) || alloc(&f->adam_m, f->n_params) ||
        alloc(&f->adam_v, f->n_params) || alloc(&f->wb, f->n_params) || alloc(&f->mu, dim) ||
        alloc(&f->log_sigma, dim)) {
        gw_flow_destroy(f);
        return fail(GW_ENOMEM, "flow parameters");
    }
    *out = f;
    return GW_OK;
}

int gw_flow_destroy(gw_flow *f)
{
    if (!f) return GW_OK;
    DeviceGuard g(f->device);
    (void)hipDeviceSynchronize();
    free_batch(f);
    void *ptrs[] = {f->params, f->grads, f->adam_m, f->adam_v, f->wb, f->mu, f->log_sigma};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete f;
    return GW_OK;
}

int64_t gw_flow_num_params(const gw_flow *f) { return f ? f->n_params : 0; }

int gw_flow_set_params(gw_flow *f, const float *params, const double *mu, const double *log_sigma)
{
    if (!f || !params || !mu || !log_sigma) return fail(GW_EINVAL, "NULL argument");
    DeviceGuard g(f->device);
    hipError_t e;
    if ((e = hipMemcpy(f->params, params, sizeof(float) * f->n_params, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(f->mu, mu, sizeof(double) * f->dim, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(f->log_sigma, log_sigma, sizeof(double) * f->dim, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(f->adam_m, 0, sizeof(float) * f->n_params)) != hipSuccess ||
        (e = hipMemset(f->adam_v, 0, sizeof(float) * f->n_params)) != hipSuccess ||
        (e = refresh_bf16(f, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(e, "gw_flow_set_params");
    f->adam_t = 0;
    return GW_OK;
}

int gw_flow_get_params(const gw_flow *f, float *params, double *mu, double *log_sigma)
{
    if (!f || !params || !mu || !log_sigma) return fail(GW_EINVAL, "NULL argument");
    DeviceGuard g(f->device);
    hipError_t e;
    if ((e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(params, f->params, sizeof(float) * f->n_params, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(mu, f->mu, sizeof(double) * f->dim, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(log_sigma, f->log_sigma, sizeof(double) * f->dim, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "gw_flow_get_params");
    return GW_OK;
}

int gw_flow_forward(gw_flow *f, const double *z, int64_t n, double *x_out, double *logq_out, hipStream_t stream)
{
    if (int rc = check_flow_call(f, z, n)) return rc;
    if (n > 0 && !x_out) return fail(GW_EINVAL, "x_out is NULL");
    if (n == 0) return GW_OK;
    DeviceGuard g(f->device);
    if (int rc = ensure_batch(f, n)) return rc;
    hipError_t e = forward_pass(f, (int)n, z, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(x_out, boundary(f, f->layers + 1), sizeof(double) * n * f->dim, hipMemcpyDeviceToDevice,
                           stream);
    if (e == hipSuccess && logq_out) {
        hipLaunchKernelGGL(gw::flow::base_density_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, (int)n, f->dim,
                           boundary(f, 0), f->sum_s, logq_out, nullptr);
        e = hipGetLastError();
    }
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_flow_forward");
}

int gw_flow_inverse(gw_flow *f, const double *x, int64_t n, double *z_out, double *logq_out, hipStream_t stream)
{
    if (int rc = check_flow_call(f, x, n)) return rc;
    if (n == 0) return GW_OK;
    DeviceGuard g(f->device);
    if (int rc = ensure_batch(f, n)) return rc;
    hipError_t e = inverse_pass(f, (int)n, x, stream);
    if (e == hipSuccess && z_out)
        e = hipMemcpyAsync(z_out, boundary(f, 0), sizeof(double) * n * f->dim, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && logq_out) {
        hipLaunchKernelGGL(gw::flow::base_density_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, (int)n, f->dim,
                           boundary(f, 0), f->sum_s, logq_out, nullptr);
        e = hipGetLastError();
    }
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_flow_inverse");
}

int gw_flow_gradients(gw_flow *f, const double *x, int64_t n, float *grad_out, double *loss_out, hipStream_t stream)
{
    if (int rc = check_flow_call(f, x, n)) return rc;
    if (n == 0) return fail(GW_EINVAL, "empty batch");
    DeviceGuard g(f->device);
    if (int rc = ensure_batch(f, n)) return rc;
    hipError_t e = gradients(f, (int)n, x, loss_out, stream);
    if (e == hipSuccess && grad_out)
        e = hipMemcpyAsync(grad_out, f->grads, sizeof(float) * f->n_params, hipMemcpyDeviceToDevice, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_flow_gradients");
}

int gw_flow_train_step(gw_flow *f, const double *x, int64_t n, float lr, double *loss_out, hipStream_t stream)
{
    if (int rc = check_flow_call(f, x, n)) return rc;
    if (n == 0) return fail(GW_EINVAL, "empty batch");
    if (!(lr > 0.0f)) return fail(GW_EINVAL, "learning rate must be > 0");
    DeviceGuard g(f->device);
    if (int rc = ensure_batch(f, n)) return rc;
    hipError_t e = gradients(f, (int)n, x, loss_out, stream);
    if (e == hipSuccess) {
        ++f->adam_t;
        const float b1 = 0.9f, b2 = 0.999f;
        const float bc1 = 1.0f - (float)std::pow(b1, (double)f->adam_t);
        const float bc2 = 1.0f - (float)std::pow(b2, (double)f->adam_t);
        hipLaunchKernelGGL(gw::flow::adam_kernel, dim3(blocks_for(f->n_params)), dim3(256), 0, stream, f->n_params,
                           f->params, f->grads, f->adam_m, f->adam_v, lr, b1, b2, 1e-8f, bc1, bc2);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = refresh_bf16(f, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_flow_train_step");
}

}  // extern "C"

GW_DEFINE_SOURCE_HASH(flow)
