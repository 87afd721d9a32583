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
// FP32 -> BF16, rounding to nearest even (one v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---------------------------------------------------------------- GEMM on MFMA
// C[M x N] = A[M x K] B[K x N] (+ bias[N]) (ReLU if relu), FP32 accumulation.
// A(i, k) = A[i sa_i + k sa_k], B(k, j) = B[k sb_k + j sb_j], both BF16.
// Block: 256 threads, a 64 x 64 output tile (blockIdx.z: K slice when split).
// The K range goes through LDS in chunks of up to 128: both operands are
// stored k-contiguous (A as [row][k], B as [col][k]) so that every lane reads
// its 8 consecutive k with one 16-byte LDS load, and the next chunk's global
// loads are issued before the current chunk's products; the bias is read at
// the start, under the first wait.  (Chunks of 256, one wait for every
// product of the flow, measured no faster: the LDS then holds two blocks per
// CU instead of four.)  Global loads move 8 BF16 (16 bytes)
// along whichever index the operand is contiguous in (template flags: A_KC /
// B_KC when contiguous in k), element by element where a vector would leave
// the matrix or is misaligned.  Each of the 4 waves owns a 32 x 32 quarter as
// 2 x 2 tiles of v_mfma_f32_16x16x32_bf16: lane l supplies A(row l%16, 8
// consecutive k of group l/16) and B(the same k, col l%16), A and B with the
// same k order, and receives D(row 4(l/16)+0..3, col l%16).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kTileMN = 64;           // output tile edge
constexpr int kChunkK = 128;          // K per LDS chunk
constexpr int kLdsK = kChunkK + 8;    // LDS row length in BF16 (16-byte aligned rows, staggered banks)
constexpr int kVecPerThread = kTileMN * kChunkK / 8 / 256;   // 16-byte vectors per thread and operand

__device__ __forceinline__ uint16_t u16_at(uint4 v, int e)
{
    const uint32_t w = e < 2 ? v.x : e < 4 ? v.y : e < 6 ? v.z : v.w;
    return (uint16_t)((e & 1) ? (w >> 16) : (w & 0xffffu));
}

// 8 BF16 of a matrix with strides (s_c, s_o) along its contiguous and other
// index: elements (c0 + e, o) for e < 8, zero where c0 + e >= c_end or the
// row is out of range (o_ok false).  vec: the 8 elements may be read as one
// aligned 16-byte vector whenever all of them are in range.
__device__ __forceinline__ uint4 load8(const uint16_t *__restrict__ base, int64_t s_o, int c0, int c_end, int o,
                                       bool o_ok, bool vec)
{
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    if (!o_ok || c0 >= c_end) return r;
    const uint16_t *p = base + (int64_t)o * s_o + c0;
    if (vec && c0 + 8 <= c_end) return *reinterpret_cast<const uint4 *>(p);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (c0 + e < c_end) w[e >> 1] |= (uint32_t)p[e] << ((e & 1) * 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// One operand's share of a chunk: KC = true when the operand is contiguous
// in k.  Tile rows (A rows or B columns) t0 .. t0 + 63 below t_end, k in
// [k0, k0 + kc) below k_hi.  Vector v of this thread: KC, tile row
// v / (kChunkK / 8) and k group v % (kChunkK / 8) (8 k each); otherwise
// k = v / 8 and tile-row group v % 8.
template <bool KC>
__device__ __forceinline__ void load_chunk(const uint16_t *__restrict__ X, int64_t s_t, int64_t s_k, int t0,
                                           int t_end, int k0, int kc, int k_hi, bool vec, uint4 (&reg)[kVecPerThread])
{
    const int tid = threadIdx.x;
    if (KC && vec && t0 + kTileMN <= t_end && k0 + kc <= k_hi) {
        // the whole chunk lies inside the matrix (the same for every thread
        // of the block): one 16-byte load per vector, rows kRowsPerPass apart
        constexpr int kGroups = kChunkK / 8, kRowsPerPass = 256 / kGroups;
        const int kg = tid % kGroups;
        const uint16_t *p = X + (int64_t)(t0 + tid / kGroups) * s_t + (k0 + 8 * kg);
        const int64_t step = (int64_t)kRowsPerPass * s_t;
#pragma unroll
        for (int e = 0; e < kVecPerThread; ++e)
            reg[e] = 8 * kg < kc ? *reinterpret_cast<const uint4 *>(p + e * step) : make_uint4(0u, 0u, 0u, 0u);
        return;
    }
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e) {
        const int v = tid + 256 * e;
        if (KC) {
            const int t = v / (kChunkK / 8), kg = v % (kChunkK / 8);
            const int k = k0 + 8 * kg;
            // contiguous in k: the 8 elements run along k, rows along t
            reg[e] = (8 * kg < kc) ? load8(X, s_t, k, k_hi, t0 + t, t0 + t < t_end, vec) : make_uint4(0u, 0u, 0u, 0u);
        } else {
            const int kk = v >> 3, tg = v & 7;
            const int k = k0 + kk;
            reg[e] = (kk < kc) ? load8(X, s_k, t0 + 8 * tg, t_end, k, k < k_hi, vec) : make_uint4(0u, 0u, 0u, 0u);
        }
    }
}

template <bool KC>
__device__ __forceinline__ void store_chunk(uint16_t (*lds)[kLdsK], int kc, const uint4 (&reg)[kVecPerThread])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e) {
        const int v = tid + 256 * e;
        if (KC) {
            const int t = v / (kChunkK / 8), kg = v % (kChunkK / 8);
            if (8 * kg < kc) *reinterpret_cast<uint4 *>(&lds[t][8 * kg]) = reg[e];
        } else {
            const int kk = v >> 3, tg = v & 7;
            if (kk < kc) {
#pragma unroll
                for (int q = 0; q < 8; ++q) lds[8 * tg + q][kk] = u16_at(reg[e], q);
            }
        }
    }
}

// K of the chunk starting at k0: up to kChunkK, rounded up to the 32 of one product step.
__device__ __forceinline__ int chunk_len(int k0, int k_hi) { return min(kChunkK, (k_hi - k0 + 31) / 32 * 32); }

// The output tile (bx, by) of K slice bz; LDS and barriers are the block's.
template <bool A_KC, bool B_KC>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int vec_a, int vec_b, int bx, int by, int bz)
{
    __shared__ __align__(16) uint16_t as[kTileMN][kLdsK];
    __shared__ __align__(16) uint16_t bs[kTileMN][kLdsK];
    __shared__ double colred[2][4][kTileMN];   // column sums: [row half][lane group][tile column]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int row0 = by * kTileMN, col0 = bx * kTileMN;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    // K slice of this block (the whole range unless split), a multiple of 32
    const int ks = ((g.K + g.split - 1) / g.split + 31) / 32 * 32;
    const int k_lo = bz * ks, k_hi = min(g.K, k_lo + ks);
    float4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};

    const int rq = 4 * (lane >> 4), lc = lane & 15;
    const bool to_partial = g.split > 1 || g.defer;
    float bias[2] = {0.f, 0.f};
    if (g.bias && !to_partial) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int j = col0 + wc + 16 * b + lc;
            bias[b] = j < g.N ? g.bias[j] : 0.f;
        }
    }
    uint4 ra[kVecPerThread], rb[kVecPerThread];
    if (k_lo < k_hi) {
        const int kc = chunk_len(k_lo, k_hi);
        load_chunk<A_KC>(g.A, g.sa_i, g.sa_k, row0, g.M, k_lo, kc, k_hi, vec_a != 0, ra);
        load_chunk<B_KC>(g.B, g.sb_j, g.sb_k, col0, g.N, k_lo, kc, k_hi, vec_b != 0, rb);
    }
    for (int k0 = k_lo; k0 < k_hi; k0 += kChunkK) {
        const int kc = chunk_len(k0, k_hi);
        __syncthreads();                       // the previous chunk's reads are done
        store_chunk<A_KC>(as, kc, ra);
        store_chunk<B_KC>(bs, kc, rb);
        __syncthreads();
        const int kn = k0 + kChunkK;
        if (kn < k_hi) {                       // next chunk in flight during the products
            const int kcn = chunk_len(kn, k_hi);
            load_chunk<A_KC>(g.A, g.sa_i, g.sa_k, row0, g.M, kn, kcn, k_hi, vec_a != 0, ra);
            load_chunk<B_KC>(g.B, g.sb_j, g.sb_k, col0, g.N, kn, kcn, k_hi, vec_b != 0, rb);
        }
        const int kq = 8 * (lane >> 4), lr = lane & 15;
        for (int kk = 0; kk < kc; kk += 32) {
            bf16x8_t av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8_t *>(&as[wr + 16 * a + lr][kk + kq]);
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const bf16x8_t *>(&bs[wc + 16 * b + lr][kk + kq]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    double csum[2] = {0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int i0 = row0 + wr + 16 * a + rq;     // this lane's 4 consecutive rows
            const int j = col0 + wc + 16 * b + lc;
            if (j >= g.N) continue;
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + r;
                v[r] = acc[a][b][r];
                if (i >= g.M) continue;
                if (to_partial) {
                    g.partial[((int64_t)bz * g.M + i) * g.N + j] = v[r];
                    continue;
                }
                if (g.bias) v[r] += bias[b];
                if (g.relu) v[r] = v[r] > 0.f ? v[r] : 0.f;
                if (g.relu_of) {
                    const uint16_t h = g.relu_of[(int64_t)i * g.ld_relu + j];
                    v[r] = ((h & 0x7fffu) != 0 && !(h & 0x8000u)) ? v[r] : 0.f;
                }
                if (g.C) g.C[(int64_t)i * g.ldc + j] = v[r];
                if (g.Cb) g.Cb[(int64_t)i * g.ldcb + j] = f32_to_bf16(v[r]);
                if (g.add_to && ((g.add_mask >> j) & 1u)) g.add_to[(int64_t)i * g.ld_add + j] += (double)v[r];
                csum[b] += (double)v[r];
            }
            if (g.CbT && !to_partial) {
                // transposed BF16 copy: the 4 rows are consecutive in column j's row of CbT
                uint16_t *t = g.CbT + (int64_t)j * g.ldcbT + i0;
                if (i0 + 3 < g.M) {
                    const uint32_t lo = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
                    const uint32_t hi = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
                    *reinterpret_cast<uint2 *>(t) = make_uint2(lo, hi);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (i0 + r < g.M) t[r] = f32_to_bf16(v[r]);
                }
            }
        }
    if (g.col_part && !to_partial) {
        // the block's 64 rows: each lane's 8, then the 4 lane groups and the
        // two row halves, in that fixed order
#pragma unroll
        for (int b = 0; b < 2; ++b) colred[wave >> 1][lane >> 4][wc + 16 * b + lc] = csum[b];
        __syncthreads();
        const int j = col0 + tid;
        if (tid < kTileMN && j < g.N) {
            double t = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) t += colred[h][q][tid];
            g.col_part[(int64_t)by * g.N + j] = t;
        }
    }
}

template <bool A_KC, bool B_KC>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g, int vec_a, int vec_b)
{
    gemm_tile<A_KC, B_KC>(g, vec_a, vec_b, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Up to three independent products, k-contiguous operands, in one launch:
// blocks [start[p], start[p + 1]) work on product p, tile x fastest, then
// tile y, then K slice.
struct GemmGroup {
    GemmArgs g0, g1, g2;
    int va[3], vb[3], gx[3], gy[3], start[4];
    LayerStrides ls;                      // per-layer strides (launches over several layers)
};

// Product p of the group for layer `layer`: its operands moved by the layer strides.
__device__ __forceinline__ void gemm_group_tile(GemmArgs g, const GemmGroup &gg, int p, int layer, int bx, int by,
                                                int bz)
{
    g.A += layer * gg.ls.sA[p];
    g.B += layer * gg.ls.sB[p];
    g.partial += layer * gg.ls.sP[p];
    gemm_tile<true, true>(g, gg.va[p], gg.vb[p], bx, by, bz);
}

// Blocks layer by layer, each layer's as start[] lays out its three products.
__global__ __launch_bounds__(256) void gemm_group_kernel(GemmGroup gg)
{
    const int layer = (int)blockIdx.x / gg.start[3];
    const int b = (int)blockIdx.x - layer * gg.start[3];
    const int p = (b >= gg.start[1]) + (b >= gg.start[2]);
    const int local = b - gg.start[p];
    const int bx = local % gg.gx[p], rest = local / gg.gx[p];
    const int by = rest % gg.gy[p], bz = rest / gg.gy[p];
    if (p == 0)
        gemm_group_tile(gg.g0, gg, 0, layer, bx, by, bz);
    else if (p == 1)
        gemm_group_tile(gg.g1, gg, 1, layer, bx, by, bz);
    else
        gemm_group_tile(gg.g2, gg, 2, layer, bx, by, bz);
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

// An operand can be read in 16-byte vectors along its contiguous index when
// that stride is 1, the other stride is a multiple of 8 elements and the base
// is 16-byte aligned (vectors start at multiples of 8 along the contiguous index).
static bool vector_ok(const uint16_t *p, int64_t s_contig, int64_t s_other)
{
    return s_contig == 1 && s_other % 8 == 0 && (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Three products with k-contiguous operands (sa_k = sb_k = 1) in one
// launch; each as gemm_bf16 would run it (split-K with defer, no reduce kernel).
hipError_t gemm_bf16_group3(const GemmArgs &a, const GemmArgs &b, const GemmArgs &c, hipStream_t stream, int layers,
                            const LayerStrides *strides)
{
    if (layers < 1 || (layers > 1 && !strides)) return hipErrorInvalidValue;
    const GemmArgs *gs[3] = {&a, &b, &c};
    GemmGroup gg;
    gg.g0 = a;
    gg.g1 = b;
    gg.g2 = c;
    gg.ls = strides ? *strides : LayerStrides{};
    for (int p = 0; p < 3; ++p)
        if (gg.ls.sA[p] % 8 != 0 || gg.ls.sB[p] % 8 != 0 || gg.ls.sP[p] % 8 != 0) return hipErrorInvalidValue;
    int start = 0;
    for (int p = 0; p < 3; ++p) {
        const GemmArgs &g = *gs[p];
        if (g.M <= 0 || g.N <= 0 || g.sa_k != 1 || g.sb_k != 1 || g.split < 1 || g.split > kMaxSplit ||
            ((g.split > 1 || g.defer) && !g.partial) || (g.split == 1 && !g.defer))
            return hipErrorInvalidValue;
        gg.va[p] = vector_ok(g.A, g.sa_k, g.sa_i);
        gg.vb[p] = vector_ok(g.B, g.sb_k, g.sb_j);
        gg.gx[p] = (g.N + kTileMN - 1) / kTileMN;
        gg.gy[p] = (g.M + kTileMN - 1) / kTileMN;
        gg.start[p] = start;
        start += gg.gx[p] * gg.gy[p] * g.split;
    }
    gg.start[3] = start;
    if ((int64_t)start * layers > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_group_kernel, dim3((unsigned)(start * layers)), dim3(256), 0, stream, gg);
    return hipGetLastError();
}

hipError_t gemm_bf16(const GemmArgs &g, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.split < 1 || g.split > kMaxSplit || ((g.split > 1 || g.defer) && !g.partial)) return hipErrorInvalidValue;
    if ((g.col_part || g.relu_of || g.CbT || g.add_to) && (g.split > 1 || g.defer)) return hipErrorInvalidValue;
    if (g.add_to && g.N > 32) return hipErrorInvalidValue;
    // the transposed copy is written 4 rows (8 bytes) at a time
    if (g.CbT && (g.ldcbT % 4 != 0 || (reinterpret_cast<uintptr_t>(g.CbT) & 7u) != 0)) return hipErrorInvalidValue;
    // A is read along k when its k stride is 1, else along i (stride 1 required then)
    const bool a_kc = g.sa_k == 1, b_kc = g.sb_k == 1;
    if ((!a_kc && g.sa_i != 1) || (!b_kc && g.sb_j != 1)) return hipErrorInvalidValue;
    const int va = a_kc ? vector_ok(g.A, g.sa_k, g.sa_i) : vector_ok(g.A, g.sa_i, g.sa_k);
    const int vb = b_kc ? vector_ok(g.B, g.sb_k, g.sb_j) : vector_ok(g.B, g.sb_j, g.sb_k);
    const dim3 grid((g.N + kTileMN - 1) / kTileMN, (g.M + kTileMN - 1) / kTileMN, g.split);
    if (a_kc && b_kc)
        hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, stream, g, va, vb);
    else if (a_kc)
        hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, stream, g, va, vb);
    else if (b_kc)
        hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, stream, g, va, vb);
    else
        hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, stream, g, va, vb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.split == 1 || g.defer) return e;
    const int64_t total = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- coupling layers
// Row b of a [n][dim] FP64 state.  `cond` has bit i set when dimension i is
// in the layer's conditioning set.

// MLP input: the conditioning dimensions of a, the others zero, as BF16 in a
// row of kInPad entries (the GEMM's K is dim; the padding stays zero).
// The masked MLP input of the next coupling, written by the kernel that
// produces that coupling's input: row b of a as BF16 in xm[b][kInPad] with
// the dimensions outside cond zero, and with xmT given also transposed,
// xmT[i ldT + b] (for the weight gradients).  xm == nullptr: none.
struct NextMask {
    uint16_t *xm;
    uint16_t *xmT;
    int64_t ldT;
    unsigned cond;
};

__device__ __forceinline__ void write_mask(const NextMask &nm, int b, int dim, const double *__restrict__ row)
{
    if (!nm.xm) return;
    for (int i = 0; i < kInPad; ++i) {
        const bool on = i < dim && ((nm.cond >> i) & 1u);
        const uint16_t v = on ? f32_to_bf16((float)row[i]) : (uint16_t)0;
        nm.xm[(int64_t)b * kInPad + i] = v;
        if (nm.xmT) nm.xmT[i * nm.ldT + b] = v;
    }
}

// With xmT given, also the transposed copy xmT[i ldT + b] (for the weight gradients).
__global__ __launch_bounds__(256) void mask_input_kernel(int n, int dim, unsigned cond, const double *__restrict__ a,
                                                         uint16_t *__restrict__ xm, uint16_t *__restrict__ xmT,
                                                         int64_t ldT)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int i = 0; i < kInPad; ++i) {
        const bool on = i < dim && ((cond >> i) & 1u);
        const uint16_t v = on ? f32_to_bf16((float)a[(int64_t)b * dim + i]) : (uint16_t)0;
        xm[(int64_t)b * kInPad + i] = v;
        if (xmT) xmT[i * ldT + b] = v;
    }
}

// Affine coupling given the MLP output (r, t) = out[b][0..dim), out[b][dim..2dim):
//   forward (dir > 0): y_T = a_T exp(s) + t;  inverse (dir < 0): y_T = (a_T - t) exp(-s);
// s = 3 tanh(r/3); conditioning dimensions are copied.  sum_s[b] += sum_T s in
// both directions (log q = log N(z) - sum_s); s is stored when s_out is set.
// Row b of the coupling, its MLP output row at out (r at [0, dim), t at [dim, 2 dim)).
__device__ __forceinline__ void coupling_row(int b, int dim, unsigned cond, int dir, const double *__restrict__ a,
                                             const float *out, double *__restrict__ y, double *__restrict__ sum_s,
                                             double *__restrict__ s_out, const NextMask &nm)
{
    double acc = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double ai = a[(int64_t)b * dim + i];
        double yi = ai, s = 0.0;
        if (!((cond >> i) & 1u)) {
            const double r = (double)out[i];
            const double t = (double)out[dim + i];
            s = 3.0 * tanh(r / 3.0);
            yi = dir > 0 ? ai * exp(s) + t : (ai - t) * exp(-s);
            acc += s;
        }
        y[(int64_t)b * dim + i] = yi;
        if (s_out) s_out[(int64_t)b * dim + i] = s;
    }
    sum_s[b] += acc;
    write_mask(nm, b, dim, y + (int64_t)b * dim);
}

__global__ __launch_bounds__(256) void coupling_kernel(int n, int dim, unsigned cond, int dir,
                                                       const double *__restrict__ a, const float *__restrict__ out,
                                                       double *__restrict__ y, double *__restrict__ sum_s,
                                                       double *__restrict__ s_out, NextMask nm)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    coupling_row(b, dim, cond, dir, a, out + (int64_t)b * 2 * dim, y, sum_s, s_out, nm);
}

// ---------------------------------------------------------------- one coupling in one kernel
// A coupling of the flow on kLayerRows rows per block, for hidden widths
// H = 128 and 256: the MLP's three products on the matrix cores with both
// hidden activations held in LDS, then the coupling of each row.  Each of the
// 4 waves owns H/4 hidden columns; lane l works on rows l%16 and k group l/16
// as in the GEMM, with the same v_mfma_f32_16x16x32_bf16 sequence over k, so
// the activations and outputs equal the GEMM path's bit for bit.  The
// weights come straight from global memory (L2-resident) in 16-byte
// fragments: W1 with padded rows (K = kInPad, zero padding), W2 [H][H] and
// W3 [2 dim][H] as stored (out, in).
constexpr int kLayerRows = 16;

struct LayerArgs {
    int n, dim, dir;
    unsigned cond;
    const uint16_t *xm;                   // [n][kInPad] masked MLP input
    const uint16_t *w1p, *w2, *w3;
    const float *b1, *b2, *b3;
    uint16_t *h1, *h2;                    // [n][H] activations, kept for the backward pass
    uint16_t *h1T, *h2T;                  // transposed copies (training) or null
    int64_t ldT;
    const double *a;
    double *y, *sum_s, *s_out;
    NextMask nm;
};

__device__ __forceinline__ bf16x8_t ld_bf16x8(const uint16_t *p) { return *reinterpret_cast<const bf16x8_t *>(p); }

template <int H>
__device__ __forceinline__ void store_hidden(const LayerArgs &p, uint16_t (*hs)[H + 8], uint16_t *hg, uint16_t *hT,
                                             const float4_t (&acc)[H / 64], const float (&bias)[H / 64], int r0,
                                             int c0, int g, int lr)
{
#pragma unroll
    for (int t = 0; t < H / 64; ++t) {
        const int j = c0 + 16 * t + lr;
        const float bj = bias[t];
        uint16_t q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v = acc[t][r] + bj;
            v = v > 0.f ? v : 0.f;
            q[r] = f32_to_bf16(v);
            hs[4 * g + r][j] = q[r];
            const int i = r0 + 4 * g + r;
            if (i < p.n) hg[(int64_t)i * H + j] = q[r];
        }
        if (hT) {
            uint16_t *t4 = hT + (int64_t)j * p.ldT + r0 + 4 * g;
            if (r0 + 4 * g + 3 < p.n) {
                *reinterpret_cast<uint2 *>(t4) = make_uint2((uint32_t)q[0] | ((uint32_t)q[1] << 16),
                                                            (uint32_t)q[2] | ((uint32_t)q[3] << 16));
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r0 + 4 * g + r < p.n) t4[r] = q[r];
            }
        }
    }
}

// The fragments of the H x H matrix w read as B(k, j) = w[j H + k] that this
// wave's columns c0 + 16 t + lr take in the k step kk = 32 k: f[t][k], 16
// bytes each from global memory.  The coupling kernels load them all at
// their start (128 VGPRs at H = 256; a block of 4 waves runs one wave per
// SIMD), so that the loads overlap the first product instead of making each
// k step of the middle one wait on L2.
template <int H>
__device__ __forceinline__ void load_square_frags(bf16x8_t (&f)[H / 64][H / 32], const uint16_t *__restrict__ w,
                                                  int c0, int g, int lr)
{
#pragma unroll
    for (int k = 0; k < H / 32; ++k)
#pragma unroll
        for (int t = 0; t < H / 64; ++t) f[t][k] = ld_bf16x8(w + (int64_t)(c0 + 16 * t + lr) * H + 32 * k + 8 * g);
}

// acc[t] += rows of xs (LDS, [16][H + 8]) times w, from its fragments f
// (load_square_frags), k step by k step.
template <int H>
__device__ __forceinline__ void products_from_lds(float4_t (&acc)[H / 64], const uint16_t (*xs)[H + 8],
                                                  const bf16x8_t (&f)[H / 64][H / 32], int g, int lr)
{
#pragma unroll
    for (int k = 0; k < H / 32; ++k) {
        const bf16x8_t av = *reinterpret_cast<const bf16x8_t *>(&xs[lr][32 * k + 8 * g]);
#pragma unroll
        for (int t = 0; t < H / 64; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, f[t][k], acc[t], 0, 0, 0);
    }
}

// A chain of couplings applied to the same rows in the order of c.layer[]:
// coupling li + 1 takes coupling li's output rows.  A row's chain does not
// involve the other rows, so one block carries its 16 rows through every
// coupling of the chain: the output element of thread (row, dimension) stays
// in its register as that thread's input of the next coupling, the next
// coupling's masked BF16 input in LDS, and each row's sum of log-scales in a
// register of one thread.  Every coupling still writes its outputs to global
// memory (the backward pass and the weight gradients read them).  The
// couplings share n, dim and sum_s; the first coupling's masked BF16 input is
// formed from its input rows (layer[0].xm is not read).
constexpr int kMaxChain = 16;

// What a chain launch does around its couplings (the flow's ends, so that a
// pass needs no other launch).
struct ChainEnds {
    int init_sum;             // the rows' sums of log-scales start from zero (else from sum_s)
    int affine_in;            // the first coupling's input is (a - mu) / sigma of the rows a = layer[0].a,
                              // and the sums start from sum log sigma
    NextMask in_mask;         // with affine_in: where the first coupling's masked input is kept (xm may be null)
    double *affine_out;       // x = mu + sigma y of the last coupling's output rows goes here (null: none),
                              // and the sums gain sum log sigma
    const double *mu, *log_sigma;
    int density;              // after the couplings, the base density of z: the last coupling's output rows,
    const double *z_in;       // or these rows (the pass's input in the forward direction) when given
    double *logq, *loss, *g;  // -|z|^2/2 - dim/2 log 2 pi - sum_s, |z|^2/2 + sum_s, z / n (each may be null)
};

struct LayerChain {
    LayerArgs layer[kMaxChain];
    int count;
    ChainEnds e;
};
static_assert(sizeof(LayerChain) <= 4096, "a chain is passed by value as the kernel's arguments (4 KiB at most)");

template <int H>
__global__ __launch_bounds__(256) void layer_kernel(LayerChain c)
{
    __shared__ __align__(16) uint16_t h1s[kLayerRows][H + 8];
    __shared__ __align__(16) uint16_t h2s[kLayerRows][H + 8];
    __shared__ __align__(16) uint16_t xin[kLayerRows][kInPad];
    __shared__ float outs[kLayerRows][kOutPad];
    __shared__ double sdet[kLayerRows][16];
    constexpr int NT = H / 64;            // 16-column tiles per wave
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * kLayerRows;
    const int lr = lane & 15, g = lane >> 4;
    const int c0 = wave * (H / 4);
    const int crr = tid >> 4, ci = tid & 15;   // the coupling's (row, dimension)
    const bf16x8_t zero8 = {};
    const int n = c.layer[0].n, dim = c.layer[0].dim;
    const bool row_ok = r0 + lr < n;
    const ChainEnds &e = c.e;
    // the rows' inputs of the first coupling, loaded first (rows clamped to
    // valid ones), and its masked BF16 input rows formed from them
    const int64_t oc = (int64_t)min(r0 + crr, n - 1) * dim + min(ci, dim - 1);
    double yv = c.layer[0].a[oc];
    double srow;                                     // used by threads 0-15
    if (e.affine_in) {
        const int k = min(ci, dim - 1);
        yv = (yv - e.mu[k]) * exp(-e.log_sigma[k]);
        double acc = 0.0;
        for (int j = 0; j < dim; ++j) acc += e.log_sigma[j];
        srow = 0.0 + acc;
    } else {
        srow = e.init_sum ? 0.0 : c.layer[0].sum_s[min(r0 + (tid & 15), n - 1)];
    }
    {
        const uint16_t x0 = (r0 + crr < n && ci < dim && ((c.layer[0].cond >> ci) & 1u)) ? f32_to_bf16((float)yv)
                                                                                         : (uint16_t)0;
        xin[crr][ci] = x0;
        if (e.affine_in && e.in_mask.xm && r0 + crr < n) {
            e.in_mask.xm[(int64_t)(r0 + crr) * kInPad + ci] = x0;
            if (e.in_mask.xmT) e.in_mask.xmT[ci * e.in_mask.ldT + r0 + crr] = x0;
        }
    }
    __syncthreads();
    for (int li = 0; li < c.count; ++li) {
        const LayerArgs &p = c.layer[li];
        // Every operand of the coupling is loaded now, unconditionally
        // (clamped to valid rows), in the order of use: the loads complete in
        // order, so that a use waits only for its own load and those before
        // it, and a load under a branch would make the wave wait for all of
        // them.  The biases, W1's fragments, then W2's, then W3's.
        const int n_out = 2 * dim;
        const int ocol = 16 * (wave & 1) + lr;
        float b1v[NT], b2v[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            b1v[t] = p.b1[c0 + 16 * t + lr];
            b2v[t] = p.b2[c0 + 16 * t + lr];
        }
        const float b3v = p.b3[min(ocol, n_out - 1)];
        // lane groups 2 and 3 hold the zero padding of K from kInPad to 32 (in
        // the input rows, so W1's fragments there may repeat real ones)
        bf16x8_t w1f[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
            w1f[t] = ld_bf16x8(p.w1p + (int64_t)(c0 + 16 * t + lr) * kInPad + 8 * (g & 1));
        bf16x8_t w2f[NT][H / 32];
        load_square_frags<H>(w2f, p.w2, c0, g, lr);
        // output columns past 2 dim repeat the last one (never read)
        bf16x8_t w3f[H / 32];
#pragma unroll
        for (int k = 0; k < H / 32; ++k)
            w3f[k] = ld_bf16x8(p.w3 + (int64_t)min(ocol, n_out - 1) * H + 32 * k + 8 * g);
        __builtin_amdgcn_sched_barrier(0);   // all loads issued before the first product waits on its own
        // h1 = relu(xm W1^T + b1), K = kInPad padded to 32 by zeros
        const bf16x8_t xs = *reinterpret_cast<const bf16x8_t *>(&xin[lr][8 * (g & 1)]);
        const bf16x8_t xa = (g < 2 && row_ok) ? xs : zero8;
        float4_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, w1f[t], float4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        store_hidden<H>(p, h1s, p.h1, p.h1T, acc, b1v, r0, c0, g, lr);
        __syncthreads();
        // h2 = relu(h1 W2^T + b2), K = H
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = float4_t{0.f, 0.f, 0.f, 0.f};
        products_from_lds<H>(acc, h1s, w2f, g, lr);
        store_hidden<H>(p, h2s, p.h2, p.h2T, acc, b2v, r0, c0, g, lr);
        __syncthreads();
        // out = h2 W3^T + b3: 2 dim <= 32 columns, one 16-column tile for each of waves 0 and 1
        if (wave < 2) {
            const int col = ocol;
            float4_t o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < H / 32; ++k) {
                const bf16x8_t av = *reinterpret_cast<const bf16x8_t *>(&h2s[lr][32 * k + 8 * g]);
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w3f[k], o, 0, 0, 0);
            }
            const float bc = col < n_out ? b3v : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) outs[4 * g + r][col] = o[r] + bc;
        }
        __syncthreads();
        // the coupling: thread (row, i) = (tid / 16, tid % 16) takes dimension
        // i of a row, then each row's log-determinant terms are added in
        // dimension order by one thread (the order of the row-at-a-time kernel)
        {
            const int rr = crr, i = ci;
            const int b = r0 + rr;
            double sv = 0.0;
            uint16_t xv = 0;
            if (b < n && i < dim) {
                const double ai = yv;
                double yi = ai;
                if (!((p.cond >> i) & 1u)) {
                    const double r = (double)outs[rr][i];
                    const double t = (double)outs[rr][dim + i];
                    sv = 3.0 * tanh(r / 3.0);
                    yi = p.dir > 0 ? ai * exp(sv) + t : (ai - t) * exp(-sv);
                }
                p.y[(int64_t)b * dim + i] = yi;
                if (p.s_out) p.s_out[(int64_t)b * dim + i] = sv;
                xv = ((p.nm.cond >> i) & 1u) ? f32_to_bf16((float)yi) : (uint16_t)0;
                if (p.nm.xm) {
                    p.nm.xm[(int64_t)b * kInPad + i] = xv;
                    if (p.nm.xmT) p.nm.xmT[i * p.nm.ldT + b] = xv;
                }
                yv = yi;
            } else if (b < n && p.nm.xm) {
                p.nm.xm[(int64_t)b * kInPad + i] = 0;         // dimensions past dim of the next input
                if (p.nm.xmT) p.nm.xmT[i * p.nm.ldT + b] = 0;
            }
            sdet[rr][i] = sv;
            xin[rr][i] = xv;                                  // the next coupling's input row
        }
        __syncthreads();
        if (tid < kLayerRows) {
            double acc_s = 0.0;
            for (int i = 0; i < dim; ++i)
                if (!((p.cond >> i) & 1u)) acc_s += sdet[tid][i];
            srow += acc_s;
        }
    }
    if (e.affine_out) {
        if (r0 + crr < n && ci < dim)
            e.affine_out[(int64_t)(r0 + crr) * dim + ci] = e.mu[ci] + exp(e.log_sigma[ci]) * yv;
        double acc = 0.0;
        for (int j = 0; j < dim; ++j) acc += e.log_sigma[j];
        srow = srow + acc;
    }
    if (tid < kLayerRows && r0 + tid < n) c.layer[0].sum_s[r0 + tid] = srow;
    if (e.density) {
        // z_i to LDS, then each row's |z|^2 in dimension order by one thread
        const double zi = e.z_in ? e.z_in[oc] : yv;
        if (e.g && r0 + crr < n && ci < dim) e.g[(int64_t)(r0 + crr) * dim + ci] = zi / (double)n;
        __syncthreads();                             // the last coupling's sums have read sdet
        sdet[crr][ci] = zi;
        __syncthreads();
        if (tid < kLayerRows && r0 + tid < n) {
            double zz = 0.0;
            for (int j = 0; j < dim; ++j) {
                const double v = sdet[tid][j];
                zz += v * v;
            }
            const double l = 0.5 * zz + srow;
            if (e.logq) e.logq[r0 + tid] = -l - 0.5 * dim * 1.8378770664093453;   // log(2 pi)
            if (e.loss) e.loss[r0 + tid] = l;
        }
    }
}

// Affine normalisation around the coupling stack: forward x = mu + sigma u,
// inverse u = (x - mu) / sigma; sum_s[b] += sum log sigma in both directions.
// init_sum: sum_s[b] starts from zero here.  Thread (row, i) = (tid / 16,
// tid % 16) of a block of 16 rows takes element i of a row, and column i of
// the next coupling's masked BF16 input (zeros past dim).
__global__ __launch_bounds__(256) void affine_kernel(int n, int dim, int dir, const double *__restrict__ mu,
                                                     const double *__restrict__ log_sigma,
                                                     const double *__restrict__ a, double *__restrict__ y,
                                                     double *__restrict__ sum_s, int init_sum, NextMask nm)
{
    const int b = blockIdx.x * 16 + (int)(threadIdx.x >> 4), i = threadIdx.x & 15;
    if (b >= n) return;
    double yi = 0.0;
    if (i < dim) {
        const double v = a[(int64_t)b * dim + i];
        yi = dir > 0 ? mu[i] + exp(log_sigma[i]) * v : (v - mu[i]) * exp(-log_sigma[i]);
        y[(int64_t)b * dim + i] = yi;
    }
    if (i == 0) {
        double acc = 0.0;
        for (int k = 0; k < dim; ++k) acc += log_sigma[k];
        sum_s[b] = (init_sum ? 0.0 : sum_s[b]) + acc;
    }
    if (nm.xm) {
        const bool on = i < dim && ((nm.cond >> i) & 1u);
        const uint16_t v = on ? f32_to_bf16((float)yi) : (uint16_t)0;
        nm.xm[(int64_t)b * kInPad + i] = v;
        if (nm.xmT) nm.xmT[i * nm.ldT + b] = v;
    }
}

// log q = -|z|^2/2 - dim/2 log(2 pi) - sum_s; the per-row training loss is
// |z|^2/2 + sum_s (the negative log density up to the constant), and with g
// given the start of its gradient, d loss / d z = z / n for the mean loss.
__global__ __launch_bounds__(256) void base_density_kernel(int n, int dim, const double *__restrict__ z,
                                                           const double *__restrict__ sum_s,
                                                           double *__restrict__ logq, double *__restrict__ loss,
                                                           double *__restrict__ g)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double zz = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double v = z[(int64_t)b * dim + i];
        zz += v * v;
        if (g) g[(int64_t)b * dim + i] = v / (double)n;
    }
    const double l = 0.5 * zz + sum_s[b];
    if (logq) logq[b] = -l - 0.5 * dim * 1.8378770664093453;   // log(2 pi)
    if (loss) loss[b] = l;
}

// ---------------------------------------------------------------- one coupling's backward in one kernel
// The row-local part of coupling l's backward pass on kLayerRows rows per
// block (hidden width H = 128 or 256), in the order of the separate kernels
// it replaces and with the same products (v_mfma_f32_16x16x32_bf16 over k in
// order):
//   dout = d loss / d(r, t) from the inverse coupling and the direct part of
//   d loss / d y (into gy); dh2 = dout W3 masked by h2 > 0; dh1 = dh2 W2
//   masked by h1 > 0; dxm = dh1 W1 added into gy on the conditioning
//   dimensions.
// The weight gradients need sums over all rows and stay split-K GEMMs; this
// kernel writes their transposed BF16 operands (doutT, dpreT, dpre2T) and the
// bias gradients' partial sums over its rows (FP64, fixed order) into
// bpart: [block][H] for b1 and b2 (at bp1, bp2), [block][2 dim] for b3.
struct BackArgs {
    int n, dim;
    unsigned cond;
    const double *g, *x, *s;              // d loss / d x, x = the coupling's output (inverse direction), s
    double *gy;                           // d loss / d y
    const uint16_t *h1T, *h2T;            // [H][ldT] activations of the forward pass, transposed
    const uint16_t *w1t, *w2t, *w3t;      // W1^T [D][H], W2^T [H][H], W3^T [H][kOutPad]
    uint16_t *doutT, *dpreT, *dpre2T;     // transposed operands of the weight gradients (row length ldT)
    int64_t ldT;
    double *bp1, *bp2, *bp3;              // bias partials [block][H], [block][H], [block][2 dim]
};

template <int H>
__device__ __forceinline__ void masked_hidden(const BackArgs &p, uint16_t (*ds)[H + 8], uint16_t *dT, double *bp,
                                              const float4_t (&acc)[H / 64], const uint2 (&h4)[H / 64], int r0,
                                              int c0, int g, int lr)
{
#pragma unroll
    for (int t = 0; t < H / 64; ++t) {
        const int j = c0 + 16 * t + lr;
        uint16_t q[4];
        double cs = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = r0 + 4 * g + r;
            float v = acc[t][r];
            if (i < p.n) {
                const uint32_t w = r < 2 ? h4[t].x : h4[t].y;
                const uint16_t hv = (uint16_t)(r % 2 == 0 ? w & 0xffffu : w >> 16);
                v = ((hv & 0x7fffu) != 0 && !(hv & 0x8000u)) ? v : 0.f;
            } else {
                v = 0.f;
            }
            q[r] = f32_to_bf16(v);
            ds[4 * g + r][j] = q[r];
            cs += (double)v;
        }
        uint16_t *t4 = dT + (int64_t)j * p.ldT + r0 + 4 * g;
        if (r0 + 4 * g + 3 < p.n) {
            *reinterpret_cast<uint2 *>(t4) = make_uint2((uint32_t)q[0] | ((uint32_t)q[1] << 16),
                                                        (uint32_t)q[2] | ((uint32_t)q[3] << 16));
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r0 + 4 * g + r < p.n) t4[r] = q[r];
        }
        // the column's sum over the block's 16 rows: each lane's 4, then the 4 lane groups
        cs += __shfl_xor(cs, 16);
        cs += __shfl_xor(cs, 32);
        if (g == 0) bp[(int64_t)blockIdx.x * H + j] = cs;
    }
}

// The backward couplings of a chain, in the order of c.layer[], carried
// through by one block per 16 rows as in layer_kernel: coupling li + 1 takes
// d loss / d y of coupling li as its d loss / d x, kept in LDS between them
// (the direct part from the head, then the MLP's part on the conditioning
// dimensions added to it).  Every coupling still writes its transposed
// operands of the weight gradients and its bias partials to global memory;
// the last one also writes d loss / d y.  The couplings share n and dim.
struct BackChain {
    BackArgs layer[kMaxChain];
    int count;
};
static_assert(sizeof(BackChain) <= 4096, "a chain is passed by value as the kernel's arguments (4 KiB at most)");

template <int H>
__global__ __launch_bounds__(256) void layer_back_kernel(BackChain c)
{
    __shared__ float dos[kLayerRows][kOutPad];
    __shared__ __align__(16) uint16_t d2s[kLayerRows][H + 8];
    __shared__ __align__(16) uint16_t d1s[kLayerRows][H + 8];
    __shared__ double gys[kLayerRows][16];
    constexpr int NT = H / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * kLayerRows;
    const int lr = lane & 15, g = lane >> 4;
    const int c0 = wave * (H / 4);
    const int n = c.layer[0].n, D = c.layer[0].dim;
    const int rr = tid >> 4, i = tid & 15;   // the head's (row, dimension)
    const int64_t oc = (int64_t)min(r0 + rr, n - 1) * D + min(i, D - 1);
    double gv = c.layer[0].g[oc];            // d loss / d x of the first coupling, loaded first
    for (int li = 0; li < c.count; ++li) {
        const BackArgs &p = c.layer[li];
        // Every operand is loaded now, unconditionally (clamped to valid
        // rows), in the order of use (the loads complete in order; a load
        // under a branch would make the wave wait for all of them): this
        // thread's element of the head, the activations' signs for the two
        // ReLU masks (4 rows of a column in 8 bytes of the transposed copies),
        // then the weight fragments of the three products (W1's rows past dim
        // repeat the last, never read).
        const double xv = p.x[oc], sv = p.s[oc];
        uint2 m2[NT], m1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t at = (int64_t)(c0 + 16 * t + lr) * p.ldT + r0 + 4 * g;
            m2[t] = *reinterpret_cast<const uint2 *>(p.h2T + at);
            m1[t] = *reinterpret_cast<const uint2 *>(p.h1T + at);
        }
        bf16x8_t w3f[NT], w2f[NT][H / 32], w1f[H / 32];
#pragma unroll
        for (int t = 0; t < NT; ++t) w3f[t] = ld_bf16x8(p.w3t + (int64_t)(c0 + 16 * t + lr) * kOutPad + 8 * g);
        load_square_frags<H>(w2f, p.w2t, c0, g, lr);
#pragma unroll
        for (int k = 0; k < H / 32; ++k) w1f[k] = ld_bf16x8(p.w1t + (int64_t)min(lr, D - 1) * H + 32 * k + 8 * g);
        // the inverse coupling's backward: thread (row, i) = (tid / 16, tid % 16)
        // takes dimension i of a row (dout columns i and D + i)
        {
            const int b = r0 + rr;
            dos[rr][i] = 0.f;
            dos[rr][16 + i] = 0.f;
            if (li > 0) gv = gys[rr][i];     // the previous coupling's d loss / d y
            __syncthreads();
            double gd = 0.0;                 // the direct part of d loss / d y
            if (b < n && i < D) {
                if ((p.cond >> i) & 1u) {
                    gd = gv;
                } else {
                    const double inv_n = 1.0 / (double)n;
                    const double si = sv, e = exp(-si);
                    const double dt = -gv * e;
                    const double ds = -gv * xv + inv_n;
                    const double dr = ds * (1.0 - (si / 3.0) * (si / 3.0));
                    gd = gv * e;
                    dos[rr][i] = (float)dr;
                    dos[rr][D + i] = (float)dt;
                }
            }
            gys[rr][i] = gd;
            __syncthreads();
            if (b < n) {
                p.doutT[(int64_t)i * p.ldT + b] = f32_to_bf16(dos[rr][i]);
                p.doutT[(int64_t)(16 + i) * p.ldT + b] = f32_to_bf16(dos[rr][16 + i]);
            }
        }
        __syncthreads();
        if (tid < 2 * D) {
            double t = 0.0;
            for (int r = 0; r < kLayerRows; ++r) t += (double)dos[r][tid];
            p.bp3[(int64_t)blockIdx.x * 2 * D + tid] = t;
        }
        // dh2 = dout W3 (K = 2 dim <= 32 in one step), masked by h2 > 0
        float4_t acc[NT];
        {
            bf16x8_t av;
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = (__bf16)dos[lr][8 * g + e];
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w3f[t], float4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
        masked_hidden<H>(p, d2s, p.dpreT, p.bp2, acc, m2, r0, c0, g, lr);
        __syncthreads();
        // dh1 = dpre2 W2 (B(k, j) = W2[k][j] = W2^T[j][k]), masked by h1 > 0
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = float4_t{0.f, 0.f, 0.f, 0.f};
        products_from_lds<H>(acc, d2s, w2f, g, lr);
        masked_hidden<H>(p, d1s, p.dpre2T, p.bp1, acc, m1, r0, c0, g, lr);
        __syncthreads();
        // dxm = dpre1 W1 (B(k, d) = W1[k][d] = W1^T[d][k]), added into d loss / d y on the conditioning dims
        if (wave == 0) {
            const int col = lr;
            float4_t o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < H / 32; ++k) {
                const bf16x8_t av = *reinterpret_cast<const bf16x8_t *>(&d1s[lr][32 * k + 8 * g]);
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w1f[k], o, 0, 0, 0);
            }
            if (col < D && ((p.cond >> col) & 1u)) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r0 + 4 * g + r < n) gys[4 * g + r][col] += (double)o[r];
            }
        }
        __syncthreads();
    }
    const BackArgs &pl = c.layer[c.count - 1];
    if (r0 + rr < n && i < D) pl.gy[(int64_t)(r0 + rr) * D + i] = gys[rr][i];
}

// ---------------------------------------------------------------- training backward

// Backward of one inverse coupling x = (y - t) e^{-s} (T dims), x_C = y_C, with
// the loss term sum_T s / n.  g = d loss / d x.  Writes d loss / d(r, t) as
// BF16 and FP32 rows of kOutPad and as BF16 columns (doutT[c ldT + b]), and
// the direct part of d loss / d y (the MLP's contribution to the conditioning
// dimensions is added later).
__global__ __launch_bounds__(256) void coupling_inv_backward_kernel(int n, int dim, unsigned cond,
                                                                    const double *__restrict__ g,
                                                                    const double *__restrict__ x,
                                                                    const double *__restrict__ s,
                                                                    uint16_t *__restrict__ dout_b,
                                                                    float *__restrict__ dout_f,
                                                                    double *__restrict__ gy,
                                                                    uint16_t *__restrict__ doutT, int64_t ldT)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double inv_n = 1.0 / (double)n;
    for (int i = 0; i < kOutPad; ++i) {
        dout_b[(int64_t)b * kOutPad + i] = 0;
        dout_f[(int64_t)b * kOutPad + i] = 0.f;
        doutT[i * ldT + b] = 0;
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
            doutT[i * ldT + b] = f32_to_bf16((float)dr);
            doutT[(dim + i) * ldT + b] = f32_to_bf16((float)dt);
        }
    }
}

// Column sums of m [rows][cols] (leading dimension ld, cols <= 64) over each
// block of 64 rows, in FP64 and a fixed order: the block's 4 waves take rows
// 4 q + w of it, then their sums are added in wave order; part [block][cols].
// The same 64-row blocks as the GEMM's column sums.
__global__ __launch_bounds__(256) void column_part_kernel(int rows, int cols, int ld, const float *__restrict__ m,
                                                          double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = (int)blockIdx.x * 64, r1 = min(rows, r0 + 64);
    double acc = 0.0;
    if (c < cols) {
#pragma unroll 4
        for (int b = r0 + w; b < r1; b += 4) acc += (double)m[(int64_t)b * ld + c];
    }
    red[w][c] = acc;
    __syncthreads();
    if (w == 0 && c < cols) part[(int64_t)blockIdx.x * cols + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// Gradient of every parameter from the partial sums the backward pass left,
// one thread per parameter, in a fixed order.  Layer l's parameters are
// w1 [H][D], b1 [H], w2 [H][H], b2 [H], w3 [2D][H], b3 [2D]; its weight
// partials (FP32) are split slices of each matrix at wpart + l * w_layer
// (w1, w2, w3 regions of kMaxSplit slices each), summed in slice order in
// FP32; its bias partials (FP64) are 64-row block sums of the gradients of
// the three layers' outputs (b1, b2: rb64 blocks of H each; b3: rb64 blocks
// of 2D), summed in block order.
struct GradParts {
    int D, H, split, rb, rb_cap;        // row blocks of the bias partials (used, allocated)
    int64_t per_layer, n_params, w_layer, b_layer;
    const float *wpart;
    const double *bpart;
};

// Parameter p's gradient from its partial sums, when a thread finishes it:
// the weights' split-K slices in slice order, and the biases' row-block
// partials in block order when there are at most 64 of them (more: a wave
// per bias element, bias_gradient).  Returns false for the biases left to the
// waves.
__device__ __forceinline__ bool param_gradient(const GradParts &gp, int64_t p, float &grad)
{
    const int64_t D = gp.D, H = gp.H;
    const int64_t l = p / gp.per_layer;
    int64_t q = p - l * gp.per_layer;
    const float *w = gp.wpart + l * gp.w_layer;
    const double *bp = gp.bpart + l * gp.b_layer;
    const int64_t sz1 = H * D, sz2 = H * H, sz3 = 2 * D * H;
    const float *wr = nullptr;
    int64_t wsz = 0;
    const double *br = nullptr;
    int64_t bcols = 0;
    if (q < sz1) {
        wr = w, wsz = sz1;
    } else if ((q -= sz1) < H) {
        br = bp, bcols = H;
    } else if ((q -= H) < sz2) {
        wr = w + kMaxSplit * sz1, wsz = sz2;
    } else if ((q -= sz2) < H) {
        br = bp + gp.rb_cap * H, bcols = H;
    } else if ((q -= H) < sz3) {
        wr = w + kMaxSplit * (sz1 + sz2), wsz = sz3;
    } else {
        q -= sz3;
        br = bp + 2 * gp.rb_cap * H, bcols = 2 * D;
    }
    if (wr) {
        float v = 0.f;
        for (int z = 0; z < gp.split; ++z) v += wr[z * wsz + q];
        grad = v;
        return true;
    }
    if (gp.rb > 64) return false;
    double t = 0.0;
    for (int64_t y = 0; y < gp.rb; ++y) t += br[y * bcols + q];
    grad = (float)t;
    return true;
}

// Bias element e (layer e / (2 H + 2 dim), then b1, b2, b3) summed over its
// row-block partials by the 64 lanes of a wave: lane k the blocks k, k + 64,
// ... in order, then the 64 lane sums by a fixed butterfly (every lane gets
// the total).  p: the element's parameter index.
__device__ __forceinline__ float bias_gradient(const GradParts &gp, int64_t e, int lane, int64_t &p)
{
    const int64_t H = gp.H, D = gp.D, per = 2 * H + 2 * D;
    const int64_t l = e / per, r = e % per;
    const double *bp = gp.bpart + l * gp.b_layer;
    const double *br;
    int64_t bcols, q;
    const int64_t base = l * gp.per_layer;
    if (r < H) {
        br = bp, bcols = H, q = r, p = base + H * D + r;
    } else if (r < 2 * H) {
        br = bp + gp.rb_cap * H, bcols = H, q = r - H, p = base + H * D + H + H * H + (r - H);
    } else {
        br = bp + 2 * gp.rb_cap * H, bcols = 2 * D, q = r - 2 * H,
        p = base + H * D + 2 * H + H * H + 2 * D * H + (r - 2 * H);
    }
    double t = 0.0;
    for (int64_t y = lane; y < gp.rb; y += 64) t += br[y * bcols + q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    return (float)t;
}

__global__ __launch_bounds__(256) void grad_finish_kernel(GradParts gp, float *__restrict__ grads)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= gp.n_params) return;
    float g;
    if (param_gradient(gp, p, g)) grads[p] = g;
}

// The biases when their partials come in more than 64 row blocks: one wave
// per bias element.
__global__ __launch_bounds__(64) void bias_finish_kernel(GradParts gp, float *__restrict__ grads)
{
    int64_t p;
    const float g = bias_gradient(gp, blockIdx.x, threadIdx.x, p);
    if (threadIdx.x == 0) grads[p] = g;
}

// out[0] = the mean of loss[0, n) (one block of 256 threads: thread t sums
// the rows t, t + 256, ... in order, then a fixed tree over the threads).
__device__ __forceinline__ void mean_block(int n, const double *__restrict__ loss, double *__restrict__ out)
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

__global__ __launch_bounds__(256) void mean_kernel(int n, const double *__restrict__ loss, double *__restrict__ out)
{
    mean_block(n, loss, out);
}

// BF16 copies of the weight matrices (FP32 master -> BF16): parameter i of
// layer i / per_layer goes to dst[layer * dst_stride + i % per_layer], and
// the weights also transposed into dstT (layer stride t_stride): W1^T [D][H],
// W2^T [H][H], W3^T [H][kOutPad] (rows padded), the backward pass's operands,
// then W1 with its rows padded to kInPad, [H][kInPad], the first product's
// operand in 16-byte vectors.
struct Bf16Copies {
    int64_t per_layer, dst_stride, t_stride;
    int D, H;
    uint16_t *dst, *dstT;
};

__device__ __forceinline__ void write_bf16(const Bf16Copies &c, int64_t i, float value)
{
    const int64_t l = i / c.per_layer;
    int64_t q = i - l * c.per_layer;
    const int64_t D = c.D, H = c.H;
    const uint16_t v = f32_to_bf16(value);
    c.dst[l * c.dst_stride + q] = v;
    uint16_t *t = c.dstT + l * c.t_stride;
    const int64_t s1 = H * D, s2 = H * H, s3 = 2 * D * H;
    if (q < s1) {                                   // W1 [H][D] -> W1^T [D][H], and padded rows
        t[(q % D) * H + q / D] = v;
        t[s1 + s2 + H * kOutPad + (q / D) * kInPad + q % D] = v;
        return;
    }
    q -= s1 + H;
    if (q < 0) return;                              // b1
    if (q < s2) {                                   // W2 [H][H] -> W2^T
        t[s1 + (q % H) * H + q / H] = v;
        return;
    }
    q -= s2 + H;
    if (q >= 0 && q < s3) t[s1 + s2 + (q % H) * kOutPad + q / H] = v;   // W3 [2D][H] -> W3^T [H][kOutPad]
}

__global__ __launch_bounds__(256) void to_bf16_kernel(int64_t count, Bf16Copies c, const float *__restrict__ src)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) write_bf16(c, i, src[i]);
}

// Adam (Kingma & Ba 2015) on FP32 master parameters: the step of parameter
// i with gradient gi; returns the new value.
struct AdamStep {
    float *p, *m, *v;
    float lr, beta1, beta2, eps, bc1, bc2;
};

__device__ __forceinline__ float adam_update(const AdamStep &a, int64_t i, float gi)
{
    const float mi = a.beta1 * a.m[i] + (1.f - a.beta1) * gi;
    const float vi = a.beta2 * a.v[i] + (1.f - a.beta2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float pi = a.p[i] - a.lr * (mi / a.bc1) / (sqrtf(vi / a.bc2) + a.eps);
    a.p[i] = pi;
    return pi;
}

// Bias tiles of the training step's last launch: 8 consecutive elements of
// one bias vector (b1, b2 or b3) of one layer.  Their row-block partials are
// staged through LDS 128 row blocks at a time, each row block's 8 values one
// contiguous 64-byte load, and each wave then sums two of the columns in the
// order of bias_gradient (lane k the blocks k, k + 64, ... in order, then the
// same butterfly).
constexpr int kBiasCols = 8, kBiasRows = 128;

__device__ __forceinline__ int64_t bias_tiles_per_layer(const GradParts &gp)
{
    return 2 * ((gp.H + kBiasCols - 1) / kBiasCols) + (2 * gp.D + kBiasCols - 1) / kBiasCols;
}

__device__ __forceinline__ void bias_tile(const GradParts &gp, int64_t tile, float *__restrict__ grads,
                                          const AdamStep &a, const Bf16Copies &c)
{
    __shared__ double bt[kBiasRows][kBiasCols + 1];
    const int64_t H = gp.H, D = gp.D, th = (H + kBiasCols - 1) / kBiasCols;
    const int64_t l = tile / bias_tiles_per_layer(gp), r = tile % bias_tiles_per_layer(gp);
    const double *bp = gp.bpart + l * gp.b_layer;
    const int64_t base = l * gp.per_layer;
    const double *br;
    int64_t bcols, len, q0, p0;
    if (r < th) {
        br = bp, bcols = H, len = H, q0 = r * kBiasCols, p0 = base + H * D;
    } else if (r < 2 * th) {
        br = bp + gp.rb_cap * H, bcols = H, len = H, q0 = (r - th) * kBiasCols, p0 = base + H * D + H + H * H;
    } else {
        br = bp + 2 * gp.rb_cap * H, bcols = 2 * D, len = 2 * D, q0 = (r - 2 * th) * kBiasCols,
        p0 = base + H * D + 2 * H + H * H + 2 * D * H;
    }
    const int ncols = (int)min((int64_t)kBiasCols, len - q0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double t0 = 0.0, t1 = 0.0;                       // this lane's sums of columns wave and wave + 4
    for (int64_t y0 = 0; y0 < gp.rb; y0 += kBiasRows) {
        const int rows = (int)min((int64_t)kBiasRows, gp.rb - y0);
        __syncthreads();                             // the previous rows are summed
        for (int i = threadIdx.x; i < rows * kBiasCols; i += blockDim.x) {
            const int y = i / kBiasCols, cc = i % kBiasCols;
            if (cc < ncols) bt[y][cc] = br[(y0 + y) * bcols + q0 + cc];
        }
        __syncthreads();
        // lane k takes the rows y0 + y with y = k (mod 64), in order
        for (int y = (int)((lane - y0 % 64 + 64) % 64); y < rows; y += 64) {
            if (wave < ncols) t0 += bt[y][wave];
            if (wave + 4 < ncols) t1 += bt[y][wave + 4];
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        t0 += __shfl_xor(t0, off);
        t1 += __shfl_xor(t1, off);
    }
    if (lane != 0) return;
    if (wave < ncols) {
        const int64_t p = p0 + q0 + wave;
        grads[p] = (float)t0;
        write_bf16(c, p, adam_update(a, p, (float)t0));
    }
    if (wave + 4 < ncols) {
        const int64_t p = p0 + q0 + wave + 4;
        grads[p] = (float)t1;
        write_bf16(c, p, adam_update(a, p, (float)t1));
    }
}

// The end of a training step in one launch: every parameter's gradient from
// its partial sums (the orders of grad_finish_kernel and bias_finish_kernel),
// its Adam update and its BF16 copies.  Blocks below weight_blocks take one
// parameter per thread; the biases that param_gradient leaves to waves go to
// the bias_tiles blocks after them (bias_tile); with loss_out given, the last
// block writes the mean of the n_rows per-row losses there (mean_block).
__global__ __launch_bounds__(256) void finish_update_kernel(GradParts gp, float *__restrict__ grads, AdamStep a,
                                                            Bf16Copies c, int weight_blocks, int64_t bias_tiles,
                                                            int n_rows, const double *__restrict__ loss,
                                                            double *__restrict__ loss_out)
{
    if (loss_out && blockIdx.x == gridDim.x - 1) {
        mean_block(n_rows, loss, loss_out);
        return;
    }
    if ((int)blockIdx.x < weight_blocks) {
        const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        float g;
        if (p >= gp.n_params || !param_gradient(gp, p, g)) return;
        grads[p] = g;
        write_bf16(c, p, adam_update(a, p, g));
        return;
    }
    const int64_t tile = (int64_t)blockIdx.x - weight_blocks;
    if (tile < bias_tiles) bias_tile(gp, tile, grads, a, c);
}

__global__ __launch_bounds__(256) void zero_kernel(int64_t n, double *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// mean of loss[0..n) into out[0] (one block, fixed order).
}  // namespace flow
}  // namespace gw

// ================================================================ host side
struct gw_flow {
    int device = 0;
    int dim = 0, layers = 0, hidden = 0;
    std::vector<unsigned> cond;           // conditioning mask per layer
    int64_t per_layer = 0, n_params = 0;
    int64_t wb_stride = 0;                // layer stride of the BF16 copy (per_layer rounded up to 8)
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    uint16_t *wb = nullptr;               // BF16 copy of params
    uint16_t *wbT = nullptr;              // BF16 transposed weights per layer (to_bf16_kernel)
    int64_t wbT_stride = 0;               // D H + H H + H kOutPad
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
    uint16_t *dpre2_b = nullptr;          // [cap][hidden], the other layer's BF16 pre-activation gradient
    // transposed BF16 copies for the weight gradients (row length ldT, a
    // multiple of 64 >= cap): activations [layers][hidden][ldT], inputs
    // [layers][kInPad][ldT], output gradients [layers][kOutPad][ldT], the two
    // pre-activation gradients [layers][hidden][ldT] (the GEMM path uses the
    // first layer's slices of the last three for every layer)
    int64_t ldT = 0;
    uint16_t *h1T = nullptr, *h2T = nullptr, *xmT = nullptr, *doutT = nullptr, *dpreT = nullptr, *dpre2T = nullptr;
    // partial sums of the gradients (summed by grad_finish_kernel or, in a
    // training step, finish_update_kernel): per layer,
    // split-K slices of the three weight matrices (FP32, w_layer floats) and
    // row-block sums of the three biases (FP64, b_layer doubles)
    float *wpart = nullptr;
    double *bpart = nullptr;
    int64_t w_layer = 0, b_layer = 0;
    int rb_cap = 0;                      // row blocks the bias partials are sized for (16-row blocks)
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

// Offsets of one layer's parameters: p the layer's start in the FP32
// parameters (and gradients), q its start in the BF16 copy, whose layers
// start at multiples of 8 elements (wb_stride) so that the weight matrices
// are 16-byte aligned for the GEMM's vector loads; w1 .. b3 within the layer.
struct LayerOff { int64_t p, q, w1, b1, w2, b2, w3, b3; };
LayerOff layer_off(const gw_flow *f, int l)
{
    const int64_t D = f->dim, H = f->hidden;
    LayerOff o;
    o.p = l * f->per_layer;
    o.q = l * f->wb_stride;
    o.w1 = 0;
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
                    f->out_f, f->dout_f, f->dout_b, f->dh, f->dpre_b, f->dpre2_b, f->wpart, f->bpart,
                    f->h1T, f->h2T, f->xmT, f->doutT, f->dpreT, f->dpre2T};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    f->bound = f->s_store = f->sum_s = f->loss = f->g = f->gy = f->bpart = nullptr;
    f->dpre2_b = f->h1T = f->h2T = f->xmT = f->doutT = f->dpreT = f->dpre2T = nullptr;
    f->xm_b = f->h1_b = f->h2_b = f->dout_b = f->dpre_b = nullptr;
    f->out_f = f->dout_f = f->dh = f->wpart = nullptr;
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
    const int rb_cap = (int)((c + gw::flow::kLayerRows - 1) / gw::flow::kLayerRows);
    const int64_t w_layer = (int64_t)gw::flow::kMaxSplit * (H * D + H * H + 2 * D * H);
    const int64_t b_layer = (int64_t)rb_cap * (2 * H + 2 * D);
    const int64_t ldT = (c + 63) / 64 * 64;
    if (alloc(&f->bound, (L + 2) * c * D) || alloc(&f->s_store, L * c * D) || alloc(&f->sum_s, c) ||
        alloc(&f->loss, c) || alloc(&f->g, c * D) || alloc(&f->gy, c * D) || alloc(&f->xm_b, L * c * kInPad) ||
        alloc(&f->h1_b, L * c * H) || alloc(&f->h2_b, L * c * H) || alloc(&f->out_f, c * 2 * D) ||
        alloc(&f->dout_f, c * kOutPad) || alloc(&f->dout_b, c * kOutPad) || alloc(&f->dh, c * H) ||
        alloc(&f->dpre_b, c * H) ||
        alloc(&f->dpre2_b, c * H) || alloc(&f->wpart, L * w_layer) || alloc(&f->bpart, L * b_layer) ||
        alloc(&f->h1T, L * H * ldT) || alloc(&f->h2T, L * H * ldT) || alloc(&f->xmT, L * kInPad * ldT) ||
        alloc(&f->doutT, L * kOutPad * ldT) || alloc(&f->dpreT, L * H * ldT) || alloc(&f->dpre2T, L * H * ldT)) {
        free_batch(f);
        return fail(GW_ENOMEM, "flow batch buffers");
    }
    f->cap = c;
    f->ldT = ldT;
    f->w_layer = w_layer;
    f->b_layer = b_layer;
    f->rb_cap = rb_cap;
    return GW_OK;
}

double *boundary(gw_flow *f, int i) { return f->bound + (int64_t)i * f->cap * f->dim; }

// The MLP of layer l on the masked input of rows [0, n): writes out_f (r, t)
// and keeps the BF16 activations of layer l for the backward pass (with
// keep_t also transposed, the weight gradients' operands).
hipError_t mlp_forward(gw_flow *f, int l, int n, bool keep_t, hipStream_t s)
{
    const int D = f->dim, H = f->hidden;
    const LayerOff o = layer_off(f, l);
    const uint16_t *xm = f->xm_b + (int64_t)l * f->cap * kInPad;
    uint16_t *h1 = f->h1_b + (int64_t)l * f->cap * H;
    uint16_t *h2 = f->h2_b + (int64_t)l * f->cap * H;
    const uint16_t *wq = f->wb + o.q;
    const float *pp = f->params + o.p;
    // W1 with rows padded to kInPad (in the transposed copy's block); the
    // padding of both operands is zero, so K = kInPad adds exact zeros only
    const uint16_t *w1p = f->wbT + (int64_t)l * f->wbT_stride + (int64_t)D * H + (int64_t)H * H +
                          (int64_t)H * kOutPad;
    GemmArgs g1{n, H, kInPad, xm, kInPad, 1, w1p, 1, kInPad, nullptr, 0, h1, H, pp + o.b1, 1};
    GemmArgs g2{n, H, H, h1, H, 1, wq + o.w2, 1, H, nullptr, 0, h2, H, pp + o.b2, 1};
    if (keep_t) {
        g1.CbT = f->h1T + (int64_t)l * H * f->ldT;
        g2.CbT = f->h2T + (int64_t)l * H * f->ldT;
        g1.ldcbT = g2.ldcbT = f->ldT;
    }
    hipError_t e;
    if ((e = gw::flow::gemm_bf16(g1, s)) != hipSuccess) return e;
    if ((e = gw::flow::gemm_bf16(g2, s)) != hipSuccess) return e;
    GemmArgs g3{n, 2 * D, H, h2, H, 1, wq + o.w3, 1, H, f->out_f, 2 * D, nullptr, 0, pp + o.b3, 0};
    return gw::flow::gemm_bf16(g3, s);
}

// Coupling l as one kernel (hidden width 128 or 256), or false when the
// width has no such kernel and the products run as separate GEMMs.
bool fused_width(const gw_flow *f) { return f->hidden == 128 || f->hidden == 256; }

// Where the kernel producing layer l's input writes that layer's masked
// MLP input (and, with keep_t, its transposed copy); none for l outside the stack.
gw::flow::NextMask mask_of(gw_flow *f, int l, bool keep_t)
{
    if (l < 0 || l >= f->layers) return gw::flow::NextMask{nullptr, nullptr, 0, 0u};
    return gw::flow::NextMask{f->xm_b + (int64_t)l * f->cap * kInPad,
                              keep_t ? f->xmT + (int64_t)l * kInPad * f->ldT : nullptr, f->ldT, f->cond[l]};
}

// The arguments of coupling l of the one-kernel path: input rows a, output
// rows y (and with s_out the log-scales), the next coupling's masked input nm.
gw::flow::LayerArgs layer_args(gw_flow *f, int l, int n, int dir, const double *a, double *y, double *s_out,
                               bool keep_t, gw::flow::NextMask nm)
{
    const int D = f->dim, H = f->hidden;
    const LayerOff o = layer_off(f, l);
    const uint16_t *wq = f->wb + o.q;
    const float *pp = f->params + o.p;
    gw::flow::LayerArgs la;
    la.n = n;
    la.dim = D;
    la.dir = dir;
    la.cond = f->cond[l];
    la.xm = f->xm_b + (int64_t)l * f->cap * kInPad;
    la.w1p = f->wbT + (int64_t)l * f->wbT_stride + (int64_t)D * H + (int64_t)H * H + (int64_t)H * kOutPad;
    la.w2 = wq + o.w2;
    la.w3 = wq + o.w3;
    la.b1 = pp + o.b1;
    la.b2 = pp + o.b2;
    la.b3 = pp + o.b3;
    la.h1 = f->h1_b + (int64_t)l * f->cap * H;
    la.h2 = f->h2_b + (int64_t)l * f->cap * H;
    la.h1T = keep_t ? f->h1T + (int64_t)l * H * f->ldT : nullptr;
    la.h2T = keep_t ? f->h2T + (int64_t)l * H * f->ldT : nullptr;
    la.ldT = f->ldT;
    la.a = a;
    la.y = y;
    la.sum_s = f->sum_s;
    la.s_out = s_out;
    la.nm = nm;
    return la;
}

// Couplings first, first + step, ... (count of them, step +1 or -1) applied in
// that order to rows [0, n) by one launch per kMaxChain couplings.  dir: +1
// the forward direction (z -> x), -1 the inverse.  Boundary l is coupling l's
// input in the forward direction; with keep_t (inverse, training) the
// transposed activations and inputs and the log-scales are kept.
// a_first: the first coupling's input rows (null: its boundary); ends: what
// the first launch does before the couplings (init_sum, affine_in, in_mask)
// and the last one after them (affine_out, density).
hipError_t layer_chain(gw_flow *f, int n, int dir, int first, int count, bool keep_t, hipStream_t s,
                       const double *a_first, const gw::flow::ChainEnds &ends)
{
    const int H = f->hidden, D = f->dim;
    const int step = dir > 0 ? 1 : -1;
    for (int done = 0; done < count;) {
        gw::flow::LayerChain c;
        c.count = std::min(count - done, gw::flow::kMaxChain);
        c.e = ends;
        if (done > 0) c.e.init_sum = c.e.affine_in = 0;
        if (done + c.count < count) {
            c.e.affine_out = nullptr;
            c.e.density = 0;
        }
        for (int k = 0; k < c.count; ++k) {
            const int l = first + step * (done + k);
            if (dir > 0)
                c.layer[k] = layer_args(f, l, n, 1, boundary(f, l), boundary(f, l + 1), nullptr, false,
                                        mask_of(f, l + 1, false));
            else
                c.layer[k] = layer_args(f, l, n, -1, boundary(f, l + 1), boundary(f, l),
                                        f->s_store + (int64_t)l * f->cap * D, keep_t, mask_of(f, l - 1, keep_t));
        }
        if (done == 0 && a_first) c.layer[0].a = a_first;
        const dim3 grid((unsigned)((n + gw::flow::kLayerRows - 1) / gw::flow::kLayerRows));
        if (H == 256)
            hipLaunchKernelGGL(gw::flow::layer_kernel<256>, grid, dim3(256), 0, s, c);
        else
            hipLaunchKernelGGL(gw::flow::layer_kernel<128>, grid, dim3(256), 0, s, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        done += c.count;
    }
    return hipSuccess;
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

// Where a pass leaves the base density of its z (each may be null; all
// null: none): log q = -|z|^2/2 - dim/2 log 2 pi - sum_s, the training loss
// |z|^2/2 + sum_s, and its gradient z / n.
struct DensityOut {
    double *logq = nullptr, *loss = nullptr, *g = nullptr;
    bool any() const { return logq || loss || g; }
};

// Inverse pass x -> z = boundary 0 over rows [0, n): the affine
// normalisation, then couplings L-1 .. 0; sum_s[b] = sum log sigma + the
// couplings' log-scales.  With keep_t the transposed activations and inputs
// are kept for the weight gradients; the log-scales always are.
hipError_t inverse_pass(gw_flow *f, int n, const double *x, bool keep_t, hipStream_t s, const DensityOut &den)
{
    const int D = f->dim, L = f->layers;
    if (fused_width(f)) {
        // one launch: the normalisation before the couplings, the density after them
        gw::flow::ChainEnds e{};
        e.affine_in = 1;
        e.in_mask = mask_of(f, L - 1, keep_t);
        e.mu = f->mu;
        e.log_sigma = f->log_sigma;
        e.density = den.any() ? 1 : 0;
        e.logq = den.logq;
        e.loss = den.loss;
        e.g = den.g;
        return layer_chain(f, n, -1, L - 1, L, keep_t, s, x, e);
    }
    hipLaunchKernelGGL(gw::flow::affine_kernel, dim3((n + 15) / 16), dim3(256), 0, s, n, D, -1, f->mu, f->log_sigma,
                       x, boundary(f, L), f->sum_s, 1, mask_of(f, L - 1, keep_t));
    GW_TRY(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        double *s_out = f->s_store + (int64_t)l * f->cap * D;
        GW_TRY(mlp_forward(f, l, n, keep_t, s));
        hipLaunchKernelGGL(gw::flow::coupling_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, f->cond[l], -1,
                           boundary(f, l + 1), f->out_f, boundary(f, l), f->sum_s, s_out, mask_of(f, l - 1, keep_t));
        GW_TRY(hipGetLastError());
    }
    if (den.any()) {
        hipLaunchKernelGGL(gw::flow::base_density_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, boundary(f, 0),
                           f->sum_s, den.logq, den.loss, den.g);
        GW_TRY(hipGetLastError());
    }
    return hipSuccess;
}

// Forward pass z -> x_out over rows [0, n): couplings 0 .. L-1, then the
// affine normalisation; sum_s as in the inverse; logq (may be null) the log
// density of x_out.  The one-kernel path is one launch that takes z as the
// first coupling's input directly; the GEMM path copies it to boundary 0
// first.  z must not overlap x_out.
hipError_t forward_pass(gw_flow *f, int n, const double *z, double *x_out, double *logq, hipStream_t s)
{
    const int D = f->dim, L = f->layers;
    if (fused_width(f)) {
        gw::flow::ChainEnds e{};
        e.init_sum = 1;
        e.affine_out = x_out;
        e.mu = f->mu;
        e.log_sigma = f->log_sigma;
        e.density = logq ? 1 : 0;
        e.z_in = z;
        e.logq = logq;
        return layer_chain(f, n, 1, 0, L, false, s, z, e);
    }
    GW_TRY(zero(n, f->sum_s, s));
    if (z != boundary(f, 0))
        GW_TRY(hipMemcpyAsync(boundary(f, 0), z, sizeof(double) * (size_t)n * D, hipMemcpyDeviceToDevice, s));
    const gw::flow::NextMask m0 = mask_of(f, 0, false);
    hipLaunchKernelGGL(gw::flow::mask_input_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, m0.cond, z, m0.xm,
                       nullptr, f->ldT);
    GW_TRY(hipGetLastError());
    for (int l = 0; l < L; ++l) {
        GW_TRY(mlp_forward(f, l, n, false, s));
        hipLaunchKernelGGL(gw::flow::coupling_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, f->cond[l], 1,
                           boundary(f, l), f->out_f, boundary(f, l + 1), f->sum_s, nullptr, mask_of(f, l + 1, false));
        GW_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(gw::flow::affine_kernel, dim3((n + 15) / 16), dim3(256), 0, s, n, D, 1, f->mu, f->log_sigma,
                       boundary(f, L), x_out, f->sum_s, 0, mask_of(f, -1, false));
    GW_TRY(hipGetLastError());
    if (logq) {
        hipLaunchKernelGGL(gw::flow::base_density_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D, z, f->sum_s,
                           logq, nullptr, nullptr);
        GW_TRY(hipGetLastError());
    }
    return hipSuccess;
}

// The BF16 copies of the flow's weights that the kernels read.
gw::flow::Bf16Copies bf16_copies(const gw_flow *f)
{
    return gw::flow::Bf16Copies{f->per_layer, f->wb_stride, f->wbT_stride, f->dim, f->hidden, f->wb, f->wbT};
}

// Gradient of the mean negative log density of rows x[0, n) with respect to
// every parameter (into f->grads); the mean loss goes to loss_out (device).
// With adam, the Adam step and the refresh of the BF16 copies follow in the
// launch that finishes the gradients.
hipError_t gradients(gw_flow *f, int n, const double *x, double *loss_out, hipStream_t s,
                     const gw::flow::AdamStep *adam = nullptr)
{
    const int D = f->dim, H = f->hidden, L = f->layers;
    // weight gradients sum over the n rows: split K = n into slices of >= 256 rows
    const int split = std::max(1, std::min(gw::flow::kMaxSplit, n / 256));
    DensityOut den;
    den.loss = f->loss;
    den.g = f->g;
    GW_TRY(inverse_pass(f, n, x, true, s, den));
    if (loss_out && !adam) {     // a training step takes the mean in its last launch
        hipLaunchKernelGGL(gw::flow::mean_kernel, dim3(1), dim3(256), 0, s, n, f->loss, loss_out);
        GW_TRY(hipGetLastError());
    }
    // the inverse pass applied couplings L-1 .. 0; go back through 0 .. L-1.
    // Every gradient of layer l is left as partial sums (split-K slices of the
    // weights, row-block sums of the biases) and summed by one kernel at the end.
    const int rb64 = (n + 63) / 64, rb16 = (n + gw::flow::kLayerRows - 1) / gw::flow::kLayerRows;
    gw::flow::BackChain chain;
    chain.count = 0;
    for (int l = 0; l < L; ++l) {
        float *wp = f->wpart + l * f->w_layer;
        double *bp = f->bpart + l * f->b_layer;
        float *wp1 = wp, *wp2 = wp + (int64_t)gw::flow::kMaxSplit * H * D,
              *wp3 = wp + (int64_t)gw::flow::kMaxSplit * (H * D + H * H);
        double *bp1 = bp, *bp2 = bp + (int64_t)f->rb_cap * H, *bp3 = bp + 2 * (int64_t)f->rb_cap * H;
        const uint16_t *h1 = f->h1_b + (int64_t)l * f->cap * H;
        const uint16_t *h2 = f->h2_b + (int64_t)l * f->cap * H;
        const int64_t T = f->ldT;
        const uint16_t *h1T = f->h1T + (int64_t)l * H * T, *h2T = f->h2T + (int64_t)l * H * T;
        const uint16_t *xmT = f->xmT + (int64_t)l * kInPad * T;
        // transposed BF16 weights of the layer: W1^T [D][H], W2^T [H][H], W3^T [H][kOutPad]
        const uint16_t *wt = f->wbT + (int64_t)l * f->wbT_stride;
        const int64_t w2t = (int64_t)D * H, w3t = (int64_t)D * H + (int64_t)H * H;
        if (fused_width(f)) {
            // the coupling's transposed operands of its weight gradients go to
            // layer l's slices, for the one launch of all layers' products
            // below; the couplings go out in chains of up to kMaxChain
            gw::flow::BackArgs ba{n, D, f->cond[l], f->g, boundary(f, l), f->s_store + (int64_t)l * f->cap * D, f->gy,
                                  h1T, h2T, wt, wt + w2t, wt + w3t, f->doutT + (int64_t)l * kOutPad * T,
                                  f->dpreT + (int64_t)l * H * T, f->dpre2T + (int64_t)l * H * T, T, bp1, bp2, bp3};
            chain.layer[chain.count++] = ba;
            if (chain.count == gw::flow::kMaxChain || l == L - 1) {
                const dim3 grid((unsigned)rb16);
                if (H == 256)
                    hipLaunchKernelGGL(gw::flow::layer_back_kernel<256>, grid, dim3(256), 0, s, chain);
                else
                    hipLaunchKernelGGL(gw::flow::layer_back_kernel<128>, grid, dim3(256), 0, s, chain);
                GW_TRY(hipGetLastError());
                chain.count = 0;
            }
            std::swap(f->g, f->gy);      // d loss / d(boundary l + 1)
            continue;
        }
        hipLaunchKernelGGL(gw::flow::coupling_inv_backward_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, D,
                           f->cond[l], f->g, boundary(f, l), f->s_store + (int64_t)l * f->cap * D, f->dout_b,
                           f->dout_f, f->gy, f->doutT, T);
        GW_TRY(hipGetLastError());
        hipLaunchKernelGGL(gw::flow::column_part_kernel, dim3(rb64), dim3(256), 0, s, n, 2 * D, kOutPad, f->dout_f, bp3);
        GW_TRY(hipGetLastError());
        // Every operand below is read k-contiguous: the sums over the batch
        // from the transposed copies (rows of length T), the products with
        // the weights from the transposed BF16 weights.
        // layer 3: dW3 = dout^T h2, db3 = colsum(dout), dh2 = dout W3,
        // dpre2 = dh2 (h2 > 0) with db2 = colsum(dpre2) in the same pass
        GemmArgs gw3{2 * D, H, n, f->doutT, T, 1, h2T, 1, T, nullptr, 0, nullptr, 0, nullptr, 0, split, wp3, 1};
        GW_TRY(gw::flow::gemm_bf16(gw3, s));
        GemmArgs gh2{n, H, 2 * D, f->dout_b, kOutPad, 1, wt + w3t, 1, kOutPad, f->dh, H, f->dpre_b, H, nullptr, 0};
        gh2.relu_of = h2;
        gh2.ld_relu = H;
        gh2.col_part = bp2;
        gh2.CbT = f->dpreT;
        gh2.ldcbT = T;
        GW_TRY(gw::flow::gemm_bf16(gh2, s));
        // layer 2: dW2 = dpre2^T h1, dh1 = dpre2 W2, dpre1 = dh1 (h1 > 0), db1 = colsum(dpre1)
        GemmArgs gw2{H, H, n, f->dpreT, T, 1, h1T, 1, T, nullptr, 0, nullptr, 0, nullptr, 0, split, wp2, 1};
        GW_TRY(gw::flow::gemm_bf16(gw2, s));
        GemmArgs gh1{n, H, H, f->dpre_b, H, 1, wt + w2t, 1, H, f->dh, H, f->dpre2_b, H, nullptr, 0};
        gh1.relu_of = h1;
        gh1.ld_relu = H;
        gh1.col_part = bp1;
        gh1.CbT = f->dpre2T;
        gh1.ldcbT = T;
        GW_TRY(gw::flow::gemm_bf16(gh1, s));
        // layer 1: dW1 = dpre1^T xm, dxm = dpre1 W1
        GemmArgs gw1{H, D, n, f->dpre2T, T, 1, xmT, 1, T, nullptr, 0, nullptr, 0, nullptr, 0, split, wp1, 1};
        GW_TRY(gw::flow::gemm_bf16(gw1, s));
        // d loss / d y += dxm on the conditioning dimensions, in the epilogue
        GemmArgs gx{n, D, H, f->dpre2_b, H, 1, wt, 1, H, nullptr, 0, nullptr, 0, nullptr, 0};
        gx.add_to = f->gy;
        gx.ld_add = D;
        gx.add_mask = f->cond[l];
        GW_TRY(gw::flow::gemm_bf16(gx, s));
        std::swap(f->g, f->gy);      // d loss / d(boundary l + 1)
    }
    if (fused_width(f)) {
        // every coupling's three weight gradients in one launch, layer by layer
        const int64_t T = f->ldT;
        float *wp = f->wpart;
        GemmArgs fw3{2 * D, H, n, f->doutT, T, 1, f->h2T, 1, T, nullptr, 0, nullptr, 0, nullptr, 0, split,
                     wp + (int64_t)gw::flow::kMaxSplit * (H * D + H * H), 1};
        GemmArgs fw2{H, H, n, f->dpreT, T, 1, f->h1T, 1, T, nullptr, 0, nullptr, 0, nullptr, 0, split,
                     wp + (int64_t)gw::flow::kMaxSplit * H * D, 1};
        GemmArgs fw1{H, D, n, f->dpre2T, T, 1, f->xmT, 1, T, nullptr, 0, nullptr, 0, nullptr, 0, split, wp, 1};
        const gw::flow::LayerStrides ls{{kOutPad * T, H * T, H * T}, {H * T, H * T, kInPad * T},
                                        {f->w_layer, f->w_layer, f->w_layer}};
        GW_TRY(gw::flow::gemm_bf16_group3(fw3, fw2, fw1, s, L, &ls));
    }
    gw::flow::GradParts parts{D, H, split, fused_width(f) ? rb16 : rb64, f->rb_cap, f->per_layer, f->n_params,
                              f->w_layer, f->b_layer, f->wpart, f->bpart};
    if (adam) {
        // the gradients' sums, the Adam step and the BF16 copies in one launch
        const int wblocks = blocks_for(f->n_params);
        const int64_t per_layer_tiles = 2 * ((H + gw::flow::kBiasCols - 1) / gw::flow::kBiasCols) +
                                        (2 * D + gw::flow::kBiasCols - 1) / gw::flow::kBiasCols;
        const int64_t tiles = parts.rb > 64 ? (int64_t)L * per_layer_tiles : 0;
        const int64_t blocks = wblocks + tiles + (loss_out ? 1 : 0);
        hipLaunchKernelGGL(gw::flow::finish_update_kernel, dim3((unsigned)blocks), dim3(256), 0, s, parts, f->grads,
                           *adam, bf16_copies(f), wblocks, tiles, n, f->loss, loss_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gw::flow::grad_finish_kernel, dim3(blocks_for(f->n_params)), dim3(256), 0, s, parts, f->grads);
    GW_TRY(hipGetLastError());
    if (parts.rb > 64) {
        hipLaunchKernelGGL(gw::flow::bias_finish_kernel, dim3((unsigned)(L * (2 * H + 2 * D))), dim3(64), 0, s, parts,
                           f->grads);
        GW_TRY(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t refresh_bf16(gw_flow *f, hipStream_t s)
{
    hipLaunchKernelGGL(gw::flow::to_bf16_kernel, dim3(blocks_for(f->n_params)), dim3(256), 0, s, f->n_params,
                       bf16_copies(f), f->params);
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
    f->wb_stride = (f->per_layer + 7) / 8 * 8;
    f->wbT_stride = (D * H + H * H + H * gw::flow::kOutPad + H * gw::flow::kInPad + 7) / 8 * 8;
    if (alloc(&f->params, f->n_params) || alloc(&f->grads, f->n_params) || alloc(&f->adam_m, f->n_params) ||
        alloc(&f->adam_v, f->n_params) || alloc(&f->wb, f->wb_stride * n_layers) ||
        alloc(&f->wbT, f->wbT_stride * n_layers) || alloc(&f->mu, dim) || alloc(&f->log_sigma, dim)) {
        gw_flow_destroy(f);
        return fail(GW_ENOMEM, "flow parameters");
    }
    // the padding of W3^T's and W1's rows is never written by to_bf16_kernel: zero it once
    if (hipMemset(f->wbT, 0, sizeof(uint16_t) * (size_t)(f->wbT_stride * n_layers)) != hipSuccess) {
        gw_flow_destroy(f);
        return fail(GW_EDEVICE, "flow parameters");
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
    void *ptrs[] = {f->params, f->grads, f->adam_m, f->adam_v, f->wb, f->wbT, f->mu, f->log_sigma};
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
    // the passes read z to the end (log q), so an x_out that overlaps it
    // takes a copy of z first
    const size_t bytes = sizeof(double) * (size_t)n * f->dim;
    const char *zb = reinterpret_cast<const char *>(z), *xb = reinterpret_cast<const char *>(x_out);
    const double *zin = z;
    hipError_t e = hipSuccess;
    if (zb < xb + bytes && xb < zb + bytes) {
        zin = boundary(f, 0);
        e = hipMemcpyAsync(boundary(f, 0), z, bytes, hipMemcpyDeviceToDevice, stream);
    }
    if (e == hipSuccess) e = forward_pass(f, (int)n, zin, x_out, logq_out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_flow_forward");
}

int gw_flow_inverse(gw_flow *f, const double *x, int64_t n, double *z_out, double *logq_out, hipStream_t stream)
{
    if (int rc = check_flow_call(f, x, n)) return rc;
    if (n == 0) return GW_OK;
    DeviceGuard g(f->device);
    if (int rc = ensure_batch(f, n)) return rc;
    DensityOut den;
    den.logq = logq_out;
    hipError_t e = inverse_pass(f, (int)n, x, false, stream, den);
    if (e == hipSuccess && z_out)
        e = hipMemcpyAsync(z_out, boundary(f, 0), sizeof(double) * n * f->dim, hipMemcpyDeviceToDevice, stream);
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
    const float b1 = 0.9f, b2 = 0.999f;
    const int64_t t = f->adam_t + 1;
    const gw::flow::AdamStep adam{f->params, f->adam_m, f->adam_v, lr, b1, b2, 1e-8f,
                                  1.0f - (float)std::pow(b1, (double)t), 1.0f - (float)std::pow(b2, (double)t)};
    hipError_t e = gradients(f, (int)n, x, loss_out, stream, &adam);
    if (e != hipSuccess) return hip_fail(e, "gw_flow_train_step");
    f->adam_t = t;
    return GW_OK;
}

}  // extern "C"

GW_DEFINE_SOURCE_HASH(flow)
