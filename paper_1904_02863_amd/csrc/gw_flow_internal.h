// Internal interface of the flow and sampler kernels (gw_flow.hip).
#pragma once

#include <cstdint>
#include <string>

#include <hip/hip_runtime.h>

namespace gw {

// Records msg as the thread's last error (gw_last_error) and returns code.
int set_error(int code, const std::string &msg);
namespace flow {

constexpr int kInPad = 16;    // MLP input row (dim <= 16)
constexpr int kOutPad = 32;   // MLP output row (2 dim <= 32)

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;     // BF16
    int64_t sa_i, sa_k;
    const uint16_t *B;     // BF16
    int64_t sb_k, sb_j;
    float *C;              // FP32 output (may be null)
    int64_t ldc;
    uint16_t *Cb;          // BF16 copy of the output (may be null)
    int64_t ldcb;
    const float *bias;     // [N] (may be null)
    int relu;
    // split-K: with split > 1 the K range is cut into `split` slices whose
    // FP32 partial products go to partial [split][M][N]; a second kernel sums
    // them in slice order and applies bias, ReLU and the outputs
    int split = 1;
    float *partial = nullptr;
    // defer: the slices go to partial (also with split 1) and are left there
    // for the caller to sum (no second kernel)
    int defer = 0;
    // backward ReLU (split 1): outputs are kept where relu_of(i, j), a BF16
    // activation [M][ld_relu], is > 0, and zeroed elsewhere
    const uint16_t *relu_of = nullptr;
    int64_t ld_relu = 0;
    // (split 1) column sums of the final FP32 outputs over each 64-row block
    // of the tile grid, in FP64 and a fixed order: col_part [ceil(M/64)][N]
    double *col_part = nullptr;
    // (split 1) transposed BF16 copy of the output: CbT[j ldcbT + i]
    // (ldcbT a multiple of 4, CbT 8-byte aligned)
    uint16_t *CbT = nullptr;
    int64_t ldcbT = 0;
    // (split 1) add_to[i ld_add + j] += output (in FP64) for the columns j
    // whose bit is set in add_mask (j < 32)
    double *add_to = nullptr;
    int64_t ld_add = 0;
    unsigned add_mask = 0;
};

constexpr int kMaxSplit = 16;

hipError_t gemm_bf16(const GemmArgs &g, hipStream_t stream);
// Per-layer element strides of a grouped launch over several layers: product
// p of layer l reads A + l sA[p] and B + l sB[p] and writes its slices to
// partial + l sP[p] (multiples of 8 elements).
struct LayerStrides {
    int64_t sA[3], sB[3], sP[3];
};

// Three products in one launch (k-contiguous operands, split-K slices left
// in their partial buffers); with layers > 1 and strides, the same three for
// each of `layers` layers, layer by layer.
hipError_t gemm_bf16_group3(const GemmArgs &a, const GemmArgs &b, const GemmArgs &c, hipStream_t stream,
                            int layers = 1, const LayerStrides *strides = nullptr);

}  // namespace flow
}  // namespace gw
