// Internal interface of the random-number and Metropolis-Hastings kernels.
#pragma once

#include <cstdint>
#include <string>

#include <hip/hip_runtime.h>

namespace gw {

// Records msg as the thread's last error (gw_last_error) and returns code.
int set_error(int code, const std::string &msg);
namespace mcmc {

constexpr int kMaxDim = 16;

// Philox streams: independent sequences for the different draws of a step.
enum : uint32_t { kStreamRandomWalk = 1, kStreamAccept = 2, kStreamFlow = 3, kStreamUser = 16 };
enum : int { kModeFlow = 0, kModeRandomWalk = 1 };

struct Box {
    double lo[kMaxDim], hi[kMaxDim];
};

hipError_t philox_raw(uint64_t seed, uint32_t stream, uint32_t step, uint64_t first, int64_t n_blocks, uint32_t *out,
                      hipStream_t s);
hipError_t philox_fill(uint64_t seed, uint32_t stream, uint32_t step, int kind, int64_t n, double *out, hipStream_t s);
hipError_t normals_for_chains(int dim, int64_t n, uint64_t seed, uint32_t stream, uint32_t step, double *out,
                              hipStream_t s);
hipError_t to_theta(int dim, int64_t n, const Box &box, const double *x, int theta_cols, double *theta,
                    double *logprior, hipStream_t s);
hipError_t rw_propose(int dim, int64_t n, const double *x, const double *chol, uint64_t seed, uint32_t step,
                      const int *mode, double *x_prop, hipStream_t s);
hipError_t accept(int dim, int64_t n, uint64_t seed, uint32_t step, double *x, double *lnp, double *logq,
                  const double *x_prop, const double *lnl_prop, const double *lp_prop, const double *logq_prop,
                  const int *mode, int *window_accepts, int *total_accepts, hipStream_t s);
hipError_t update_mode(int64_t n, int *window_accepts, int window, double threshold, int *mode, hipStream_t s);
hipError_t adapt_chol(int dim, int64_t n, const double *x, double scale, double floor, double *chol, double *mean,
                      double *cov, hipStream_t s);
hipError_t count_sum(int64_t n, const int *counts, int64_t *out, hipStream_t s);
hipError_t gather_rows(int dim, int64_t n_out, const double *src, int64_t n_src, uint64_t seed, uint32_t stream,
                       uint32_t step, double *dst, hipStream_t s);

}  // namespace mcmc
}  // namespace gw
