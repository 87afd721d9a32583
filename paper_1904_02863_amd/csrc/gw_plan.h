// Launch planning of the single-event tile kernel (host side): the LDS tile
// size and the split of a call into (sample group, bin chunk) work items.
// Kept apart from the API code because it decides what the kernel reads and
// writes per launch.
#pragma once

#include <algorithm>
#include <cstdint>

#include "gw_internal.h"

// Bytes of LDS per tile block (tiles plus, on the FP64 path, the phasor
// table); two blocks per CU fit in 160 KB.
#ifndef GW_TILE_LDS_BUDGET
#define GW_TILE_LDS_BUDGET (72 * 1024)
#endif
// Work distribution: 0, one block per (group, chunk) item in one wave of
// resident blocks; R >= 1, a persistent grid over one work queue per XCD,
// the chunks in R rounds of one item per resident block, round r (R > 1)
// covering half the bins the earlier rounds left.  The queue evens out what
// a static split leaves uneven: the wave arbiter favours the oldest wave of a
// SIMD, so co-resident blocks of equal work finish far apart, and a SIMD left
// with one wave issues at about half rate.
#ifndef GW_TILE_ROUNDS
#define GW_TILE_ROUNDS 6
#endif

namespace gw {

// Bins [k_begin, k_end) of chunk c among n_chunks chunks of n_eff bins.
// rounds <= 1: equal chunks.  rounds R > 1: the chunks come in R rounds of
// n_chunks / R equal chunks each; round r < R - 1 covers the next half of the
// bins still left (n_eff/2, n_eff/4, ...) and the last round the rest, so that
// a queue handing out chunks in index order ends on small ones.
__host__ __device__ inline void chunk_range(int64_t n_eff, int64_t c, int n_chunks, int rounds, int64_t &k_begin,
                                            int64_t &k_end)
{
    if (rounds <= 1) {
        int64_t cb = (n_eff + n_chunks - 1) / n_chunks;
        cb = cb > 1 ? cb : 1;
        k_begin = c * cb < n_eff ? c * cb : n_eff;
        k_end = k_begin + cb < n_eff ? k_begin + cb : n_eff;
        return;
    }
    const int64_t per = n_chunks / rounds;
    const int64_t r = c / per, j = c % per;
    const int64_t rb = n_eff - (n_eff >> r);
    const int64_t re = (r == rounds - 1) ? n_eff : n_eff - (n_eff >> (r + 1));
    k_begin = rb + (re - rb) * j / per;
    k_end = rb + (re - rb) * (j + 1) / per;
}

// Item k of work queue x (kQueues queues): queue x holds the chunks
// c = x (mod kQueues) in index order, all n_groups sample groups of a chunk
// together.  False once the queue is exhausted.
__host__ __device__ inline bool queue_item(int x, int k, int n_groups, int n_chunks, int &chunk, int &group)
{
    const int n_x = x < n_chunks ? n_groups * ((n_chunks - x + kQueues - 1) / kQueues) : 0;
    if (k >= n_x) return false;
    chunk = x + kQueues * (k / n_groups);
    group = k % n_groups;
    return true;
}

inline int tile_bins_for(int n_det, int form, bool mixed)
{
    int t = 2048;
    while (t > 64 && lnl_tile_lds_bytes(n_det, t, form, mixed) > (size_t)GW_TILE_LDS_BUDGET) t /= 2;
    return t;
}

// resident: blocks of this kernel that fit on the device at once; rounds:
// work-queue rounds (0: one block per item), GW_TILE_ROUNDS by default.
inline TilePlan plan_single_event(int64_t n_bins, int64_t n_samples, int form, int tile_bins, int64_t resident,
                                  int rounds = GW_TILE_ROUNDS)
{
    TilePlan p;
    p.tile_bins = tile_bins;
    p.n_groups = (int)((n_samples + kBlock - 1) / kBlock);
    int64_t chunks = (resident + p.n_groups - 1) / p.n_groups;
    const int64_t max_chunks = std::max<int64_t>(1, n_bins / 64);     // at least 64 bins per chunk
    chunks = std::max<int64_t>(1, std::min(chunks, max_chunks));
    p.chunk_bins = (n_bins + chunks - 1) / chunks;
    p.n_chunks = (int)((n_bins + p.chunk_bins - 1) / p.chunk_bins);
    p.rounds = 0;
    p.blocks = p.n_groups * p.n_chunks;
    // the ISCO end leaves the device-side band unknown here and usually short:
    // one item per resident block
    if (rounds >= 1 && form != kFormSplitIsco && (int64_t)p.n_chunks * rounds * 64 <= n_bins) {
        p.rounds = rounds;
        p.n_chunks *= rounds;
        p.chunk_bins = (n_bins + p.n_chunks - 1) / p.n_chunks;
        p.blocks = (int)std::min<int64_t>((int64_t)p.n_groups * p.n_chunks, resident);
    }
    return p;
}

}  // namespace gw
