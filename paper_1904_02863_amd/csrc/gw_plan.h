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

inline int tile_bins_for(int n_det, int form, bool mixed)
{
    int t = 2048;
    while (t > 64 && lnl_tile_lds_bytes(n_det, t, form, mixed) > (size_t)GW_TILE_LDS_BUDGET) t /= 2;
    return t;
}

// resident: blocks of this kernel that fit on the device at once.
inline TilePlan plan_single_event(int64_t n_bins, int64_t n_samples, int form, int tile_bins, int64_t resident)
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
    const int rounds = GW_TILE_ROUNDS;
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
