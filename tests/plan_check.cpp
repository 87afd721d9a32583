// Host check of the single-event launch planning and work distribution
// (gw_plan.h), built and run by tests/test_plan_host.py: chunk ranges tile
// the band exactly and in order, the per-XCD queues hand out every (chunk,
// group) item exactly once, and plans obey their rules.  Prints "ok <cases>"
// and exits 0, or prints the first failure and exits 1.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "gw_plan.h"

static int fail(const char *what, long long a, long long b, long long c, long long d)
{
    std::printf("FAIL %s: %lld %lld %lld %lld\n", what, a, b, c, d);
    return 1;
}

int main()
{
    long long cases = 0;
    // chunk ranges, every rounds value, many band sizes (zero included)
    const int64_t sizes[] = {0, 1, 2, 7, 63, 64, 65, 1000, 4017, 12345, 259585, 1040897, 16736257};
    for (int64_t n_eff : sizes)
        for (int rounds = 0; rounds <= 8; ++rounds)
            for (int per : {1, 2, 3, 7, 8, 16, 32, 48, 171, 256}) {
                const int n_chunks = per * (rounds > 1 ? rounds : 1);
                int64_t pos = 0;
                for (int c = 0; c < n_chunks; ++c) {
                    int64_t b, e;
                    gw::chunk_range(n_eff, c, n_chunks, rounds, b, e);
                    if (b < 0 || e < b || e > n_eff) return fail("range bounds", n_eff, rounds, n_chunks, c);
                    if (e > b) {
                        if (b != pos) return fail("range gap or overlap", n_eff, rounds, n_chunks, c);
                        pos = e;
                    }
                }
                if (pos != n_eff) return fail("range cover", n_eff, rounds, n_chunks, pos);
                ++cases;
            }
    // per-XCD queues: every item exactly once
    for (int n_chunks : {1, 3, 7, 8, 9, 16, 100, 192, 288, 1000})
        for (int n_groups : {1, 2, 5, 16, 17, 300}) {
            std::vector<int> seen((size_t)n_chunks * n_groups, 0);
            for (int x = 0; x < gw::kQueues; ++x)
                for (int k = 0;; ++k) {
                    int chunk = -1, group = -1;
                    if (!gw::queue_item(x, k, n_groups, n_chunks, chunk, group)) break;
                    if (chunk < 0 || chunk >= n_chunks || group < 0 || group >= n_groups || chunk % gw::kQueues != x)
                        return fail("queue item", x, k, chunk, group);
                    if (++seen[(size_t)chunk * n_groups + group] != 1) return fail("queue repeat", x, k, chunk, group);
                }
            for (int v : seen)
                if (v != 1) return fail("queue cover", n_chunks, n_groups, v, 0);
            ++cases;
        }
    // plans
    const int64_t samples[] = {1, 255, 256, 300, 4096, 5000, 100000};
    for (int64_t n_bins : sizes) {
        if (n_bins < 1) continue;
        for (int64_t n_samples : samples)
            for (int form : {0, 1, 2})
                for (int64_t resident : {256LL, 512LL, 768LL})
                for (int tile : {256, 512, 1024})
                for (int want : {-1, 0, 4, 6, 8}) {
                    // want < 0: the default number of rounds
                    const gw::TilePlan p = want < 0 ? gw::plan_single_event(n_bins, n_samples, form, tile, resident)
                                                    : gw::plan_single_event(n_bins, n_samples, form, tile, resident, want);
                    const int rounds = want < 0 ? GW_TILE_ROUNDS : want;
                    const int groups = (int)((n_samples + 255) / 256);
                    if (p.tile_bins != tile) return fail("plan tile", n_bins, n_samples, p.tile_bins, tile);
                    if (p.n_groups != groups) return fail("plan groups", n_bins, n_samples, p.n_groups, groups);
                    if (p.n_chunks < 1 || (int64_t)p.n_chunks > n_bins) return fail("plan chunks", n_bins, n_samples, p.n_chunks, 0);
                    if (p.rounds != 0 && p.rounds != rounds) return fail("plan rounds", n_bins, n_samples, p.rounds, rounds);
                    if (form == 1 && p.rounds != 0) return fail("plan isco static", n_bins, n_samples, p.rounds, 0);
                    if (p.rounds > 0) {
                        if (p.n_chunks % p.rounds != 0) return fail("plan round split", n_bins, n_samples, p.n_chunks, p.rounds);
                        if ((int64_t)p.n_chunks * 64 > n_bins) return fail("plan chunk size", n_bins, n_samples, p.n_chunks, 0);
                        if (p.blocks > resident || p.blocks < 1) return fail("plan blocks", n_bins, n_samples, p.blocks, resident);
                    } else {
                        if (p.blocks != p.n_groups * p.n_chunks) return fail("plan static blocks", n_bins, n_samples, p.blocks, 0);
                        if (p.chunk_bins * p.n_chunks < n_bins) return fail("plan static cover", n_bins, n_samples, p.chunk_bins, p.n_chunks);
                    }
                    ++cases;
                }
    }
    std::printf("ok %lld\n", cases);
    return 0;
}
