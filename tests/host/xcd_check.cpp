// The tile order of the pass launches (qk::xcd_tile with qk::xcd_group_bits):
// for every tile count a sweep can have, and for the half counts of the
// two-tiles-per-workgroup launches (grouping derived from the full count's, as
// the pair launcher does), every tile is visited exactly once, and the
// grouping is the largest one (at most 16 consecutive tiles per XCD) that
// keeps the order a permutation.
#include "qaoa_internal.h"

#include <cstdio>
#include <vector>

static bool permutes(uint64_t count, uint32_t G)
{
    std::vector<unsigned char> seen(count, 0);
    for (uint64_t L = 0; L < count; ++L) {
        const uint64_t t = qk::xcd_tile(L, G);
        if (t >= count || seen[t]) return false;
        seen[t] = 1;
    }
    return true;
}

int main()
{
    int bad = 0;
    std::vector<uint64_t> counts;
    for (int k = 0; k <= 22; ++k) counts.push_back(1ull << k);
    for (uint64_t c : {3ull, 24ull, 48ull, 96ull, 384ull, 1536ull, 40ull * 1024}) counts.push_back(c);
    for (uint64_t count : counts) {
        const uint32_t g = qk::xcd_group_bits(count, 4);
        if (!permutes(count, g)) {
            std::printf("tile order of %llu tiles (G = %u) is not a permutation\n", (unsigned long long)count, g);
            ++bad;
        }
        // largest admissible grouping
        for (uint32_t h = g + 1; h <= 4; ++h)
            if (count % (8ull << h) == 0) {
                std::printf("grouping %u of %llu tiles is not the largest\n", g, (unsigned long long)count);
                ++bad;
            }
        if (count >= 2 && count % 2 == 0) {
            const uint64_t pairs = count / 2;
            const uint32_t gp = qk::xcd_group_bits(pairs, g);
            if (gp > g || !permutes(pairs, gp)) {
                std::printf("pair order of %llu pairs (G = %u) is not a permutation\n", (unsigned long long)pairs, gp);
                ++bad;
            }
        }
    }
    // the single-tile grouping applied to the pairs is not a permutation for some counts
    if (permutes(8, qk::xcd_group_bits(16, 4))) {
        std::printf("expected the 16-tile grouping to fail on 8 pairs\n");
        ++bad;
    }
    if (bad) return 1;
    std::printf("tile order ok\n");
    return 0;
}
