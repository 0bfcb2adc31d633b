// Host check of the pass planner (run under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py): for every
// precision, n in [1, 40] and every cap on the qubits of a later pass, each
// plan entry must have a valid kernel geometry and the targets must cover the
// n qubits exactly once.
#include "qaoa_internal.h"

#include <cstdio>

int main()
{
    long tiles = 0;
    for (int c64 = 0; c64 < 2; ++c64)
        for (int n = 1; n <= 40; ++n)
            for (int kmax = 0; kmax <= 12; ++kmax) {
                const std::vector<qk::PassPlan> pl = qk::plan_passes(n, c64 != 0, kmax);
                uint64_t seen = 0;
                for (const qk::PassPlan &p : pl) {
                    qk::Geometry g;
                    if (!qk::make_geometry(n, p, &g)) {
                        std::printf("no geometry: n=%d c64=%d kmax=%d\n", n, c64, kmax);
                        return 1;
                    }
                    if ((seen & p.target_bits) || (p.target_bits & ~p.tile_bits)) {
                        std::printf("bad targets: n=%d c64=%d kmax=%d\n", n, c64, kmax);
                        return 1;
                    }
                    seen |= p.target_bits;
                    tiles += g.tbits;
                }
                if (seen != (1ull << n) - 1) {
                    std::printf("qubits not covered: n=%d c64=%d kmax=%d\n", n, c64, kmax);
                    return 1;
                }
            }
    std::printf("plans ok (%ld tile bits)\n", tiles);
    return 0;
}
