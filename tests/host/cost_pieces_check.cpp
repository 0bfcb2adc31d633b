// Host check of the cost-diagonal pieces (run under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py).  For random
// MaxCut, QUBO and 0-1 polynomial instances it evaluates C[z] the way the cost
// kernel does -- offset, then for each piece in order, add wq[q] when the
// wavefront bits and the lane bits of z pass the piece's tests, with
// lane = z bits 0-5, q = z bits 6-9 and the wavefront bits = z bits >= 10 --
// and compares every entry bit for bit (signed zeros included) with the plain
// definition: the offset plus the weights of the active terms, added in term
// order (Sec. IV-A, Eq. (2); MaxCut terms are x_i XOR x_j).
#include "qaoa_internal.h"

#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

namespace {

double emulate(const std::vector<qk::CostPiece> &pc, double offset, uint64_t z)
{
    const uint64_t zw = z & ~((1ull << qk::kCostUniformBit) - 1ull);
    const uint32_t lane = (uint32_t)(z & 63u), q = (uint32_t)((z >> 6) & 15u);
    double acc = offset;
    for (const qk::CostPiece &p : pc) {
        if ((zw & p.umask) != p.uval) continue;
        if ((lane & p.lanes & 63u) != (p.lanes >> 8)) continue;
        acc += p.wq[q];
    }
    return acc;
}

bool same(double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; }

int check(const char *what, int n, const std::vector<qk::CostPiece> &pc, double offset,
          const std::vector<double> &ref)
{
    for (uint64_t z = 0; z < (1ull << n); ++z) {
        const double g = emulate(pc, offset, z);
        if (!same(g, ref[z])) {
            std::printf("%s n=%d z=%llu: %.17g vs %.17g\n", what, n, (unsigned long long)z, g, ref[z]);
            return 1;
        }
    }
    return 0;
}

}  // namespace

int main()
{
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    long entries = 0;
    for (int trial = 0; trial < 60; ++trial) {
        const int n = 2 + (int)(rng() % 13);  // 2..14: every bit class (lane, entry, wavefront)
        const int m = (int)(rng() % 40);
        std::vector<int32_t> e;
        std::vector<double> w;
        for (int k = 0; k < m; ++k) {
            const int i = (int)(rng() % n);
            int j = (int)(rng() % n);
            if (j == i) j = (i + 1) % n;
            e.push_back(i);
            e.push_back(j);
            // integer, real and signed-zero weights
            const int kind = (int)(rng() % 4);
            w.push_back(kind == 0 ? (double)(int)(rng() % 7) - 3.0 : kind == 1 ? -0.0 : U(rng));
        }
        // MaxCut: C[z] = sum over cut edges in edge order, starting from +0
        {
            std::vector<double> ref(1ull << n);
            for (uint64_t z = 0; z < ref.size(); ++z) {
                double c = 0.0;
                for (int k = 0; k < m; ++k)
                    if (((z >> e[2 * k]) ^ (z >> e[2 * k + 1])) & 1ull) c += w[k];
                ref[z] = c;
            }
            if (check("maxcut", n, qk::cost_pieces_maxcut(m, e.data(), w.data()), 0.0, ref)) return 1;
            std::vector<double> ones(1ull << n);
            for (uint64_t z = 0; z < ones.size(); ++z) {
                double c = 0.0;
                for (int k = 0; k < m; ++k)
                    if (((z >> e[2 * k]) ^ (z >> e[2 * k + 1])) & 1ull) c += 1.0;
                ones[z] = c;
            }
            if (check("maxcut unit", n, qk::cost_pieces_maxcut(m, e.data(), nullptr), 0.0, ones)) return 1;
        }
        // QUBO: offset, pairs in order, then linear terms in variable order
        {
            std::vector<double> h(n);
            for (int i = 0; i < n; ++i) h[i] = (trial % 5 == 0) ? -0.0 : U(rng);
            const double offset = (trial % 3 == 0) ? -0.0 : U(rng);
            std::vector<double> ref(1ull << n);
            for (uint64_t z = 0; z < ref.size(); ++z) {
                double c = offset;
                for (int k = 0; k < m; ++k)
                    if ((z >> e[2 * k]) & (z >> e[2 * k + 1]) & 1ull) c += w[k];
                for (int i = 0; i < n; ++i)
                    if ((z >> i) & 1ull) c += h[i];
                ref[z] = c;
            }
            if (check("qubo", n, qk::cost_pieces_qubo(n, m, e.data(), w.data(), h.data()), offset, ref))
                return 1;
        }
        // 0-1 polynomial with random masks (the empty mask is a constant term)
        {
            const int L = (int)(rng() % 30);
            std::vector<uint64_t> mk(L);
            std::vector<double> wk(L);
            for (int k = 0; k < L; ++k) {
                mk[k] = rng() & ((1ull << n) - 1ull) & rng();
                wk[k] = U(rng);
            }
            const double offset = U(rng);
            std::vector<double> ref(1ull << n);
            for (uint64_t z = 0; z < ref.size(); ++z) {
                double c = offset;
                for (int k = 0; k < L; ++k)
                    if ((z & mk[k]) == mk[k]) c += wk[k];
                ref[z] = c;
            }
            if (check("poly", n, qk::cost_pieces_poly(L, mk.data(), wk.data()), offset, ref)) return 1;
        }
        entries += 4l << n;
    }
    std::printf("cost pieces ok (%ld entries)\n", entries);
    return 0;
}
