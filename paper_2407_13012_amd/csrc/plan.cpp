// Pass planning for the mixer layer (host only).
//
// The mixer prod_j exp(-i b X_j) (Eq. (1)) factorises over qubits and its
// factors commute, so a layer may rotate any group of qubits per sweep over
// the state.  A sweep here is a tiled pass: a workgroup owns 2^TB amplitudes
// whose indices differ only in TB chosen bits (the tile bits; TB = 12 for
// 16-byte amplitudes, 13 for 8-byte ones, 64 KiB either way) and rotates the
// target bits among them.  The plan fixes, for one layer, the tile bits and
// target bits of each pass:
//   * pass 0 rotates a contiguous run of low bits [0, TB - x0) plus x0 high
//     bits, so its global accesses are runs of >= 64 consecutive amplitudes;
//   * passes 1.. keep the S = TB - k lowest bits as non-rotated spectators
//     (runs of 2^S consecutive amplitudes) and rotate k <= 10 further bits,
//     so that runs are >= 64 bytes at either precision;
//   * bits whose stride spans a 2 MiB page (bit >= 17 for 16-byte amplitudes,
//     >= 18 for 8-byte ones) are spread evenly over the passes, since every
//     such target bit doubles the number of pages one tile touches.
#include "qaoa_internal.h"

#include <algorithm>

namespace qk {

namespace {

uint64_t low_mask(int b) { return b >= 64 ? ~0ull : ((1ull << b) - 1ull); }

// Split the set bits of `m` (restricted to [0, n)) into maximal runs of
// consecutive bits, listed in ascending order.
std::vector<std::pair<int, int>> runs_of(uint64_t m, int n)
{
    std::vector<std::pair<int, int>> r;  // (first bit, length)
    int b = 0;
    while (b < n) {
        if (!((m >> b) & 1ull)) {
            ++b;
            continue;
        }
        int e = b;
        while (e < n && ((m >> e) & 1ull)) ++e;
        r.push_back({b, e - b});
        b = e;
    }
    return r;
}

std::vector<PassPlan> plan_simple(int n, int TB, int kmax)
{
    std::vector<PassPlan> out;
    out.push_back({low_mask(TB), low_mask(TB)});
    const int r = n - TB, P = (r + kmax - 1) / kmax;
    int h = TB;
    for (int i = 0; i < P; ++i) {
        const int k = r / P + (i < r % P ? 1 : 0);
        const uint64_t tg = low_mask(k) << h;
        out.push_back({tg | low_mask(TB - k), tg});
        h += k;
    }
    return out;
}

bool plan_ok(int n, int TB, const std::vector<PassPlan> &pl)
{
    uint64_t seen = 0;
    for (const PassPlan &p : pl) {
        if (__builtin_popcountll(p.tile_bits) != std::min(n, TB)) return false;
        if ((p.target_bits & ~p.tile_bits) || (seen & p.target_bits)) return false;
        seen |= p.target_bits;
        Geometry g;
        if (!make_geometry(n, p, &g)) return false;
    }
    return seen == low_mask(n);
}

}  // namespace

std::vector<PassPlan> plan_passes(int n, bool c64, int kmax)
{
    const int TB = tile_bits(c64);
    if (n <= TB) return {{low_mask(n), low_mask(n)}};
    if (kmax < 1) kmax = 1;
    // >= TB - 10 spectator bits: runs of >= 4 (16-byte) or >= 8 (8-byte) amplitudes
    if (kmax > 10) kmax = 10;
    const int page = c64 ? 18 : 17;
    const int r = n - TB, P1 = (r + kmax - 1) / kmax;
    std::vector<int> k(P1 + 1), x(P1 + 1, 0), cap(P1 + 1);
    k[0] = TB;
    for (int i = 0; i < P1; ++i) k[i + 1] = r / P1 + (i < r % P1 ? 1 : 0);
    cap[0] = TB - 6;  // pass 0 keeps >= 64 consecutive amplitudes
    for (int i = 1; i <= P1; ++i) cap[i] = k[i];
    int left = std::max(0, n - page);
    while (left > 0) {
        bool moved = false;
        for (int i = 0; i <= P1 && left > 0; ++i)
            if (x[i] < cap[i]) {
                ++x[i];
                --left;
                moved = true;
            }
        if (!moved) break;
    }
    std::vector<PassPlan> out(P1 + 1);
    int nc = TB - x[0];           // next non-crossing bit to hand out
    int cr = std::max(page, TB);  // next crossing bit to hand out
    if (n <= page) cr = n;
    // Crossing bits are handed out in ascending blocks: pass 1 first, then
    // pass 0, then passes 2..  (the order measured fastest at n = 32).
    std::vector<int> order;
    if (P1 >= 1) order.push_back(1);
    order.push_back(0);
    for (int i = 2; i <= P1; ++i) order.push_back(i);
    std::vector<uint64_t> crossing(P1 + 1, 0);
    for (int i : order)
        for (int j = 0; j < x[i]; ++j) crossing[i] |= 1ull << cr++;
    out[0].target_bits = low_mask(TB - x[0]) | crossing[0];
    out[0].tile_bits = out[0].target_bits;
    for (int i = 1; i <= P1; ++i) {
        uint64_t tg = crossing[i];
        for (int j = 0; j < k[i] - x[i]; ++j) tg |= 1ull << nc++;
        out[i].target_bits = tg;
        out[i].tile_bits = tg | low_mask(TB - k[i]);
    }
    if (!plan_ok(n, TB, out)) out = plan_simple(n, TB, kmax);
    return out;
}

bool make_geometry(int n, const PassPlan &pp, Geometry *g)
{
    *g = Geometry{};
    const auto tr = runs_of(pp.tile_bits, n);
    const auto fr = runs_of(low_mask(n) & ~pp.tile_bits, n);
    if ((int)tr.size() > kTileRuns || (int)fr.size() > kFreeRuns) return false;
    uint32_t local = 0;
    for (size_t i = 0; i < tr.size(); ++i) {
        g->t_src[i] = local;
        g->t_dst[i] = (uint32_t)tr[i].first;
        g->t_len[i] = (uint32_t)tr[i].second;
        for (int j = 0; j < tr[i].second; ++j)
            if ((pp.target_bits >> (tr[i].first + j)) & 1ull) g->tmask |= 1u << (local + j);
        local += (uint32_t)tr[i].second;
    }
    uint32_t t = 0;
    for (size_t i = 0; i < fr.size(); ++i) {
        g->f_src[i] = t;
        g->f_dst[i] = (uint32_t)fr[i].first;
        g->f_len[i] = (uint32_t)fr[i].second;
        t += (uint32_t)fr[i].second;
    }
    g->tbits = local;
    // accesses are coalesced only if the lowest tile bits start at bit 0
    return tr.empty() ? false : tr[0].first == 0;
}

}  // namespace qk
