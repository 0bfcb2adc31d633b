// Host side of the cost-diagonal build (Sec. IV-A, Eq. (2)): every term of a
// MaxCut, QUBO or 0-1 polynomial cost is turned into one or two "pieces" in
// the thread layout of the cost kernel, so that the kernel can skip a term
// for a whole wavefront when one of its variables decides it there.
//
// Layout of the kernel (kernels.hip, k_cost_pieces): z bits 0-5 are the lane,
// bits 6-9 the index q of a thread's 16 entries, bits >= 10 are the same for
// every thread of a wavefront.  A piece is a conjunction of literals
// (variable v has value b); its literals on bits >= 10 become a wave-uniform
// test, those on bits 0-5 a per-lane test, and those on bits 6-9 the set of
// entries q it covers.
//   0-1 term (Eq. (2), QUBO pair or linear term): one piece, every variable 1.
//   MaxCut edge (x_i XOR x_j): the pieces (x_i, x_j) = (1, 0) and (0, 1); when
//   both variables sit in bits 6-9 they form one piece covering the q with
//   unequal bits.
// The pieces of a term cover disjoint sets of z, so adding the weight once
// per covering piece, term after term, adds exactly the active terms in the
// given order.
#include "qaoa_internal.h"

namespace qk {
namespace {

struct Lit {
    int v;
    int b;
};

void fill_weights(CostPiece &p)
{
    for (int q = 0; q < 16; ++q) p.wq[q] = ((p.qpat >> q) & 1u) ? p.w : -0.0;
}

CostPiece make_piece(const Lit *lits, int nlit, double w)
{
    CostPiece p{};
    p.w = w;
    uint32_t rm = 0, rv = 0, lm = 0, lv = 0;
    for (int i = 0; i < nlit; ++i) {
        const int v = lits[i].v;
        const uint32_t b = lits[i].b ? 1u : 0u;
        if (v >= kCostUniformBit) {
            p.umask |= 1ull << v;
            p.uval |= (uint64_t)b << v;
        } else if (v >= kCostLaneBits) {
            rm |= 1u << (v - kCostLaneBits);
            rv |= b << (v - kCostLaneBits);
        } else {
            lm |= 1u << v;
            lv |= b << v;
        }
    }
    for (uint32_t q = 0; q < 16; ++q)
        if ((q & rm) == rv) p.qpat |= 1u << q;
    p.lanes = lm | (lv << 8);
    fill_weights(p);
    return p;
}

// Appends the pieces of one term; pieces of the term with the same wave and
// lane tests are merged (their entry sets are disjoint).
void push_term(std::vector<CostPiece> &out, const CostPiece *pc, int np)
{
    const size_t first = out.size();
    for (int i = 0; i < np; ++i) {
        bool merged = false;
        for (size_t k = first; k < out.size(); ++k)
            if (out[k].umask == pc[i].umask && out[k].uval == pc[i].uval && out[k].lanes == pc[i].lanes) {
                out[k].qpat |= pc[i].qpat;
                fill_weights(out[k]);
                merged = true;
                break;
            }
        if (!merged) out.push_back(pc[i]);
    }
}

void push_and(std::vector<CostPiece> &out, uint64_t mask, double w)
{
    Lit lits[64];
    int nl = 0;
    for (int v = 0; v < 64; ++v)
        if ((mask >> v) & 1ull) lits[nl++] = Lit{v, 1};
    const CostPiece p = make_piece(lits, nl, w);
    push_term(out, &p, 1);
}

}  // namespace

std::vector<CostPiece> cost_pieces_maxcut(int64_t m, const int32_t *edges, const double *w)
{
    std::vector<CostPiece> out;
    out.reserve((size_t)m * 2);
    for (int64_t k = 0; k < m; ++k) {
        const int i = edges[2 * k], j = edges[2 * k + 1];
        const double wk = w ? w[k] : 1.0;
        const Lit a[2] = {{i, 1}, {j, 0}}, b[2] = {{i, 0}, {j, 1}};
        const CostPiece pc[2] = {make_piece(a, 2, wk), make_piece(b, 2, wk)};
        push_term(out, pc, 2);
    }
    return out;
}

std::vector<CostPiece> cost_pieces_qubo(int n, int64_t m, const int32_t *pairs, const double *J,
                                        const double *h)
{
    std::vector<CostPiece> out;
    out.reserve((size_t)m + (h ? (size_t)n : 0));
    for (int64_t k = 0; k < m; ++k)
        push_and(out, (1ull << pairs[2 * k]) | (1ull << pairs[2 * k + 1]), J[k]);
    if (h)
        for (int i = 0; i < n; ++i) push_and(out, 1ull << i, h[i]);
    return out;
}

std::vector<CostPiece> cost_pieces_poly(int64_t L, const uint64_t *masks, const double *w)
{
    std::vector<CostPiece> out;
    out.reserve((size_t)L);
    for (int64_t k = 0; k < L; ++k) push_and(out, masks[k], w[k]);
    return out;
}

}  // namespace qk
