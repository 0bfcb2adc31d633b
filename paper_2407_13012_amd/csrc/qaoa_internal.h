// Internal interface between the C-ABI layer (api.cpp) and the gfx950 kernels
// (kernels.hip).  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qaoa.h"

#include <string>
#include <vector>

namespace qk {

// Tile geometry of the streaming pass kernel: a workgroup owns 2^12
// complex128 amplitudes (256 threads) or 2^13 complex64 ones (512 threads),
// 16 per thread and 64 KiB of state either way.
constexpr int kTileBits = 12;    // complex128
constexpr int kTileBits64 = 13;  // complex64
constexpr int tile_bits(bool c64) { return c64 ? kTileBits64 : kTileBits; }
constexpr int kTile = 1 << kTileBits;  // elements per workgroup of the plain streaming kernels
constexpr int kThreads = 256;          // threads per workgroup of every kernel but the complex64 passes

// Pass modes.
enum PassMode : int {
    kFwd = 0,   // one vector: [init|load] [phase] mixer [E] store
    kTurn = 1,  // last forward group fused with the first backward group
    kBwd = 2,   // two vectors: mixer^dag with <lam|X_j|phi>, [phase^dag with <lam|C|phi>]
    kTurnPhase = 3, // turn pass of a one-pass layer (n <= TB): also applies and undoes the phase
    // Layer-boundary passes.  Consecutive layers visit their mixer groups in
    // opposite orders, so the last group of layer l and the first group of
    // layer l+1 share a geometry and one sweep serves both:
    kFwdFuse = 4,   // group of layer l, phase of layer l+1, same group of layer l+1
    kBwdFuse = 5    // their inverses with the <lam|X|phi> terms of both layers and <lam|C|phi>
};

// Pass flags.
enum PassFlags : int {
    kInit = 1,       // generate |+> instead of loading the state
    kPhaseIn = 2,    // multiply by exp(-i gamma_in C) before the mixer group
    kEOut = 4,       // accumulate sum C |psi|^2 (kFwd after the mixer; always in kTurn)
    kPhaseOut = 8,   // (kBwd, kTurn) accumulate Im <lam|C|phi>, then multiply both by exp(+i gamma_out C)
    kNoStore = 16,   // skip the final store (last backward pass)
    kBetaAcc = 32,   // add the <lam|X|phi> partial to the existing one instead of overwriting
    kStream = 64,    // nontemporal loads/stores (tiles with long contiguous runs)
    kBetaAcc2 = 128, // kBetaAcc for the second rotation's partials (kBwdFuse)
    kLamFromC = 256, // (kBwd) lam = C phi formed from the loaded phi instead of loaded
    kFarPhase = 512  // |gamma| max|C| may leave the fast phase reduction's range
};

// Below this bound on |gamma| max|C| every phase takes the fast reduction
// (complex128: Cody-Waite for |x| < 1e6; complex64: the fp32 path for
// |g1 C| < 4096), with a factor of 2 to spare for rounding of gamma and C.
constexpr double near_phase_limit(bool c64) { return c64 ? 2048.0 : 5.0e5; }

// One pass of a mixer layer.  A tile is the set of 2^TB basis indices that
// agree outside `tile_bits` (TB = tile_bits(c64)); the pass rotates the qubits
// in `target_bits` (a subset of tile_bits; the rest are spectators kept for
// contiguous access).
struct PassPlan {
    uint64_t tile_bits;
    uint64_t target_bits;
};

constexpr int kTileRuns = 4;  // runs of consecutive global bits inside a tile
constexpr int kFreeRuns = 5;  // runs of consecutive global bits of the tile index

// Tile geometry in kernel form: tile-local bit (src + i) of run r sits at
// global bit (dst + i), i < len; likewise for the tile-index bits.
struct Geometry {
    uint32_t t_src[kTileRuns], t_dst[kTileRuns], t_len[kTileRuns];
    uint32_t f_src[kFreeRuns], f_dst[kFreeRuns], f_len[kFreeRuns];
    uint32_t tmask;  // tile-local bits that are rotated
    uint32_t tbits;  // number of valid tile-local bits (TB, or n when n < TB)
};

// Pass plan of one mixer layer on n qubits (host).  Every qubit is a target of
// exactly one pass; the first pass holds bits [0, TB - x) plus x high bits.
// Qubits whose stride crosses a 2 MiB page are spread evenly over the passes
// so that no tile touches more than a few dozen pages.
// kmax bounds the qubits rotated by each pass after the first (at most 10, so
// that at least TB - 10 spectator bits give runs of >= 64 bytes).
std::vector<PassPlan> plan_passes(int n, bool c64, int kmax = 10);
// Kernel geometry of a plan entry; returns false if it needs more runs than supported.
bool make_geometry(int n, const PassPlan &pp, Geometry *g);

struct PassArgs {
    void *psi;          // state / phi (in-out)
    void *lam;          // adjoint vector (kTurn: out, kBwd: in-out)
    const void *cost;   // cost diagonal (fp64 for c128, fp32 for c64)
    double *part_e;     // per-block partial sums, indexed by blockIdx.x
    double *part_b;
    double *part_g;
    Geometry geo;
    uint32_t xcd_g;     // 2^xcd_g consecutive tiles go to one XCD (0: hardware order)
    // Mixer rotations in factored form.  exp(-i b X) = f (p I - i q X) with
    // (f, p, q) = (cos b, 1, tan b) when |cos b| >= |sin b| ("tan" mode) and
    // (sin b, cot b, 1) otherwise, so a rotation costs one FMA per component;
    // the factor f^k of the k rotated qubits is applied once per pass.
    uint32_t tan_mode;  // 1: p = 1, mul = q;  0: q = 1, mul = p
    double mul_f;       // forward rotation exp(-i b X): the non-unit coefficient
    double mul_b;       // inverse rotation exp(+i b X)
    double fac_f, fac_b;  // per-rotation factor f (forward, inverse)
    double scl_f, scl_b;  // f^k over the pass's k target qubits
    double gamma_in;    // kPhaseIn multiplies by exp(-i gamma_in C)
    double gamma_out;   // kPhaseOut multiplies by exp(+i gamma_out C)
    double amp0;        // 2^{-n/2}
    int flags;
    // Second rotation of a layer-boundary pass (the other layer's angle), same form.
    uint32_t tan_mode2;
    double mul_f2, mul_b2, fac_b2, scl_f2, scl_b2;
    double *part_b2;    // <lam|X|phi> partials of the second rotation's layer
};

// Tile visited by workgroup L when 2^G consecutive tiles go to each XCD
// (workgroups are dealt to the 8 XCDs in turn): tiles that share cache lines
// and DRAM rows then meet in one XCD's L2.  A permutation of [0, count) when
// 8 * 2^G divides count.
__host__ __device__ inline uint64_t xcd_tile(uint64_t L, uint32_t G)
{
    return G ? ((L & ~((8ull << G) - 1ull)) | ((L & 7ull) << G) | ((L >> 3) & ((1ull << G) - 1ull))) : L;
}
// The largest G <= gmax for which xcd_tile permutes [0, count); 0 if none.
inline uint32_t xcd_group_bits(uint64_t count, uint32_t gmax)
{
    for (uint32_t g = gmax; g >= 1; --g)
        if (count % (8ull << g) == 0) return g;
    return 0;
}

// Launchers; all return the launch status.  `c64` selects complex64/fp32 cost.
hipError_t launch_pass(int mode, bool c64, const PassArgs &a, uint64_t nblocks, hipStream_t s);
// Pass kernels of one precision (R = double: complex128, float: complex64)
// and spectator class SP (passes.hip, one translation unit per pair): SP >= 0
// for full-tile passes that rotate every tile bit from SP up, -1 for the
// kernels that read the target mask at run time.
template <typename R, int SP>
hipError_t launch_pass_sp(int mode, const PassArgs &a, uint64_t nblocks, hipStream_t s);
// Spectator class of a pass with kernels of its own (0 or 2..7), else -1.
int static_spectators(const Geometry &g, bool c64, int mode);
hipError_t launch_sum_slots(const double *parts, uint64_t count, uint64_t stride, int nslots,
                            double *out, hipStream_t s);

// Cost diagonal (Sec. IV-A, Eq. (2)).  The kernel gives each thread 16
// entries: z bits 0-5 are its lane, bits 6-9 the entry index q, and bits >= 10
// are common to a wavefront.  Terms are uploaded as pieces (cost_terms.cpp):
// a piece adds w to entry q of a thread when the wave bits match
// (z & umask) == uval, the lane bits match (lane & lm) == lv, and bit q of
// qpat is set (wq[q] holds w there and -0.0 elsewhere).  The pieces of one
// term cover disjoint sets of z.
constexpr int kCostLaneBits = 6;
constexpr int kCostUniformBit = 10;
struct CostPiece {
    uint64_t umask;  // tested z bits >= 10
    uint64_t uval;   // their required values
    uint32_t lanes;  // bits 0-5: tested lane bits lm; bits 8-13: required values lv
    uint32_t qpat;   // entries q (bit q) covered, from the literals on bits 6-9
    double w;        // the term's weight
    double wq[16];   // per entry q: w if bit q of qpat is set, else -0.0
};
std::vector<CostPiece> cost_pieces_maxcut(int64_t m, const int32_t *edges, const double *w);
std::vector<CostPiece> cost_pieces_qubo(int n, int64_t m, const int32_t *pairs, const double *J,
                                        const double *h);
std::vector<CostPiece> cost_pieces_poly(int64_t L, const uint64_t *masks, const double *w);
// C[z] = offset + the weights of the pieces covering z, in piece order;
// `pieces` is device memory.
hipError_t launch_cost_pieces(bool c64, void *C, int n, const CostPiece *pieces, int64_t count,
                              double offset, hipStream_t s);
hipError_t launch_fill_plus(bool c64, void *psi, int n, hipStream_t s);
hipError_t launch_expect(bool c64, const void *psi, const void *C, int n, double *parts,
                         hipStream_t s);
hipError_t launch_minmax(bool c64, const void *C, int n, double *pmin, double *pmax,
                         hipStream_t s);
hipError_t launch_minmax_final(const double *pmin, const double *pmax, uint64_t count,
                               double *out, hipStream_t s);
hipError_t launch_widen_cost(const float *C32, double *out, uint64_t N, hipStream_t s);

// Sampling: sub-block masses, their exclusive scan, then one thread per shot.
int sample_subblock_bits(int n);
uint64_t scan_scratch_doubles(uint64_t count);
hipError_t launch_submass(bool c64, const void *psi, int n, int sbits, double *sub,
                          hipStream_t s);
hipError_t launch_exclusive_scan(const double *in, uint64_t count, double *out, double *scratch,
                                 hipStream_t s);
hipError_t launch_shots(bool c64, const void *psi, const void *C, int n, int sbits,
                        const double *pre, uint64_t nsub, int64_t shots, uint64_t seed,
                        uint64_t *z, double *cost, hipStream_t s);

// E and the gradient from the summed slots: E = res[0], dbeta[l] = 2 res[1 + l],
// dgamma[l] = 2 res[1 + p + l] (device pointers; E may be NULL).
hipError_t launch_gradient_out(const double *res, int p, double *E, double *dgamma, double *dbeta,
                               hipStream_t s);

// No-allocation gradient (qaoa_gradient_noalloc): the caller supplies device
// scratch for the adjoint vector, the partial sums and the summed slots.
constexpr int kNoAllocMaxLayers = 32;
int handle_device(qaoa_handle h);
size_t noalloc_need(qaoa_handle h, int p);  // bytes of scratch for depth p
// Argument checks (no HIP call), including noalloc_need(h, p) <= cap.
qaoa_status noalloc_check(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                          const double *dgamma, const double *dbeta, size_t cap);
qaoa_status gradient_on_scratch(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                                double *E, double *dgamma, double *dbeta, int32_t out_is_device,
                                void *scratch);

// Message reported by qaoa_last_error_message (thread-local, shared by all calls).
void set_error_message(const std::string &m);
std::string error_message();

}  // namespace qk
