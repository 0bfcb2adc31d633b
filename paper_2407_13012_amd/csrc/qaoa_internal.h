// Internal interface between the C-ABI layer (api.cpp) and the gfx950 kernels
// (kernels.hip).  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qk {

// Tile geometry of the streaming pass kernel: one workgroup owns 2^12
// amplitudes, 256 threads x 16 amplitudes in registers.
constexpr int kTileBits = 12;
constexpr int kTile = 1 << kTileBits;
constexpr int kThreads = 256;

// Pass modes.
enum PassMode : int {
    kFwd = 0,   // one vector: [init|load] [phase] mixer [E] store
    kTurn = 1,  // last forward group fused with the first backward group
    kBwd = 2    // two vectors: mixer^dag with <lam|X_j|phi>, [phase^dag with <lam|C|phi>]
};

// Pass flags.
enum PassFlags : int {
    kInit = 1,       // generate |+> instead of loading the state
    kPhaseIn = 2,    // multiply by exp(-i gamma_in C) before the mixer group
    kEOut = 4,       // accumulate sum C |psi|^2 (kFwd after the mixer; always in kTurn)
    kPhaseOut = 8,   // (kBwd, kTurn) accumulate Im <lam|C|phi>, then multiply both by exp(+i gamma_out C)
    kNoStore = 16,   // skip the final store (last backward pass)
    kBetaAcc = 32    // add the <lam|X|phi> partial to the existing one instead of overwriting
};

// A mixer group: tile bits are [0, S) (spectators or targets) and [h, h+k);
// S + k = 12 for n >= 12.  Targets are the tile bits >= S and < tbits.
struct Group {
    int S, h, k;
};

struct PassArgs {
    void *psi;          // state / phi (in-out)
    void *lam;          // adjoint vector (kTurn: out, kBwd: in-out)
    const void *cost;   // cost diagonal (fp64 for c128, fp32 for c64)
    double *part_e;     // per-block partial sums, indexed by blockIdx.x
    double *part_b;
    double *part_g;
    uint32_t S, h;      // group geometry
    uint32_t ta_bits;   // h - S: tile-index bits placed at [S, h)
    uint32_t tb_shift;  // h + k: remaining tile-index bits placed from here
    uint32_t tbits;     // number of valid tile bits (12, or n when n < 12)
    uint32_t xcd_remap; // map consecutive tiles to one XCD (needs #tiles % 32 == 0)
    double cm, sm;      // mixer: cos(beta), sin(beta) of exp(-i beta X) (kFwd, kTurn forward)
    double cu, su;      // mixer^dag coefficients: cos(beta), -sin(beta) (kBwd, kTurn backward)
    double gamma_in;    // kPhaseIn multiplies by exp(-i gamma_in C)
    double gamma_out;   // kPhaseOut multiplies by exp(+i gamma_out C)
    double amp0;        // 2^{-n/2}
    int flags;
};

// Launchers; all return the launch status.  `c64` selects complex64/fp32 cost.
hipError_t launch_pass(int mode, bool c64, const PassArgs &a, uint64_t nblocks, hipStream_t s);
hipError_t launch_sum_slots(const double *parts, uint64_t count, uint64_t stride, int nslots,
                            double *out, hipStream_t s);
hipError_t launch_cost_maxcut(bool c64, void *C, int n, int64_t m, const int32_t *edges,
                              const double *w, hipStream_t s);
hipError_t launch_cost_qubo(bool c64, void *C, int n, int64_t m, const int32_t *pairs,
                            const double *J, const double *h, double offset, hipStream_t s);
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

}  // namespace qk
