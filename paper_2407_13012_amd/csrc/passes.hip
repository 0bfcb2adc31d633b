// Pass kernels (k_pass, k_pass_fuse, and the tile-pair kernels k_fwd_pair,
// k_init_pair, k_fuse_pair) of one precision and one spectator class.
//
// This file is compiled once per (QK_PASS_REAL, QK_PASS_SP): QK_PASS_REAL is
// double (complex128 tiles) or float (complex64 tiles), QK_PASS_SP the number
// S of spectator tile bits the kernels assume (the S lowest tile bits are not
// rotated, every other tile bit is), or -1 for kernels that read the pass's
// target mask at run time.  With S fixed every rotation stage of the tile code
// is taken or left out at compile time: a stage under a run-time branch leaves
// its results in new registers and the join after it copies them back, about
// a quarter of the VALU work of a two-vector pass.  Such kernels also take the
// pass's access kind (streaming or not) and the phase range as constants; the
// launcher sends passes that disagree to the run-time-mask kernels.  The tile
// code itself (load, phase, rotations, transposes, reductions, stores) is in
// tile_device.h; the kernels and the host launcher of each translation unit
// are its own.
#include "tile_device.h"

#ifndef QK_PASS_REAL
#error "QK_PASS_REAL (double or float) must be defined"
#endif
#ifndef QK_PASS_SP
#error "QK_PASS_SP (spectator class, -1 for the run-time mask) must be defined"
#endif

namespace qk {
namespace {

// Two workgroups per CU (their LDS tiles fill it): 8 waves per CU for
// complex128, 16 for complex64, whose registers are capped accordingly.  The
// one-pass turn (n <= TB) runs a single workgroup and keeps the full register file.
template <typename R, int MODE, bool TM, int SP>
__global__ __launch_bounds__(Tr<R>::NT) __attribute__((amdgpu_waves_per_eu(MODE == kTurnPhase ? 1 : Tr<R>::MINW))) void k_pass(PassArgs a)
{
    __shared__ typename Tr<R>::V lds[kLdsTotal<R>];
    const uint64_t b = blockIdx.x;
    const uint64_t t = xcd_tile(b, a.xcd_g);
    double sums[4];
    tile_pass<R, MODE, TM, TM, SP>(a, t, lds, sums);
    // one partial per workgroup
    if (threadIdx.x == 0) {
        if (MODE == kTurn || MODE == kTurnPhase || (MODE == kFwd && (a.flags & kEOut))) a.part_e[b] = sums[0];
        if (MODE != kFwd) a.part_b[b] = (a.flags & kBetaAcc) ? a.part_b[b] + sums[1] : sums[1];
        if (MODE == kTurnPhase || (MODE == kBwd && (a.flags & kPhaseOut))) a.part_g[b] = sums[2];
    }
}

// Plain forward sweep (no phase, no E, full tiles of spectator class SP), two
// tiles per workgroup: tiles 2i and 2i + 1, which differ in the lowest free
// bit.  With 64-byte runs (4 complex128 or 8 complex64 amplitudes) each run of
// one is the other half of a 128-byte cache line of the other, so one
// workgroup reads whole lines; in every class twice the bytes per workgroup
// are in flight and the two tiles' stages and transposes interleave, as the
// backward sweep does with its two vectors.  Measured at n = 32: 25.2 vs
// 27.2 ms per complex128 sweep, 12.9 vs 14.9 ms per complex64 sweep.
template <typename R, bool TM, int SP>
__global__ __launch_bounds__(Tr<R>::NT) __attribute__((amdgpu_waves_per_eu(Tr<R>::MINW))) void k_fwd_pair(PassArgs a)
{
    using V = typename Tr<R>::V;
    constexpr int WB = Tr<R>::WB, NR = Tr<R>::NR;
    constexpr bool strm = stream_class(SP);
    __shared__ V lds[kLdsTotal<R>];
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const Geometry &g = a.geo;
    const Targets<SP> tg{g.tmask};
    const uint64_t t0 = 2 * xcd_tile(blockIdx.x, a.xcd_g);
    const uint64_t b0 = tile_base(t0, g), b1 = tile_base(t0 + 1, g);
    V *psi = (V *)a.psi;
    V u[NR], w[NR];
    {
        const uint64_t pA = dep(elem<0, WB>(lane, wave, 0), g);
        const RegOffsets<0, WB> off(g);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            u[r] = ld(&psi[b0 | pA | off(r)], strm);
            w[r] = ld(&psi[b1 | pA | off(r)], strm);
        }
    }
    // (measured: with this priority instruction after the loads the complex128
    // sweep takes 25.2 instead of 27.7 ms at n = 32, on every placement tried)
    __builtin_amdgcn_s_setprio(0);
    const R mf = (R)a.mul_f;
    mix_stage<0, TM, true>(u, mf, tg);
    mix_stage<0, TM, true>(w, mf, tg);
    if constexpr (SP >= 4 && WB == 2) {
        // complex128 with no target among B's register bits: A to C directly
        xpose<0, 2>(u, lds, lane, wave);
        xpose<0, 2>(w, lds, lane, wave);
    } else {
        xpose<0, 1>(u, lds, lane, wave);
        xpose<0, 1>(w, lds, lane, wave);
        mix_stage<1, TM, true>(u, mf, tg);
        mix_stage<1, TM, true>(w, mf, tg);
        xpose<1, 2>(u, lds, lane, wave);
        xpose<1, 2>(w, lds, lane, wave);
    }
    mix_stage<2, TM, true>(u, mf, tg);
    mix_stage<2, TM, true>(w, mf, tg);
    const R sf = (R)a.scl_f;
    uint32_t tid2 = threadIdx.x;
    asm volatile("" : "+v"(tid2));
    const uint64_t pC = dep(elem<2, WB>(tid2 & 63u, tid2 >> 6, 0), g);
    const RegOffsets<2, WB> off(g);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        st(vscale(u[r], sf), &psi[b0 | pC | off(r)], strm);
        st(vscale(w[r], sf), &psi[b1 | pC | off(r)], strm);
    }
}

// The first sweep of an evolution (layer 1's phase on the uniform state, then
// its first mixer group: no state is read, the cost entries are), two tiles per
// workgroup: tiles of the first group are runs of 4096 amplitudes, so here the
// pair gains nothing in cache lines, but the two tiles' independent arithmetic
// (sincos of every entry, rotations, transposes) interleaves, as in the
// two-vector sweeps.  The arithmetic per amplitude is tile_pass's for kFwd
// with kInit | kPhaseIn, so results are bitwise the same.  Its runs are long,
// so its accesses are nontemporal (kStream, which the launcher requires).
template <typename R, bool TM>
__global__ __launch_bounds__(Tr<R>::NT) __attribute__((amdgpu_waves_per_eu(Tr<R>::MINW))) void k_init_pair(PassArgs a)
{
    using V = typename Tr<R>::V;
    using CT = typename Tr<R>::CT;
    constexpr int WB = Tr<R>::WB, NR = Tr<R>::NR, SP = 0;
    __shared__ V lds[kLdsTotal<R>];
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const Geometry &g = a.geo;
    const Targets<SP> tg{g.tmask};
    const uint64_t t0 = 2 * xcd_tile(blockIdx.x, a.xcd_g);
    const uint64_t b0 = tile_base(t0, g), b1 = tile_base(t0 + 1, g);
    const CT *cost = (const CT *)a.cost;
    CT cu[NR], cw[NR];
    {
        const uint64_t pA = dep(elem<0, WB>(lane, wave, 0), g);
        const RegOffsets<0, WB> off(g);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cu[r] = ldnt(&cost[b0 | pA | off(r)]);
            cw[r] = ldnt(&cost[b1 | pA | off(r)]);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    const V a0 = {(R)a.amp0, (R)0};
    V u[NR], w[NR];
    {
        // four entries at a time: left to itself the scheduler overlaps all 32
        // evaluations and runs out of registers
        const auto PK = phase_consts<R>(-a.gamma_in);
#pragma unroll
        for (int h = 0; h < NR; h += 4) {
#pragma unroll
            for (int r = h; r < h + 4; ++r) {
                R c, s;
                phase_cs<true>(-a.gamma_in, cu[r], c, s, PK);
                u[r] = cmul(a0, c, s);
                phase_cs<true>(-a.gamma_in, cw[r], c, s, PK);
                w[r] = cmul(a0, c, s);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const R mf = (R)a.mul_f;
    mix_stage<0, TM, true>(u, mf, tg);
    mix_stage<0, TM, true>(w, mf, tg);
    xpose<0, 1>(u, lds, lane, wave);
    xpose<0, 1>(w, lds, lane, wave);
    mix_stage<1, TM, true>(u, mf, tg);
    mix_stage<1, TM, true>(w, mf, tg);
    xpose<1, 2>(u, lds, lane, wave);
    xpose<1, 2>(w, lds, lane, wave);
    mix_stage<2, TM, true>(u, mf, tg);
    mix_stage<2, TM, true>(w, mf, tg);
    const R sf = (R)a.scl_f;
    V *psi = (V *)a.psi;
    uint32_t tid2 = threadIdx.x;
    asm volatile("" : "+v"(tid2));
    const uint64_t pC = dep(elem<2, WB>(tid2 & 63u, tid2 >> 6, 0), g);
    const RegOffsets<2, WB> off(g);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        stnt(vscale(u[r], sf), &psi[b0 | pC | off(r)]);
        stnt(vscale(w[r], sf), &psi[b1 | pC | off(r)]);
    }
}

// Layer-boundary forward sweep (tile_pass_fwd_fuse) in tile pairs: the two
// tiles' rotations of layer l, the phase of layer l + 1 and its rotations,
// interleaved; the arithmetic per amplitude is tile_pass_fwd_fuse's.
template <typename R, bool TM, bool TM2, int SP>
__global__ __launch_bounds__(Tr<R>::NT) __attribute__((amdgpu_waves_per_eu(Tr<R>::MINW))) void k_fuse_pair(PassArgs a)
{
    using V = typename Tr<R>::V;
    using CT = typename Tr<R>::CT;
    constexpr int WB = Tr<R>::WB, NR = Tr<R>::NR;
    constexpr bool strm = stream_class(SP);
    __shared__ V lds[kLdsTotal<R>];
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const Geometry &g = a.geo;
    const Targets<SP> tg{g.tmask};
    const uint64_t t0 = 2 * xcd_tile(blockIdx.x, a.xcd_g);
    const uint64_t b0 = tile_base(t0, g), b1 = tile_base(t0 + 1, g);
    V *psi = (V *)a.psi;
    const CT *cost = (const CT *)a.cost;
    CT cu[NR], cw[NR];
    V u[NR], w[NR];
    {
        const uint64_t pC = dep(elem<2, WB>(lane, wave, 0), g);
        const RegOffsets<2, WB> off(g);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cu[r] = ld(&cost[b0 | pC | off(r)], strm);
            cw[r] = ld(&cost[b1 | pC | off(r)], strm);
        }
    }
    {
        const uint64_t pA = dep(elem<0, WB>(lane, wave, 0), g);
        const RegOffsets<0, WB> off(g);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            u[r] = ld(&psi[b0 | pA | off(r)], strm);
            w[r] = ld(&psi[b1 | pA | off(r)], strm);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    const R m1 = (R)a.mul_f, m2 = (R)a.mul_f2;
    constexpr bool kSkipB = SP >= 4 && WB == 2;
    mix_stage<0, TM, true>(u, m1, tg);
    mix_stage<0, TM, true>(w, m1, tg);
    if constexpr (kSkipB) {
        xpose<0, 2>(u, lds, lane, wave);
        xpose<0, 2>(w, lds, lane, wave);
    } else {
        xpose<0, 1>(u, lds, lane, wave);
        xpose<0, 1>(w, lds, lane, wave);
        mix_stage<1, TM, true>(u, m1, tg);
        mix_stage<1, TM, true>(w, m1, tg);
        xpose<1, 2>(u, lds, lane, wave);
        xpose<1, 2>(w, lds, lane, wave);
    }
    mix_stage<2, TM, true>(u, m1, tg);
    mix_stage<2, TM, true>(w, m1, tg);
    {
        const R s1 = (R)a.scl_f;
        const auto PK = phase_consts<R>(-a.gamma_in);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            R c, s;
            phase_cs<true>(-a.gamma_in, cu[r], c, s, PK);
            u[r] = cmul(vscale(u[r], s1), c, s);
            phase_cs<true>(-a.gamma_in, cw[r], c, s, PK);
            w[r] = cmul(vscale(w[r], s1), c, s);
        }
    }
    mix_stage<2, TM2, true>(u, m2, tg);
    mix_stage<2, TM2, true>(w, m2, tg);
    if constexpr (kSkipB) {
        xpose<2, 0>(u, lds, lane, wave);
        xpose<2, 0>(w, lds, lane, wave);
    } else {
        xpose<2, 1>(u, lds, lane, wave);
        xpose<2, 1>(w, lds, lane, wave);
        mix_stage<1, TM2, true>(u, m2, tg);
        mix_stage<1, TM2, true>(w, m2, tg);
        xpose<1, 0>(u, lds, lane, wave);
        xpose<1, 0>(w, lds, lane, wave);
    }
    mix_stage<0, TM2, true>(u, m2, tg);
    mix_stage<0, TM2, true>(w, m2, tg);
    const R s2 = (R)a.scl_f2;
    uint32_t tid2 = threadIdx.x;
    asm volatile("" : "+v"(tid2));
    const uint64_t pA = dep(elem<0, WB>(tid2 & 63u, tid2 >> 6, 0), g);
    const RegOffsets<0, WB> off(g);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        st(vscale(u[r], s2), &psi[b0 | pA | off(r)], strm);
        st(vscale(w[r], s2), &psi[b1 | pA | off(r)], strm);
    }
}

// Layer-boundary passes (kFwdFuse, kBwdFuse); TM / TM2 are the factored forms
// of the two rotations.  Same tile order and partial layout as k_pass.
template <typename R, int MODE, bool TM, bool TM2, int SP>
__global__ __launch_bounds__(Tr<R>::NT) __attribute__((amdgpu_waves_per_eu(Tr<R>::MINW))) void k_pass_fuse(PassArgs a)
{
    __shared__ typename Tr<R>::V lds[kLdsTotal<R>];
    const uint64_t b = blockIdx.x;
    const uint64_t t = xcd_tile(b, a.xcd_g);
    if constexpr (MODE == kFwdFuse) {
        tile_pass_fwd_fuse<R, TM, TM2, SP>(a, t, lds);
    } else {
        double sums[4];
        tile_pass<R, kBwdFuse, TM, TM2, SP>(a, t, lds, sums);
        if (threadIdx.x == 0) {
            a.part_b[b] = (a.flags & kBetaAcc) ? a.part_b[b] + sums[1] : sums[1];
            a.part_g[b] = sums[2];
            a.part_b2[b] = (a.flags & kBetaAcc2) ? a.part_b2[b] + sums[3] : sums[3];
        }
    }
}

// Arguments of a tile-pair launch: the XCD grouping must divide the number of
// pairs (xcd_tile is a permutation of [0, count) only when 8 * 2^G divides count).
PassArgs pair_args(const PassArgs &a, uint64_t pairs)
{
    PassArgs b = a;
    b.xcd_g = xcd_group_bits(pairs, a.xcd_g);
    return b;
}

template <typename R, bool TM, int SP>
void launch_single(int mode, const PassArgs &a, dim3 grid, hipStream_t s)
{
    const dim3 block(Tr<R>::NT);
    if constexpr (SP == 0) {
        // the first sweep of an evolution in tile pairs (an even number of full tiles)
        if (mode == kFwd && a.flags == (kInit | kPhaseIn | kStream) && a.geo.tbits == (uint32_t)Tr<R>::TB &&
            grid.x % 2 == 0 && grid.x >= 2) {
            hipLaunchKernelGGL((k_init_pair<R, TM>), dim3(grid.x / 2), block, 0, s, pair_args(a, grid.x / 2));
            return;
        }
    }
    // plain forward sweeps in tile pairs (an even number of full tiles): every
    // complex128 class; complex64 only in class 3, whose runs are 64 bytes (at
    // n = 26 its classes 6 and 7 were 2 % slower in pairs, complex128's class 5
    // 1.5 % faster)
    if constexpr (SP >= 0 && (sizeof(R) == 8 || SP == 3)) {
        constexpr int kPlainMask = kInit | kPhaseIn | kEOut | kNoStore;
        if (mode == kFwd && !(a.flags & kPlainMask) && a.geo.tbits == (uint32_t)Tr<R>::TB && grid.x % 2 == 0 &&
            grid.x >= 2) {
            hipLaunchKernelGGL((k_fwd_pair<R, TM, SP>), dim3(grid.x / 2), block, 0, s, pair_args(a, grid.x / 2));
            return;
        }
    }
    if (mode == kFwd) hipLaunchKernelGGL((k_pass<R, kFwd, TM, SP>), grid, block, 0, s, a);
    else if (mode == kTurn) hipLaunchKernelGGL((k_pass<R, kTurn, TM, SP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_pass<R, kBwd, TM, SP>), grid, block, 0, s, a);
}

template <typename R, int MODE, int SP>
void launch_fuse(const PassArgs &a, dim3 grid, hipStream_t s)
{
    const dim3 block(Tr<R>::NT);
    const int sel = (a.tan_mode ? 2 : 0) + (a.tan_mode2 ? 1 : 0);
    if constexpr (MODE == kFwdFuse && SP >= 0) {
        // in tile pairs (an even number of full tiles)
        if (a.geo.tbits == (uint32_t)Tr<R>::TB && grid.x % 2 == 0 && grid.x >= 2) {
            const PassArgs b = pair_args(a, grid.x / 2);
            const dim3 pg(grid.x / 2);
            if (sel == 3) hipLaunchKernelGGL((k_fuse_pair<R, true, true, SP>), pg, block, 0, s, b);
            else if (sel == 2) hipLaunchKernelGGL((k_fuse_pair<R, true, false, SP>), pg, block, 0, s, b);
            else if (sel == 1) hipLaunchKernelGGL((k_fuse_pair<R, false, true, SP>), pg, block, 0, s, b);
            else hipLaunchKernelGGL((k_fuse_pair<R, false, false, SP>), pg, block, 0, s, b);
            return;
        }
    }
    if (sel == 3) hipLaunchKernelGGL((k_pass_fuse<R, MODE, true, true, SP>), grid, block, 0, s, a);
    else if (sel == 2) hipLaunchKernelGGL((k_pass_fuse<R, MODE, true, false, SP>), grid, block, 0, s, a);
    else if (sel == 1) hipLaunchKernelGGL((k_pass_fuse<R, MODE, false, true, SP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_pass_fuse<R, MODE, false, false, SP>), grid, block, 0, s, a);
}

}  // namespace

template <typename R, int SP>
hipError_t launch_pass_sp(int mode, const PassArgs &a, uint64_t nblocks, hipStream_t s)
{
    const dim3 grid((unsigned)nblocks);
    if (mode == kFwdFuse) {
        launch_fuse<R, kFwdFuse, SP>(a, grid, s);
    } else if (mode == kBwdFuse) {
        launch_fuse<R, kBwdFuse, SP>(a, grid, s);
    } else if (mode == kTurnPhase) {
        // the one-pass turn (n <= TB): its tile holds every qubit, no spectators
        if constexpr (SP > 0) return hipErrorInvalidValue;
        else {
            const dim3 block(Tr<R>::NT);
            if (a.tan_mode) hipLaunchKernelGGL((k_pass<R, kTurnPhase, true, SP>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_pass<R, kTurnPhase, false, SP>), grid, block, 0, s, a);
        }
    } else if (a.tan_mode) {
        launch_single<R, true, SP>(mode, a, grid, s);
    } else {
        launch_single<R, false, SP>(mode, a, grid, s);
    }
    return hipGetLastError();
}

template hipError_t launch_pass_sp<QK_PASS_REAL, QK_PASS_SP>(int, const PassArgs &, uint64_t, hipStream_t);

}  // namespace qk
