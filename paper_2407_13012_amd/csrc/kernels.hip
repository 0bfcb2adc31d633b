// gfx950 kernels of the QAOA statevector path.
//
// Streaming pass kernel (k_pass)
//   The mixer U_M(b) = prod_j exp(-i b X_j) is a product of commuting
//   single-qubit rotations (Eq. (1); Sec. IV-B applies them gate by gate).
//   Instead of one full-state sweep per qubit, a pass loads a tile of 2^12
//   amplitudes whose index bits cover a group of qubits, applies every rotation
//   of that group in registers, and writes the tile back once.  A tile is the
//   set of indices with bits [0,S) and [h,h+k) free (S + k = 12); the other
//   n-12 bits are fixed by the workgroup.  Each of the 256 threads holds 16
//   amplitudes; three register arrangements (A, B, C) each put four different
//   tile bits into the register index, and two LDS transposes move between
//   them, so every tile bit is a register bit once.
//     A: lane = bits 0-5,        reg = bits 6-9,         wave = bits 10-11
//     B: reg = bits 0-3,         lane = bits 4-9,        wave = bits 10-11
//     C: lane = bits 0-3,6,7,    reg = bits 4,5,10,11,   wave = bits 8-9
//   Global loads happen in A and stores in C; with S = 2 every access is a
//   64 B run of consecutive amplitudes, with S >= 6 a 1 KiB run.
//
//   The phase layer exp(-i g C) (Sec. IV-B, Euler's formula) is applied to a
//   tile right after loading it in the first pass of a layer, and the
//   expectation sum C|psi|^2 (Sec. IV-D) is accumulated in the last pass, so
//   neither costs a sweep of its own.
//
//   Adjoint gradient (Sec. II-B, IV-C): with lam = C psi, a backward pass loads
//   (phi, lam), adds Im(conj(lam_z) phi_{z^2^j}) for every pair of the group
//   (this is Im <lam|X_j|phi>, unchanged by any mixer factor applied to both),
//   applies exp(+i b X_j) to both, and in the last pass of a layer adds
//   C Im(conj(lam) phi) and undoes the phase.  Layer states are recomputed by
//   these inverse layers; none is stored.  The "turn" pass fuses the last
//   forward group with the first backward group: it evolves psi through the
//   group, forms E and lam = C phi, then undoes the group on lam; phi after
//   the undo is exactly what memory already holds, so it is not written.
//
// Every reduction is a fixed-order tree (shuffle within a wave, then LDS),
// one partial per workgroup, summed by k_sum_slots in fixed order: results are
// bitwise reproducible.
#include "qaoa_internal.h"

#include <math.h>

namespace qk {
namespace {

template <typename R>
struct Tr;
template <>
struct Tr<double> {
    using V = double2;
    using CT = double;
};
template <>
struct Tr<float> {
    using V = float2;
    using CT = float;
};

// Streaming accesses: with long contiguous runs every line is used once per
// pass, so loads and stores may carry the nontemporal hint.  (The builtins take
// clang vector types; values are kept in HIP vector types, which the compiler
// register-allocates far more tightly.)
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldnt(const double2 *p)
{
    const d2v t = __builtin_nontemporal_load((const d2v *)p);
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ float2 ldnt(const float2 *p)
{
    const f2v t = __builtin_nontemporal_load((const f2v *)p);
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ double ldnt(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ldnt(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void stnt(double2 v, double2 *p)
{
    d2v t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, (d2v *)p);
}
__device__ __forceinline__ void stnt(float2 v, float2 *p)
{
    f2v t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, (f2v *)p);
}

// ------------------------------------------------------------ tile geometry

// LDS slot of tile element e: one padding slot after every 16 elements.  In all
// three arrangements any 16 consecutive lanes then hit distinct 16 B bank
// groups, and the slot is additive over the thread part and the register part
// of e, so every access is one base register plus an immediate offset.
constexpr int kLdsSlots = kTile + kTile / 16;
__host__ __device__ __forceinline__ constexpr uint32_t lds_slot(uint32_t e) { return e + (e >> 4); }

template <int ARR>
__host__ __device__ __forceinline__ constexpr uint32_t elem(uint32_t lane, uint32_t wave,
                                                            uint32_t r)
{
    return ARR == 0   ? (lane | (r << 6) | (wave << 10))
           : ARR == 1 ? (r | (lane << 4) | (wave << 10))
                      : ((lane & 15u) | ((r & 3u) << 4) | ((lane >> 4) << 6) | (wave << 8) |
                         ((r >> 2) << 10));
}

// Tile bit held by register-index bit q in arrangement ARR.
template <int ARR>
__host__ __device__ constexpr uint32_t regbit(int q)
{
    return ARR == 0 ? 6 + q : (ARR == 1 ? q : (q < 2 ? 4 + q : 8 + q));
}

// Tile-local index -> offset of the amplitude from the tile base.
__device__ __forceinline__ uint64_t dep(uint32_t e, const Geometry &g)
{
    uint64_t o = 0;
#pragma unroll
    for (int r = 0; r < kTileRuns; ++r)
        o |= (uint64_t)((e >> g.t_src[r]) & ((1u << g.t_len[r]) - 1u)) << g.t_dst[r];
    return o;
}

// Tile index -> base index of the tile (the tile bits set to zero).
__device__ __forceinline__ uint64_t tile_base(uint64_t t, const Geometry &g)
{
    uint64_t o = 0;
#pragma unroll
    for (int r = 0; r < kFreeRuns; ++r)
        o |= ((t >> g.f_src[r]) & ((1ull << g.f_len[r]) - 1ull)) << g.f_dst[r];
    return o;
}

// ------------------------------------------------------------ arithmetic

template <typename V, typename R>
__device__ __forceinline__ V cmul(V v, R c, R s)
{
    V o;
    o.x = v.x * c - v.y * s;
    o.y = v.x * s + v.y * c;
    return o;
}

template <typename V, typename R>
__device__ __forceinline__ V vscale(V v, R f)
{
    V o;
    o.x = v.x * f;
    o.y = v.y * f;
    return o;
}

template <typename V>
__device__ __forceinline__ double norm2(V v)
{
    return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// Im(conj(u) v)
template <typename V>
__device__ __forceinline__ double imcx(V u, V v)
{
    return (double)u.x * (double)v.y - (double)u.y * (double)v.x;
}

// sin and cos of x in fp64.  Cody-Waite reduction x = k pi/2 + r with pi/2
// split into two 33-bit parts and a remainder (k pi/2 is exact for |k| < 2^20),
// then the Taylor series of sin (to r^17) and cos (to r^18) on |r| <= pi/4,
// whose truncation error is below 1e-19.  Larger arguments use the library.
__device__ __forceinline__ void sincos_cw(double x, double &s, double &c)
{
    if (!(fabs(x) < 1.0e6)) {
        sincos(x, &s, &c);
        return;
    }
    const double k = rint(x * 0x1.45f306dc9c883p-1);  // 2/pi
    double r = fma(-k, 0x1.921fb54400000p+0, x);
    r = fma(-k, 0x1.0b4611a600000p-34, r);
    r = fma(-k, 0x1.3198a2e037073p-69, r);
    const double r2 = r * r;
    double ps = 2.8114572543455206e-15;  //  1/17!
    ps = fma(ps, r2, -7.647163731819816e-13);   // -1/15!
    ps = fma(ps, r2, 1.6059043836821613e-10);   //  1/13!
    ps = fma(ps, r2, -2.505210838544172e-08);   // -1/11!
    ps = fma(ps, r2, 2.7557319223985893e-06);   //  1/9!
    ps = fma(ps, r2, -0.0001984126984126984);   // -1/7!
    ps = fma(ps, r2, 0.008333333333333333);     //  1/5!
    ps = fma(ps, r2, -0.16666666666666666);     // -1/3!
    const double sr = fma(ps * r2, r, r);
    double pc = -1.5619206968586225e-16;  // -1/18!
    pc = fma(pc, r2, 4.779477332387385e-14);    //  1/16!
    pc = fma(pc, r2, -1.1470745597729725e-11);  // -1/14!
    pc = fma(pc, r2, 2.08767569878681e-09);     //  1/12!
    pc = fma(pc, r2, -2.755731922398589e-07);   // -1/10!
    pc = fma(pc, r2, 2.48015873015873e-05);     //  1/8!
    pc = fma(pc, r2, -0.001388888888888889);    // -1/6!
    pc = fma(pc, r2, 0.041666666666666664);     //  1/4!
    pc = fma(pc, r2, -0.5);                     // -1/2!
    const double cr = fma(pc, r2, 1.0);
    const int q = (int)(((long long)k) & 3);
    // x = k pi/2 + r: rotate (cos r, sin r) by q quarter turns
    const double s0 = (q & 1) ? cr : sr, c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

// cos / sin of g * C.  complex128: fp64.  complex64: the product is formed and
// reduced modulo 2 pi in fp64, then an fp32 sincos is taken.
__device__ __forceinline__ void phase_cs(double g, double cval, double &c, double &s)
{
    sincos_cw(g * cval, s, c);
}
__device__ __forceinline__ void phase_cs(double g, float cval, float &c, float &s)
{
    const double th = g * (double)cval;
    const double k = rint(th * 0.15915494309189535);
    double r = fma(-k, 6.283185307179586, th);
    r = fma(-k, 2.4492935982947064e-16, r);
    sincosf((float)r, &s, &c);
}

// Factored rotation exp(-i b X) / f on the pair (a, b'):
//   tan mode (TM):  a <- a - i m b',     b' <- b' - i m a
//   cot mode:       a <- m a - i b',     b' <- m b' - i a
// (same formula for the inverse rotation with its own m); one FMA per component.
template <bool TM, typename V, typename R>
__device__ __forceinline__ void bfly(V &a, V &b, R m)
{
    const R ax = a.x, ay = a.y, bx = b.x, by = b.y;
    if constexpr (TM) {
        a.x = fma(m, by, ax);
        a.y = fma(-m, bx, ay);
        b.x = fma(m, ay, bx);
        b.y = fma(-m, ax, by);
    } else {
        a.x = fma(m, ax, by);
        a.y = fma(m, ay, -bx);
        b.x = fma(m, bx, ay);
        b.y = fma(m, by, -ax);
    }
}

template <int ARR, bool TM, typename V, typename R>
__device__ __forceinline__ void mix_stage(V (&v)[16], R m, uint32_t tmask)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if ((tmask >> regbit<ARR>(q)) & 1u) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) bfly<TM>(v[r], v[r | (1 << q)], m);
        }
    }
}

// Adjoint stage: for each target bit, add Im<lam|X_j|phi> over the register
// pairs (weighted by sig2, the squared factor both vectors still miss), then
// apply the factored inverse rotation to both.
template <int ARR, bool TM, typename V, typename R>
__device__ __forceinline__ void adj_stage(V (&f)[16], V (&l)[16], R m, uint32_t tmask,
                                          double &sig2, double f2, double &accB)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if ((tmask >> regbit<ARR>(q)) & 1u) {
            double ps = 0.0;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) {
                    const int r1 = r | (1 << q);
                    ps += imcx(l[r], f[r1]) + imcx(l[r1], f[r]);
                }
            accB = fma(sig2, ps, accB);
            sig2 *= f2;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) {
                    bfly<TM>(l[r], l[r | (1 << q)], m);
                    bfly<TM>(f[r], f[r | (1 << q)], m);
                }
        }
    }
}

// Sum over the target bits owned by arrangement ARR of Im<lam|X_j|phi> on the
// register pairs, times w (the product of the factors both vectors miss).
template <int ARR, typename V>
__device__ __forceinline__ void beta_terms(const V (&f)[16], const V (&l)[16], uint32_t tmask,
                                           double w, double &accB)
{
    double ps = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if ((tmask >> regbit<ARR>(q)) & 1u) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) {
                    const int r1 = r | (1 << q);
                    ps += imcx(l[r], f[r1]) + imcx(l[r1], f[r]);
                }
        }
    }
    accB = fma(w, ps, accB);
}

__host__ __device__ __forceinline__ int popc(uint32_t x) { return __builtin_popcount(x); }

__device__ __forceinline__ double upow(double f, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= f;
    return r;
}

template <int FROM, int TO, typename V>
__device__ __forceinline__ void xpose(V (&v)[16], V *lds, uint32_t lane, uint32_t wave)
{
    V *wr = lds + lds_slot(elem<FROM>(lane, wave, 0));
    V *rd = lds + lds_slot(elem<TO>(lane, wave, 0));
#pragma unroll
    for (int r = 0; r < 16; ++r) wr[lds_slot(elem<FROM>(0, 0, r))] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = rd[lds_slot(elem<TO>(0, 0, r))];
    __syncthreads();
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Sum of `x` over a 256-thread block in fixed order; valid in thread 0.
// `scratch` must hold 4 doubles and not be in use by other threads.
__device__ __forceinline__ double block_sum(double x, double *scratch)
{
    x = wave_sum(x);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((scratch[0] + scratch[1]) + scratch[2]) + scratch[3];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ T ld(const T *p, bool stream)
{
    return stream ? ldnt(p) : *p;
}
template <typename T>
__device__ __forceinline__ void st(T v, T *p, bool stream)
{
    if (stream) stnt(v, p);
    else *p = v;
}

// ------------------------------------------------------------ pass kernel

template <typename R, int MODE, bool TM>
__global__ __launch_bounds__(kThreads) void k_pass(PassArgs a)
{
    using V = typename Tr<R>::V;
    using CT = typename Tr<R>::CT;
    __shared__ V lds[kLdsSlots];

    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t b = blockIdx.x;
    // 2^G consecutive tiles per XCD: workgroups are dealt to the 8 XCDs in turn
    const uint32_t G = a.xcd_g;
    const uint64_t t = G ? ((b & ~((8ull << G) - 1ull)) | ((b & 7ull) << G) | ((b >> 3) & ((1ull << G) - 1ull)))
                         : b;
    const Geometry &g = a.geo;
    const uint64_t base = tile_base(t, g);
    const bool full = g.tbits == (uint32_t)kTileBits;
    const uint32_t lim = 1u << g.tbits;
    const uint32_t tmask = g.tmask;
    const bool strm = (a.flags & kStream) != 0;
    V *psi = (V *)a.psi;
    V *lam = (V *)a.lam;
    const CT *cost = (const CT *)a.cost;

    // Global index of register r in arrangement A / C: a per-thread part plus a
    // part that depends on r only (the same for every thread of the grid).
    const uint64_t thrA = base | dep(elem<0>(lane, wave, 0), g);
    const uint64_t thrC = base | dep(elem<2>(lane, wave, 0), g);
#define ZA(r) (thrA | dep(elem<0>(0, 0, (r)), g))
#define ZC(r) (thrC | dep(elem<2>(0, 0, (r)), g))
#define VA(r) (full || elem<0>(lane, wave, (r)) < lim)
#define VC(r) (full || elem<2>(lane, wave, (r)) < lim)

    double accE = 0.0, accB = 0.0, accG = 0.0;
    const V zero = {(R)0, (R)0};

    // All global loads of the pass are issued up front (cost entries first);
    // loads placed after the arithmetic were found to serialise with it.
    constexpr bool TURN = MODE == kTurn || MODE == kTurnPhase;
    // which optional steps this launch performs (compile-time where the mode decides)
    const bool phaseIn = MODE == kTurnPhase || (MODE == kFwd && (a.flags & kPhaseIn));
    const bool phaseOut = MODE == kTurnPhase || (MODE == kBwd && (a.flags & kPhaseOut));
    const bool costC = TURN || phaseOut || (MODE == kFwd && (a.flags & kEOut));
    CT cin[16], cv[16];
    if (phaseIn) {
#pragma unroll
        for (int r = 0; r < 16; ++r) cin[r] = VA(r) ? ld(&cost[ZA(r)], strm) : (CT)0;
    }
    if (costC) {
#pragma unroll
        for (int r = 0; r < 16; ++r) cv[r] = VC(r) ? ld(&cost[ZC(r)], strm) : (CT)0;
    }

    if constexpr (MODE == kFwd || TURN) {
        V v[16];
        if (a.flags & kInit) {
            const V a0 = {(R)a.amp0, (R)0};
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = VA(r) ? a0 : zero;
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = VA(r) ? ld(&psi[ZA(r)], strm) : zero;
        }
        if (phaseIn) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (VA(r)) {
                    R c, s;
                    phase_cs(-a.gamma_in, cin[r], c, s);
                    v[r] = cmul(v[r], c, s);
                }
        }
        const R mf = (R)a.mul_f;
        mix_stage<0, TM>(v, mf, tmask);
        xpose<0, 1>(v, lds, lane, wave);
        mix_stage<1, TM>(v, mf, tmask);
        xpose<1, 2>(v, lds, lane, wave);
        mix_stage<2, TM>(v, mf, tmask);
        const R sf = (R)a.scl_f;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = vscale(v[r], sf);

        if constexpr (MODE == kFwd) {
            if (a.flags & kEOut) {
#pragma unroll
                for (int r = 0; r < 16; ++r) accE += (double)cv[r] * norm2(v[r]);
            }
            if (!(a.flags & kNoStore)) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (VC(r)) st(v[r], &psi[ZC(r)], strm);
            }
        } else {
            // v is the final state phi on this tile: E, lam = C phi, then undo the
            // group on both, visiting the register arrangements C, B, A; lam is
            // stored from A (from C when the phase is undone too).
            V l[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                accE += (double)cv[r] * norm2(v[r]);
                l[r] = vscale(v[r], (R)cv[r]);
            }
            // Materialise the E sum here: left to the compiler it is sunk to its use
            // after the backward stages, keeping phi and C live (register spills).
            asm volatile("" : "+v"(accE));
            const R mb = (R)a.mul_b;
            const R sb = (R)a.scl_b;
            if constexpr (MODE == kTurn) {
                // <lam|X_j|phi> of an arrangement's bits is taken at its entry, where
                // both vectors sit at the same point.  Arrangement C: the final point.
                // Then undo C's rotations on lam only; phi before stage C is still in
                // LDS from the forward B->C transpose, so it is re-read, not recomputed.
                const int kA = popc(tmask & (15u << 6)), kB = popc(tmask & 15u);
                const int kC = popc(tmask & ((3u << 4) | (3u << 10)));
                const double ff = a.fac_f, fb = a.fac_b;
                beta_terms<2>(v, l, tmask, 1.0, accB);
                mix_stage<2, TM>(l, mb, tmask);
                {
                    const V *rd = lds + lds_slot(elem<1>(lane, wave, 0));
#pragma unroll
                    for (int r = 0; r < 16; ++r) v[r] = rd[lds_slot(elem<1>(0, 0, r))];
                    __syncthreads();
                }
                xpose<2, 1>(l, lds, lane, wave);
                // lam misses fb^kC, phi (forward stages A, B) misses ff^(kA+kB)
                beta_terms<1>(v, l, tmask, upow(fb, kC) * upow(ff, kA + kB), accB);
                mix_stage<1, TM>(l, mb, tmask);
                mix_stage<1, TM>(v, mb, tmask);
                xpose<1, 0>(v, lds, lane, wave);
                xpose<1, 0>(l, lds, lane, wave);
                beta_terms<0>(v, l, tmask, upow(fb, kC + 2 * kB) * upow(ff, kA + kB), accB);
                mix_stage<0, TM>(l, mb, tmask);
                if (!(a.flags & kNoStore)) {
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (VA(r)) st(vscale(l[r], sb), &lam[ZA(r)], strm);
                }
            } else {
            const double f2 = a.fac_b * a.fac_b;
            double sig2 = 1.0;
            adj_stage<2, TM>(v, l, mb, tmask, sig2, f2, accB);
            xpose<2, 1>(v, lds, lane, wave);
            xpose<2, 1>(l, lds, lane, wave);
            adj_stage<1, TM>(v, l, mb, tmask, sig2, f2, accB);
            xpose<1, 0>(v, lds, lane, wave);
            xpose<1, 0>(l, lds, lane, wave);
            adj_stage<0, TM>(v, l, mb, tmask, sig2, f2, accB);
                xpose<0, 2>(l, lds, lane, wave);
                xpose<0, 2>(v, lds, lane, wave);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    l[r] = vscale(l[r], sb);
                    if (VC(r)) {
                        accG += (double)cv[r] * imcx(l[r], vscale(v[r], sb));
                        R c, s;
                        phase_cs(a.gamma_out, cv[r], c, s);
                        l[r] = cmul(l[r], c, s);
                    }
                }
                if (!(a.flags & kNoStore)) {
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (VC(r)) st(l[r], &lam[ZC(r)], strm);
                }
            }
        }
    } else {
        V f[16], l[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const bool ok = VA(r);
            f[r] = ok ? ld(&psi[ZA(r)], strm) : zero;
            l[r] = ok ? ld(&lam[ZA(r)], strm) : zero;
        }
        const R mb = (R)a.mul_b;
        const double f2 = a.fac_b * a.fac_b;
        double sig2 = 1.0;
        adj_stage<0, TM>(f, l, mb, tmask, sig2, f2, accB);
        xpose<0, 1>(f, lds, lane, wave);
        xpose<0, 1>(l, lds, lane, wave);
        adj_stage<1, TM>(f, l, mb, tmask, sig2, f2, accB);
        xpose<1, 2>(f, lds, lane, wave);
        xpose<1, 2>(l, lds, lane, wave);
        adj_stage<2, TM>(f, l, mb, tmask, sig2, f2, accB);
        const R sb = (R)a.scl_b;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            f[r] = vscale(f[r], sb);
            l[r] = vscale(l[r], sb);
        }
        if (phaseOut) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (VC(r)) {
                    accG += (double)cv[r] * imcx(l[r], f[r]);
                    R c, s;
                    phase_cs(a.gamma_out, cv[r], c, s);
                    f[r] = cmul(f[r], c, s);
                    l[r] = cmul(l[r], c, s);
                }
        }
        if (!(a.flags & kNoStore)) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (VC(r)) {
                    st(f[r], &psi[ZC(r)], strm);
                    st(l[r], &lam[ZC(r)], strm);
                }
        }
    }
#undef ZA
#undef ZC
#undef VA
#undef VC

    // Fixed-order block reductions; one partial per workgroup.
    double *red = (double *)lds;  // every LDS read above completed before the last barrier
    const bool wantE = TURN || (MODE == kFwd && (a.flags & kEOut));
    const bool wantB = MODE != kFwd;
    const bool wantG = phaseOut;
    if (wantE) {
        const double s = block_sum(accE, red);
        if (tid == 0) a.part_e[b] = s;
    }
    if (wantB) {
        const double s = block_sum(accB, red);
        if (tid == 0) a.part_b[b] = (a.flags & kBetaAcc) ? a.part_b[b] + s : s;
    }
    if (wantG) {
        const double s = block_sum(accG, red);
        if (tid == 0) a.part_g[b] = s;
    }
}

// ------------------------------------------------------------ reductions

// out[k] = sum_{i < count} parts[k * stride + i], one workgroup per slot, fixed order.
__global__ __launch_bounds__(kThreads) void k_sum_slots(const double *parts, uint64_t count,
                                                        uint64_t stride, double *out)
{
    __shared__ double red[4];
    const double *p = parts + (uint64_t)blockIdx.x * stride;
    double acc = 0.0;
    for (uint64_t i = threadIdx.x; i < count; i += kThreads) acc += p[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Expectation of a stored state: one partial per 4096 amplitudes.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect(const typename Tr<R>::V *psi,
                                                     const typename Tr<R>::CT *C, uint64_t N,
                                                     double *parts)
{
    __shared__ double red[4];
    const uint64_t b0 = (uint64_t)blockIdx.x * kTile;
    double acc = 0.0;
#pragma unroll 4
    for (int r = 0; r < kTile / kThreads; ++r) {
        const uint64_t z = b0 + (uint64_t)r * kThreads + threadIdx.x;
        if (z < N) acc += (double)C[z] * norm2(psi[z]);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

template <typename CT>
__global__ __launch_bounds__(kThreads) void k_minmax(const CT *C, uint64_t N, double *pmin,
                                                     double *pmax)
{
    __shared__ double red[2][kThreads];
    const uint64_t b0 = (uint64_t)blockIdx.x * kTile;
    double lo = INFINITY, hi = -INFINITY;
    for (int r = 0; r < kTile / kThreads; ++r) {
        const uint64_t z = b0 + (uint64_t)r * kThreads + threadIdx.x;
        if (z < N) {
            const double v = (double)C[z];
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
    red[0][threadIdx.x] = lo;
    red[1][threadIdx.x] = hi;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmin[blockIdx.x] = red[0][0];
        pmax[blockIdx.x] = red[1][0];
    }
}

__global__ __launch_bounds__(kThreads) void k_minmax_final(const double *pmin, const double *pmax,
                                                           uint64_t count, double *out)
{
    __shared__ double red[2][kThreads];
    double lo = INFINITY, hi = -INFINITY;
    for (uint64_t i = threadIdx.x; i < count; i += kThreads) {
        lo = fmin(lo, pmin[i]);
        hi = fmax(hi, pmax[i]);
    }
    red[0][threadIdx.x] = lo;
    red[1][threadIdx.x] = hi;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

// ------------------------------------------------------------ cost diagonal

// C[z] = sum over cut edges of w_k, in edge order (Sec. IV-A; MaxCut term = x_i XOR x_j).
template <typename CT>
__global__ __launch_bounds__(kThreads) void k_cost_maxcut(CT *C, uint64_t N, int64_t m,
                                                          const int32_t *edges, const double *w)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t z = (uint64_t)blockIdx.x * kThreads + threadIdx.x; z < N; z += stride) {
        double acc = 0.0;
        for (int64_t k = 0; k < m; ++k) {
            const int i = edges[2 * k], j = edges[2 * k + 1];
            const double wk = w ? w[k] : 1.0;
            const bool cut = ((z >> i) ^ (z >> j)) & 1ull;
            acc = cut ? acc + wk : acc;
        }
        C[z] = (CT)acc;
    }
}

// C[z] = offset + sum_k J_k x_i x_j + sum_i h_i x_i in that order (Eq. (2), degree <= 2).
template <typename CT>
__global__ __launch_bounds__(kThreads) void k_cost_qubo(CT *C, uint64_t N, int n, int64_t m,
                                                        const int32_t *pairs, const double *J,
                                                        const double *h, double offset)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t z = (uint64_t)blockIdx.x * kThreads + threadIdx.x; z < N; z += stride) {
        double acc = offset;
        for (int64_t k = 0; k < m; ++k) {
            const int i = pairs[2 * k], j = pairs[2 * k + 1];
            const bool on = ((z >> i) & (z >> j)) & 1ull;
            acc = on ? acc + J[k] : acc;
        }
        if (h)
            for (int i = 0; i < n; ++i) {
                const bool on = (z >> i) & 1ull;
                acc = on ? acc + h[i] : acc;
            }
        C[z] = (CT)acc;
    }
}

// General 0-1 polynomial of Eq. (2): term k (mask m_k, weight w_k) is active in
// z iff every variable of its mask is 1, (z AND m_k) == m_k; terms are added in
// the given order after the offset.
template <typename CT>
__global__ __launch_bounds__(kThreads) void k_cost_poly(CT *C, uint64_t N, int64_t L,
                                                        const uint64_t *masks, const double *w,
                                                        double offset)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t z = (uint64_t)blockIdx.x * kThreads + threadIdx.x; z < N; z += stride) {
        double acc = offset;
        for (int64_t k = 0; k < L; ++k) {
            const uint64_t m = masks[k];
            acc = ((z & m) == m) ? acc + w[k] : acc;
        }
        C[z] = (CT)acc;
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_fill_plus(typename Tr<R>::V *psi, uint64_t N, R amp)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t z = (uint64_t)blockIdx.x * kThreads + threadIdx.x; z < N; z += stride) {
        typename Tr<R>::V v;
        v.x = amp;
        v.y = (R)0;
        psi[z] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_widen(const float *C32, double *out, uint64_t N)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t z = (uint64_t)blockIdx.x * kThreads + threadIdx.x; z < N; z += stride)
        out[z] = (double)C32[z];
}

// ------------------------------------------------------------ sampling

// Philox-4x32-10 (Salmon et al., SC'11): ten rounds of the two 32x32->64
// multiplies with M0 = 0xD2511F53 and M1 = 0xCD9E8D57, key bumped by the Weyl
// constants 0x9E3779B9 / 0xBB67AE85 between rounds.
__device__ __forceinline__ double philox_uniform53(uint64_t seed, uint64_t s)
{
    uint32_t x0 = (uint32_t)s, x1 = (uint32_t)(s >> 32), x2 = 0u, x3 = 0u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    const uint64_t w = ((uint64_t)x1 << 32) | x0;
    return (double)(w >> 11) * 0x1.0p-53;
}

// Mass of each sub-block of 2^sbits amplitudes: one wave per sub-block, each
// lane sums a fixed set of elements in order, then a shuffle tree.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_submass(const typename Tr<R>::V *psi, uint64_t N,
                                                      int sbits, uint64_t nsub, double *sub)
{
    const uint64_t j = (uint64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (j >= nsub) return;  // whole wave exits together
    const uint64_t sb = 1ull << sbits, z0 = j << sbits;
    double acc = 0.0;
    for (uint64_t i = lane; i < sb; i += 64) {
        const uint64_t z = z0 + i;
        if (z < N) acc += norm2(psi[z]);
    }
    acc = wave_sum(acc);
    if (lane == 0) sub[j] = acc;
}

constexpr int kScanChunk = kThreads * 16;  // entries per workgroup in the scan

// Per-chunk totals.
__global__ __launch_bounds__(kThreads) void k_scan_partial(const double *in, uint64_t count,
                                                           double *tot)
{
    __shared__ double red[4];
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk;
    double acc = 0.0;
    for (int r = 0; r < 16; ++r) {
        const uint64_t i = c0 + (uint64_t)threadIdx.x * 16 + r;
        if (i < count) acc += in[i];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) tot[blockIdx.x] = s;
}

// Exclusive scan of `x` across the 256 threads of a block (thread-ordered);
// returns the exclusive prefix for this thread and the block total in *total.
__device__ __forceinline__ double block_exclusive(double x, double *sh, double *total)
{
    sh[threadIdx.x] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int i = 0; i < kThreads; ++i) {
            const double v = sh[i];
            sh[i] = run;
            run += v;
        }
        sh[kThreads] = run;
    }
    __syncthreads();
    const double r = sh[threadIdx.x];
    *total = sh[kThreads];
    __syncthreads();
    return r;
}

// Exclusive scan of the chunk totals (at most kScanChunk of them) in place;
// tot[nchunks] receives the grand total.
__global__ __launch_bounds__(kThreads) void k_scan_top(double *tot, uint64_t nchunks)
{
    __shared__ double sh[kThreads + 1];
    double v[16];
    double local = 0.0;
    for (int r = 0; r < 16; ++r) {
        const uint64_t i = (uint64_t)threadIdx.x * 16 + r;
        v[r] = i < nchunks ? tot[i] : 0.0;
        local += v[r];
    }
    double total;
    double run = block_exclusive(local, sh, &total);
    for (int r = 0; r < 16; ++r) {
        const uint64_t i = (uint64_t)threadIdx.x * 16 + r;
        if (i < nchunks) tot[i] = run;
        run += v[r];
    }
    if (threadIdx.x == 0) tot[nchunks] = total;
}

// out[i] = sum_{k < i} in[k] for i <= count (out[count] = total).
__global__ __launch_bounds__(kThreads) void k_scan_final(const double *in, uint64_t count,
                                                         const double *tot, uint64_t nchunks,
                                                         double *out)
{
    __shared__ double sh[kThreads + 1];
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk;
    double v[16];
    double local = 0.0;
    for (int r = 0; r < 16; ++r) {
        const uint64_t i = c0 + (uint64_t)threadIdx.x * 16 + r;
        v[r] = i < count ? in[i] : 0.0;
        local += v[r];
    }
    double total;
    double run = tot[blockIdx.x] + block_exclusive(local, sh, &total);
    for (int r = 0; r < 16; ++r) {
        const uint64_t i = c0 + (uint64_t)threadIdx.x * 16 + r;
        if (i < count) out[i] = run;
        run += v[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[count] = tot[nchunks];
}

// One thread per shot: u -> target t = u * total, binary search over the
// sub-block prefix, then a sequential scan inside the sub-block for the first
// z whose cumulative mass exceeds t.  A zero-probability z never satisfies the
// test (its cumulative mass equals its predecessor's), so it is never returned.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_shots(const typename Tr<R>::V *psi,
                                                    const typename Tr<R>::CT *C, uint64_t N,
                                                    int sbits, const double *pre, uint64_t nsub,
                                                    int64_t shots, uint64_t seed, uint64_t *zout,
                                                    double *cout)
{
    const uint64_t s = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= (uint64_t)shots) return;
    const double T = pre[nsub];
    const double t = philox_uniform53(seed, s) * T;
    uint64_t lo = 0, hi = nsub - 1;  // smallest j with pre[j+1] > t
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (pre[mid + 1] > t) hi = mid;
        else lo = mid + 1;
    }
    const uint64_t z0 = lo << sbits;
    const uint64_t zend = min(N, z0 + (1ull << sbits));
    double acc = pre[lo];
    uint64_t zsel = ~0ull, zlast = z0;
    for (uint64_t z = z0; z < zend; ++z) {
        const double pz = norm2(psi[z]);
        if (pz > 0.0) zlast = z;
        acc += pz;
        if (acc > t) {
            zsel = z;
            break;
        }
    }
    if (zsel == ~0ull) zsel = zlast;  // rounding left t at the sub-block's end
    zout[s] = zsel;
    if (cout) cout[s] = (double)C[zsel];
}

inline unsigned grid_for(uint64_t N, uint64_t cap = 1ull << 20)
{
    uint64_t g = (N + kThreads - 1) / kThreads;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (unsigned)g;
}

}  // namespace

// ------------------------------------------------------------ launchers

template <typename R, bool TM>
static void launch_pass_t(int mode, const PassArgs &a, dim3 grid, hipStream_t s)
{
    if (mode == kFwd) hipLaunchKernelGGL((k_pass<R, kFwd, TM>), grid, dim3(kThreads), 0, s, a);
    else if (mode == kTurn) hipLaunchKernelGGL((k_pass<R, kTurn, TM>), grid, dim3(kThreads), 0, s, a);
    else if (mode == kTurnPhase)
        hipLaunchKernelGGL((k_pass<R, kTurnPhase, TM>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((k_pass<R, kBwd, TM>), grid, dim3(kThreads), 0, s, a);
}

hipError_t launch_pass(int mode, bool c64, const PassArgs &a, uint64_t nblocks, hipStream_t s)
{
    const dim3 grid((unsigned)nblocks);
    if (!c64) {
        if (a.tan_mode) launch_pass_t<double, true>(mode, a, grid, s);
        else launch_pass_t<double, false>(mode, a, grid, s);
    } else {
        if (a.tan_mode) launch_pass_t<float, true>(mode, a, grid, s);
        else launch_pass_t<float, false>(mode, a, grid, s);
    }
    return hipGetLastError();
}

hipError_t launch_sum_slots(const double *parts, uint64_t count, uint64_t stride, int nslots,
                            double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_slots, dim3(nslots), dim3(kThreads), 0, s, parts, count, stride, out);
    return hipGetLastError();
}

hipError_t launch_cost_maxcut(bool c64, void *C, int n, int64_t m, const int32_t *edges,
                              const double *w, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (c64)
        hipLaunchKernelGGL(k_cost_maxcut<float>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (float *)C, N, m, edges, w);
    else
        hipLaunchKernelGGL(k_cost_maxcut<double>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (double *)C, N, m, edges, w);
    return hipGetLastError();
}

hipError_t launch_cost_qubo(bool c64, void *C, int n, int64_t m, const int32_t *pairs,
                            const double *J, const double *h, double offset, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (c64)
        hipLaunchKernelGGL(k_cost_qubo<float>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (float *)C, N, n, m, pairs, J, h, offset);
    else
        hipLaunchKernelGGL(k_cost_qubo<double>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (double *)C, N, n, m, pairs, J, h, offset);
    return hipGetLastError();
}

hipError_t launch_cost_poly(bool c64, void *C, int n, int64_t L, const uint64_t *masks,
                            const double *w, double offset, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (c64)
        hipLaunchKernelGGL(k_cost_poly<float>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (float *)C, N, L, masks, w, offset);
    else
        hipLaunchKernelGGL(k_cost_poly<double>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (double *)C, N, L, masks, w, offset);
    return hipGetLastError();
}

hipError_t launch_fill_plus(bool c64, void *psi, int n, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    const double amp = 1.0 / sqrt((double)N);
    if (c64)
        hipLaunchKernelGGL(k_fill_plus<float>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (Tr<float>::V *)psi, N, (float)amp);
    else
        hipLaunchKernelGGL(k_fill_plus<double>, dim3(grid_for(N)), dim3(kThreads), 0, s,
                           (Tr<double>::V *)psi, N, amp);
    return hipGetLastError();
}

hipError_t launch_expect(bool c64, const void *psi, const void *C, int n, double *parts,
                         hipStream_t s)
{
    const uint64_t N = 1ull << n;
    const unsigned nb = (unsigned)((N + kTile - 1) / kTile);
    if (c64)
        hipLaunchKernelGGL(k_expect<float>, dim3(nb), dim3(kThreads), 0, s, (const Tr<float>::V *)psi,
                           (const float *)C, N, parts);
    else
        hipLaunchKernelGGL(k_expect<double>, dim3(nb), dim3(kThreads), 0, s,
                           (const Tr<double>::V *)psi, (const double *)C, N, parts);
    return hipGetLastError();
}

hipError_t launch_minmax(bool c64, const void *C, int n, double *pmin, double *pmax,
                         hipStream_t s)
{
    const uint64_t N = 1ull << n;
    const unsigned nb = (unsigned)((N + kTile - 1) / kTile);
    if (c64)
        hipLaunchKernelGGL(k_minmax<float>, dim3(nb), dim3(kThreads), 0, s, (const float *)C, N,
                           pmin, pmax);
    else
        hipLaunchKernelGGL(k_minmax<double>, dim3(nb), dim3(kThreads), 0, s, (const double *)C,
                           N, pmin, pmax);
    return hipGetLastError();
}

hipError_t launch_minmax_final(const double *pmin, const double *pmax, uint64_t count,
                               double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(kThreads), 0, s, pmin, pmax, count, out);
    return hipGetLastError();
}

hipError_t launch_widen_cost(const float *C32, double *out, uint64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_widen, dim3(grid_for(N)), dim3(kThreads), 0, s, C32, out, N);
    return hipGetLastError();
}

int sample_subblock_bits(int n)
{
    int sb = n - 24 > 8 ? n - 24 : 8;
    return sb < n ? sb : n;
}

uint64_t scan_scratch_doubles(uint64_t count)
{
    return (count + kScanChunk - 1) / kScanChunk + 1;
}

hipError_t launch_submass(bool c64, const void *psi, int n, int sbits, double *sub,
                          hipStream_t s)
{
    const uint64_t N = 1ull << n, nsub = 1ull << (n - sbits);
    const unsigned nb = (unsigned)((nsub + 3) / 4);
    if (c64)
        hipLaunchKernelGGL(k_submass<float>, dim3(nb), dim3(kThreads), 0, s, (const Tr<float>::V *)psi,
                           N, sbits, nsub, sub);
    else
        hipLaunchKernelGGL(k_submass<double>, dim3(nb), dim3(kThreads), 0, s,
                           (const Tr<double>::V *)psi, N, sbits, nsub, sub);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const double *in, uint64_t count, double *out, double *scratch,
                                 hipStream_t s)
{
    const uint64_t nchunks = (count + kScanChunk - 1) / kScanChunk;
    if (nchunks > (uint64_t)kScanChunk) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)nchunks), dim3(kThreads), 0, s, in, count,
                       scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, scratch, nchunks);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nchunks), dim3(kThreads), 0, s, in, count,
                       scratch, nchunks, out);
    return hipGetLastError();
}

hipError_t launch_shots(bool c64, const void *psi, const void *C, int n, int sbits,
                        const double *pre, uint64_t nsub, int64_t shots, uint64_t seed,
                        uint64_t *z, double *cost, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    const unsigned nb = (unsigned)(((uint64_t)shots + kThreads - 1) / kThreads);
    if (c64)
        hipLaunchKernelGGL(k_shots<float>, dim3(nb), dim3(kThreads), 0, s, (const Tr<float>::V *)psi,
                           (const float *)C, N, sbits, pre, nsub, shots, seed, z, cost);
    else
        hipLaunchKernelGGL(k_shots<double>, dim3(nb), dim3(kThreads), 0, s,
                           (const Tr<double>::V *)psi, (const double *)C, N, sbits, pre, nsub, shots,
                           seed, z, cost);
    return hipGetLastError();
}

}  // namespace qk
