// Device-side building blocks of the tiled pass, shared by the per-pass
// kernels (kernels.hip) and the batched engine (batch.hip).  Included by each
// translation unit; everything here has internal linkage.
#pragma once
#include "qaoa_internal.h"

#include <math.h>

#include <type_traits>

namespace qk {
namespace {

template <typename R>
struct Tr;
// Amplitude type, cost-entry type and tile shape per precision: 2^TB
// amplitudes per workgroup of NT = 2^(TB-4) threads (NW = 2^WB waves of 64),
// NR = 16 amplitudes per thread.
template <>
struct Tr<double> {
    using V = double2;
    using CT = double;
    static constexpr int TB = kTileBits;
    static constexpr int WB = TB - 10;
    static constexpr int NW = 1 << WB;
    static constexpr int NT = 64 * NW;
    static constexpr int NR = 16;
    static constexpr int MINW = 2;  // waves per SIMD the pass kernels must allow (two workgroups per CU)
};
template <>
struct Tr<float> {
    using V = float2;
    using CT = float;
    static constexpr int TB = kTileBits64;
    static constexpr int WB = TB - 10;
    static constexpr int NW = 1 << WB;
    static constexpr int NT = 64 * NW;
    static constexpr int NR = 16;
    static constexpr int MINW = 4;
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

// LDS slot of tile element e: one padding slot after every 16 elements, and 8
// more before the upper half of a 13-bit tile.  In all three arrangements any
// 16 consecutive lanes then hit distinct banks, and the slot is additive over
// the thread part and the register part of e, so every access is one base
// register plus an immediate offset.
template <typename R>
constexpr int kLdsSlots = (1 << Tr<R>::TB) + (1 << Tr<R>::TB) / 16 + 8 * ((1 << Tr<R>::TB) >> 13);
// The workgroup's LDS: the padded transpose slots plus room for the per-wave
// partial sums of the block reduction (4 values x NW waves of doubles).
template <typename R>
constexpr int kLdsTotal = kLdsSlots<R> + (int)(4 * Tr<R>::NW * sizeof(double) / sizeof(typename Tr<R>::V));
template <int WB>
__host__ __device__ __forceinline__ constexpr uint32_t lds_slot(uint32_t e)
{
    return e + (e >> 4) + (WB == 3 ? ((e >> 12) << 3) : 0u);
}

// Register arrangements of a tile of 2^(10+WB) elements (lane: 6 bits,
// register index: 4 bits, wave: WB = 2 or 3 bits).  With WB = 2:
//   A: lane = bits 0-5,      reg = bits 6-9,         wave = bits 10-11
//   B: reg = bits 0-3,       lane = bits 4-9,        wave = bits 10-11
//   C: lane = bits 0-3,6,7,  reg = bits 4,5,10,11,   wave = bits 8-9
// With WB = 3 the extra tile bit 12 is the top wave bit in A and C, and lane
// bit 1 in B (where the lanes hold bits 4, 12, 5-8 and the waves bits 9-11):
// it is never a register bit, and its rotation pairs lanes l and l ^ 2 in B,
// which a DPP quad permutation reaches without LDS traffic.
template <int ARR, int WB>
__host__ __device__ __forceinline__ constexpr uint32_t elem(uint32_t lane, uint32_t wave,
                                                            uint32_t r)
{
    return ARR == 0   ? (lane | (r << 6) | (wave << 10))
           : ARR == 1 ? (WB == 2 ? (r | (lane << 4) | (wave << 10))
                                 : (r | ((lane & 1u) << 4) | (((lane >> 1) & 1u) << 12) | ((lane >> 2) << 5) |
                                    (wave << 9)))
           : WB == 2 ? ((lane & 15u) | ((r & 3u) << 4) | ((lane >> 4) << 6) | (wave << 8) | ((r >> 2) << 10))
                     : ((lane & 15u) | ((r & 3u) << 4) | ((lane >> 4) << 6) | ((wave & 3u) << 8) |
                        ((r >> 2) << 10) | ((wave >> 2) << 12));
}

// Tile bit held by register-index bit q in arrangement ARR.
template <int ARR>
__host__ __device__ constexpr uint32_t regbit(int q)
{
    return ARR == 0 ? 6 + q : (ARR == 1 ? q : (q < 2 ? 4 + q : 8 + q));
}

// Tile bits rotated while the tile is in arrangement ARR (each tile bit once):
// the register bits, plus in B the lane-held bit 12 of 13-bit tiles.
template <int ARR, int WB>
__host__ __device__ constexpr uint32_t owned()
{
    return ARR == 0 ? (15u << 6) : ARR == 1 ? (15u | (WB == 3 ? 1u << 12 : 0u)) : ((3u << 4) | (3u << 10));
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

// Offset of register r in arrangement ARR (the part of an amplitude's global
// index that depends on r only).  dep() sends each tile bit to one global
// bit, and the register index occupies its own tile bits, so the offset of r
// is the OR of the offsets of its set bits: four dep() evaluations per
// arrangement instead of one per register.
template <int ARR, int WB>
struct RegOffsets {
    uint64_t b[4];
    __device__ __forceinline__ explicit RegOffsets(const Geometry &g)
    {
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = dep(elem<ARR, WB>(0, 0, 1u << q), g);
    }
    __device__ __forceinline__ uint64_t operator()(int r) const
    {
        return ((r & 1) ? b[0] : 0ull) | ((r & 2) ? b[1] : 0ull) | ((r & 4) ? b[2] : 0ull) |
               ((r & 8) ? b[3] : 0ull);
    }
};

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
// acc + Im(conj(u) v) as two chained FMAs.
template <typename V>
__device__ __forceinline__ double imcx_acc(V u, V v, double acc)
{
    return fma(-(double)u.y, (double)v.x, fma((double)u.x, (double)v.y, acc));
}
// complex64: the products of one target bit's 16 register pairs (or 16 lane
// pairs) are summed in fp32, as accurate as the amplitudes themselves, and
// each such partial sum is then accumulated in fp64.
__device__ __forceinline__ float imcx_acc(float2 u, float2 v, float acc)
{
    return fmaf(-u.y, v.x, fmaf(u.x, v.y, acc));
}
template <typename V>
struct PairSum {
    using T = double;
};
template <>
struct PairSum<float2> {
    using T = float;
};

// sin and cos of x in fp64.  Cody-Waite reduction x = k pi/2 + r with pi/2
// split into two 33-bit parts and a remainder (k pi/2 is exact for |k| < 2^20),
// then the Taylor series of sin (to r^17) and cos (to r^18) on |r| <= pi/4,
// whose truncation error is below 1e-19.  Larger arguments use the library.
//
// The fp64 constants are held in scalar registers for a whole loop over a
// thread's amplitudes (PhaseK, built once per loop by phase_consts()): an fp64
// operand that is not an inline constant would otherwise be rebuilt in vector
// registers, two moves per constant, for every amplitude.
struct PhaseK {
    double k[20];
};
// complex64: the angle g split into two floats, g = g1 + g2 to about 48 bits.
struct PhaseK32 {
    float g1, g2;
};
template <typename R>
__device__ __forceinline__ PhaseK32 phase_consts(double g, std::enable_if_t<std::is_same<R, float>::value, int> = 0)
{
    const float g1 = (float)g;
    return {g1, (float)(g - (double)g1)};
}
template <typename R>
__device__ __forceinline__ PhaseK phase_consts(double, std::enable_if_t<std::is_same<R, double>::value, int> = 0)
{
    PhaseK K = {{
        0x1.45f306dc9c883p-1,    // 2/pi
        0x1.921fb54400000p+0,    // pi/2: leading 33 bits
        0x1.0b4611a600000p-34,   //       next 33 bits
        0x1.3198a2e037073p-69,   //       remainder
        2.8114572543455206e-15,  //  1/17!   sin r / r - 1 in powers of r^2, highest first
        -7.647163731819816e-13,  // -1/15!
        1.6059043836821613e-10,  //  1/13!
        -2.505210838544172e-08,  // -1/11!
        2.7557319223985893e-06,  //  1/9!
        -0.0001984126984126984,  // -1/7!
        0.008333333333333333,    //  1/5!
        -0.16666666666666666,    // -1/3!
        -1.5619206968586225e-16, // -1/18!   cos r in powers of r^2, highest first
        4.779477332387385e-14,   //  1/16!
        -1.1470745597729725e-11, // -1/14!
        2.08767569878681e-09,    //  1/12!
        -2.755731922398589e-07,  // -1/10!
        2.48015873015873e-05,    //  1/8!
        -0.001388888888888889,   // -1/6!
        0.041666666666666664,    //  1/4!   (then -1/2! and 1 are inline constants)
    }};
#pragma unroll
    for (int i = 0; i < 20; ++i) asm volatile("" : "+s"(K.k[i]));
    return K;
}
// Arguments beyond the reduction's range (never met by the phases of real
// instances) go to the library's sincos, kept out of line so that the 16
// unrolled phase evaluations of a tile do not each carry a copy of it.
__device__ __attribute__((noinline)) double2 sincos_far(double x)
{
    double s, c;
    sincos(x, &s, &c);
    return make_double2(s, c);
}
// NEAR: the caller guarantees |x| < 1e6 (kernels of a spectator class; the
// launcher sends passes whose |gamma| max|C| could reach it elsewhere), so the
// out-of-line fallback and its call sites, which constrain register
// allocation, are left out.
template <bool NEAR = false>
__device__ __forceinline__ void sincos_cw(double x, double &s, double &c, const PhaseK &K)
{
    if (!NEAR && !(fabs(x) < 1.0e6)) {
        const double2 sc = sincos_far(x);
        s = sc.x;
        c = sc.y;
        return;
    }
    const double k = rint(x * K.k[0]);
    double r = fma(-k, K.k[1], x);
    r = fma(-k, K.k[2], r);
    r = fma(-k, K.k[3], r);
    const double r2 = r * r;
    double ps = K.k[4];
#pragma unroll
    for (int i = 5; i < 12; ++i) ps = fma(ps, r2, K.k[i]);
    const double sr = fma(ps * r2, r, r);
    double pc = K.k[12];
#pragma unroll
    for (int i = 13; i < 20; ++i) pc = fma(pc, r2, K.k[i]);
    pc = fma(pc, r2, -0.5);
    const double cr = fma(pc, r2, 1.0);
    const int q = (int)(((long long)k) & 3);
    // x = k pi/2 + r: rotate (cos r, sin r) by q quarter turns
    const double s0 = (q & 1) ? cr : sr, c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

// cos / sin of g * C.  complex128: fp64 (sincos_cw).  complex64: the reduction
// x = g C = k pi/2 + r runs in fp32: with g = g1 + g2 (PhaseK32) and C an fp32
// value, g1 C = p + pe exactly (pe from one FMA) and g2 C is below 2^-24 |x|;
// k = rint(p 2/pi); pi/2 is split into P1 + P2 + P3 with 12-bit P1 and P2, so
// for |k| < 2^12 the products k P1, k P2 are exact and r = p - k P1 is too
// (Sterbenz); r = ((p - k P1) - k P2 - k P3) + (pe + g2 C) is within 1.5 fp32
// ulps of pi/4 of the exact reduced argument (checked against fp64 on 2e5
// random products up to |x| = 6000).  |r| may exceed pi/4 by the rounding of
// p 2/pi; the polynomials below stay accurate there.  Then the Taylor series
// of sin to r^9 and of cos to r^8 in fp32 (truncation below 3e-8).  Arguments
// with |p| >= 4096 (k beyond 2^12) take the fp64 reduction instead, with r
// clamped to [-pi/4, pi/4] so that even arguments too large for it (|x| beyond
// ~2^50, far past fp32 phase resolution) give a unit-modulus factor.  K holds
// the constants of the complex128 form and the split angle of the complex64 one.
template <bool NEAR = false>
__device__ __forceinline__ void phase_cs(double g, double cval, double &c, double &s, const PhaseK &K)
{
    sincos_cw<NEAR>(g * cval, s, c, K);
}
// NEAR: the caller guarantees |g1 C| < 4096 (see sincos_cw), the fp32 path.
template <bool NEAR = false>
__device__ __forceinline__ void phase_cs(double g, float cval, float &c, float &s, const PhaseK32 &K)
{
    float r;
    int q;
    const float p = K.g1 * cval;
    if (NEAR || fabsf(p) < 4096.0f) {
        const float pe = fmaf(K.g1, cval, -p);
        const float k = rintf(p * 0x1.45f306p-1f);          // 2/pi
        float rr = fmaf(-k, 0x1.922p+0f, p);                // pi/2: 12-bit head
        rr = fmaf(-k, -0x1.2aep-18f, rr);                   //       12-bit second part
        rr = fmaf(-k, -0x1.de974p-31f, rr);                 //       remainder
        r = rr + (pe + K.g2 * cval);
        q = (int)k;
    } else {
        const double th = g * (double)cval;
        const double k = rint(th * 0.6366197723675814);  // 2/pi
        double rd = fma(-k, 1.5707963267948966, th);
        rd = fma(-k, 6.123233995736766e-17, rd);
        r = fminf(fmaxf((float)rd, -0.785398163f), 0.785398163f);
        q = (int)(k - 4.0 * floor(k * 0.25));  // k mod 4, defined for any k
    }
    const float r2 = r * r;
    float ps = 2.7557319e-6f;               //  1/9!
    ps = fmaf(ps, r2, -1.98412698e-4f);     // -1/7!
    ps = fmaf(ps, r2, 8.33333333e-3f);      //  1/5!
    ps = fmaf(ps, r2, -0.166666667f);       // -1/3!
    const float sr = fmaf(ps * r2, r, r);
    float pc = 2.48015873e-5f;              //  1/8!
    pc = fmaf(pc, r2, -1.38888889e-3f);     // -1/6!
    pc = fmaf(pc, r2, 4.16666667e-2f);      //  1/4!
    pc = fmaf(pc, r2, -0.5f);               // -1/2!
    const float cr = fmaf(pc, r2, 1.0f);
    // x = k pi/2 + r: rotate (cos r, sin r) by q quarter turns (q & 3 = k mod 4)
    const float s0 = (q & 1) ? cr : sr, c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
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

// Wave bits of a tile of amplitudes of type V (2 for complex128, 3 for complex64).
template <typename V>
constexpr int kWaveBits = 2;
template <>
constexpr int kWaveBits<float2> = 3;

// Amplitude held by lane l ^ 2 (the partner across tile bit 12 in arrangement
// B of a 13-bit tile): a DPP quad permutation [2, 3, 0, 1].
__device__ __forceinline__ float lane_xor2(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));
}
template <typename V>
__device__ __forceinline__ V lane_partner(V v)
{
    V o;
    o.x = lane_xor2(v.x);
    o.y = lane_xor2(v.y);
    return o;
}

// The factored rotation of bfly() across lanes: both members of a pair get the
// same formula, with the partner's amplitude p in place of the other register.
template <bool TM, typename V, typename R>
__device__ __forceinline__ void bfly_lane(V &s, V p, R m)
{
    if constexpr (TM) {
        s.x = fma(m, p.y, s.x);
        s.y = fma(-m, p.x, s.y);
    } else {
        s.x = fma(m, s.x, p.y);
        s.y = fma(m, s.y, -p.x);
    }
}

// Target bits of a pass as the stages see them.  Every full-tile pass of the
// plan rotates all tile bits from some S up (the S lowest bits are
// spectators).  With SP = S >= 0 that is known at compile time and every stage
// is taken or left out statically; with SP < 0 the tile-local mask decides at
// run time under wave-uniform branches (partial tiles, other plans).
template <int SP>
struct Targets {
    uint32_t tmask;
    __device__ __forceinline__ bool has(uint32_t bit) const
    {
        if constexpr (SP >= 0) return bit >= (uint32_t)SP;
        else return (tmask >> bit) & 1u;
    }
};

// Rotations of the target bits among the register bits of arrangement ARR
// (and, for 13-bit tiles in B, the lane-held bit 12).  Each register bit's
// stage runs under a wave-uniform branch.  The butterflies leave their
// results in new registers, and the values must sit in the same registers
// wherever the taken and the skipped path meet; with SKIP_COPY an empty asm
// statement redefines the values on the skipped path, so the register copies
// of that join are made there (where a pass skips a bit, once per tile)
// instead of after every taken stage: a third fewer VALU instructions in the
// compute of a complex128 forward pass, 2-3 % off those passes' time.  It is
// applied to complex128 tiles only (complex64 forward passes measured 11 %
// slower with it) and not in kernels that hold a second vector beside v,
// where it raises the register count past the kernel's budget.
template <int ARR, bool TM, bool SKIP_COPY = false, int SP, typename V, typename R>
__device__ __forceinline__ void mix_stage(V (&v)[16], R m, Targets<SP> tg)
{
    constexpr int WB = kWaveBits<V>;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (tg.has(regbit<ARR>(q))) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) bfly<TM>(v[r], v[r | (1 << q)], m);
        } else if constexpr (SKIP_COPY && SP < 0 && std::is_same<V, double2>::value) {
#pragma unroll
            for (int r = 0; r < 16; ++r) asm volatile("" : "+v"(v[r].x), "+v"(v[r].y));
        }
    }
    if constexpr (ARR == 1 && WB == 3) {
        if (tg.has(12)) {
#pragma unroll
            for (int r = 0; r < 16; ++r) bfly_lane<TM>(v[r], lane_partner(v[r]), m);
        }
    }
}

// Adjoint stage: for each target bit, add Im<lam|X_j|phi> over the register
// pairs (weighted by sig2, the squared factor both vectors still miss), then
// apply the factored inverse rotation to both.  Across lanes (tile bit 12 of
// 13-bit tiles, arrangement B) each lane adds Im(conj(lam) phi_partner); the
// two lanes of a pair together give the pair's term.
template <int ARR, bool TM, int SP, typename V, typename R>
__device__ __forceinline__ void adj_stage(V (&f)[16], V (&l)[16], R m, Targets<SP> tg,
                                          double &sig2, double f2, double &accB)
{
    constexpr int WB = kWaveBits<V>;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (tg.has(regbit<ARR>(q))) {
            typename PairSum<V>::T ps = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) {
                    const int r1 = r | (1 << q);
                    ps = imcx_acc(l[r1], f[r], imcx_acc(l[r], f[r1], ps));
                }
            accB = fma(sig2, (double)ps, accB);
            // The sum is formed here, while the stage's inputs are live: left to
            // the compiler it can be sunk towards its use at the end of the tile,
            // keeping the inputs of every stage alive (spills in straight-line code).
            asm volatile("" : "+v"(accB));
            sig2 *= f2;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) {
                    bfly<TM>(l[r], l[r | (1 << q)], m);
                    bfly<TM>(f[r], f[r | (1 << q)], m);
                }
        }
    }
    if constexpr (ARR == 1 && WB == 3) {
        if (tg.has(12)) {
            typename PairSum<V>::T ps = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const V fp = lane_partner(f[r]), lp = lane_partner(l[r]);
                ps = imcx_acc(l[r], fp, ps);
                bfly_lane<TM>(l[r], lp, m);
                bfly_lane<TM>(f[r], fp, m);
            }
            accB = fma(sig2, (double)ps, accB);
            asm volatile("" : "+v"(accB));
            sig2 *= f2;
        }
    }
}

// Sum over the target bits owned by arrangement ARR of Im<lam|X_j|phi> on the
// register (and lane) pairs, times w (the product of the factors both vectors miss).
template <int ARR, int SP, typename V>
__device__ __forceinline__ void beta_terms(const V (&f)[16], const V (&l)[16], Targets<SP> tg,
                                           double w, double &accB)
{
    constexpr int WB = kWaveBits<V>;
    using PS = typename PairSum<V>::T;
    // complex128: one fp64 chain over all bits; complex64: fp32 per bit
    double ps = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (tg.has(regbit<ARR>(q))) {
            PS pq = 0;
            if constexpr (std::is_same<PS, double>::value) pq = ps;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << q))) {
                    const int r1 = r | (1 << q);
                    pq = imcx_acc(l[r1], f[r], imcx_acc(l[r], f[r1], pq));
                }
            if constexpr (std::is_same<PS, double>::value) ps = pq;
            else ps += (double)pq;
        }
    }
    if constexpr (ARR == 1 && WB == 3) {
        if (tg.has(12)) {
            PS pq = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) pq = imcx_acc(l[r], lane_partner(f[r]), pq);
            ps += (double)pq;
        }
    }
    accB = fma(w, ps, accB);
    asm volatile("" : "+v"(accB));
}

__host__ __device__ __forceinline__ int popc(uint32_t x) { return __builtin_popcount(x); }

__device__ __forceinline__ double upow(double f, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= f;
    return r;
}

// Workgroup barrier ordering LDS accesses only: a wave waits for its own LDS
// operations, not for its outstanding global loads and stores, so a tile's
// transposes do not stall on memory traffic that they do not depend on.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int FROM, int TO, typename V>
__device__ __forceinline__ void xpose(V (&v)[16], V *lds, uint32_t lane, uint32_t wave)
{
    constexpr int WB = kWaveBits<V>;
    V *wr = lds + lds_slot<WB>(elem<FROM, WB>(lane, wave, 0));
    V *rd = lds + lds_slot<WB>(elem<TO, WB>(lane, wave, 0));
#pragma unroll
    for (int r = 0; r < 16; ++r) wr[lds_slot<WB>(elem<FROM, WB>(0, 0, r))] = v[r];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = rd[lds_slot<WB>(elem<TO, WB>(0, 0, r))];
    lds_barrier();
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

// Fixed-order sums over a block of NW waves of up to four values (with NW = 4
// each as block_sum would give it), valid in thread 0, with one barrier.
// `red` holds 4 NW doubles outside the transpose slots, so the caller's next
// LDS writes need no further barrier: thread 0 reads `red` before it reaches
// the next one.
template <int NW>
__device__ __forceinline__ void block_sums4(const double (&x)[4], const bool (&want)[4], double *red,
                                            double (&out)[4])
{
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    double w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = want[k] ? wave_sum(x[k]) : 0.0;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[NW * k + wave] = w[k];
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        out[k] = 0.0;
        if (threadIdx.x == 0 && want[k]) {
            double t = red[NW * k];
#pragma unroll
            for (int i = 1; i < NW; ++i) t += red[NW * k + i];
            out[k] = t;
        }
    }
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

// Kernels compiled for a spectator class S (full tiles whose S lowest tile bits
// are not rotated) take their access kind as a constant: the pass plans give
// such tiles a first run from global bit 0 of at least 6 bits exactly when
// S = 0 or S >= 6, which is when a pass streams (kStream); the launcher sends a
// pass whose flag disagrees to the run-time-mask kernels.  Without the run-time
// choice each load and store is one access instead of two under a branch
// (a quarter fewer instructions in the backward sweep).  The tile's fullness
// stays a run-time test: its branches keep the scheduler from hoisting the
// address arithmetic of every access, which as a constant spills registers.
__host__ __device__ constexpr bool stream_class(int S) { return S == 0 || S >= 6; }

// One pass over tile t: load, [phase], rotations, [E / adjoint terms / phase
// undo], store.  The workgroup's sums of the E, <lam|X|phi> and <lam|C|phi>
// terms are returned in sums[0..2] (valid in thread 0; zero when not taken).
// RES: psi and lam point into LDS (a whole one-tile instance held there), and
// a two-vector pass may take the LDS of psi for its transposes, so all loads
// of the tile complete before the first transpose writes.
template <typename R, int MODE, bool TM, bool TM2 = TM, int SP = -1, bool RES = false>
__device__ __forceinline__ void tile_pass(const PassArgs &a, uint64_t t, typename Tr<R>::V *lds,
                                          double (&sums)[4])
{
    using V = typename Tr<R>::V;
    using CT = typename Tr<R>::CT;
    constexpr int WB = Tr<R>::WB, NR = Tr<R>::NR;
    // The thread index is passed through an empty asm so that the per-thread
    // addresses and masks derived from it are formed inside each tile pass: a
    // caller that loops over tiles would otherwise keep them live across the
    // loop, next to the amplitudes held per thread.
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const Geometry &g = a.geo;
    const uint64_t base = tile_base(t, g);
    const bool full = g.tbits == (uint32_t)Tr<R>::TB;
    const uint32_t lim = 1u << g.tbits;
    const Targets<SP> tg{g.tmask};
    const bool strm = !RES && (SP >= 0 ? stream_class(SP) : (a.flags & kStream) != 0);
    V *psi = (V *)a.psi;
    V *lam = (V *)a.lam;
    const CT *cost = (const CT *)a.cost;

    // Global index of register r in arrangement A / C: a per-thread part plus a
    // part that depends on r only (the same for every thread of the grid).
    const uint64_t thrA = base | dep(elem<0, WB>(lane, wave, 0), g);
    const uint64_t thrC = base | dep(elem<2, WB>(lane, wave, 0), g);
    const RegOffsets<0, WB> offA(g);
    const RegOffsets<2, WB> offC(g);
#define ZA(r) (thrA | offA(r))
#define ZC(r) (thrC | offC(r))
#define VA(r) (full || elem<0, WB>(lane, wave, (r)) < lim)
#define VC(r) (full || elem<2, WB>(lane, wave, (r)) < lim)
    // Block sums of the tile's E, <lam|X|phi> and <lam|C|phi> terms, taken
    // before the final stores so that the workgroup retires right after issuing them.
#define REDUCE()                                                                        \
    do {                                                                                \
        if (wantE || wantB || wantG) {                                                  \
            const double x_[4] = {accE, accB, accG, accB2};                             \
            const bool w_[4] = {wantE, wantB, wantG, MODE == kBwdFuse};                 \
            block_sums4<Tr<R>::NW>(x_, w_, (double *)(lds + kLdsSlots<R>), sums);                \
        } else {                                                                        \
            sums[0] = sums[1] = sums[2] = sums[3] = 0.0;                                \
        }                                                                               \
    } while (0)

    double accE = 0.0, accB = 0.0, accG = 0.0;
    const V zero = {(R)0, (R)0};

    // The single-group sweeps raise the wave priority while their loads are
    // issued, so that a workgroup starting a tile gets its loads in flight ahead
    // of the arithmetic of the other workgroup on the CU (measured: forward
    // 26.9 vs 27.8 ms, backward 43 vs 44 ms at n = 32; the layer-boundary
    // sweeps, whose arithmetic dominates, are faster without it).
    constexpr bool kPrio = MODE != kBwdFuse;
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(2);
    // All global loads of the pass are issued up front (cost entries first);
    // loads placed after the arithmetic were found to serialise with it.
    constexpr bool TURN = MODE == kTurn || MODE == kTurnPhase;
    // complex128 passes whose B arrangement holds no target bit (S >= 4 spectator
    // bits, all of B's register bits) go from A to C and back with one transpose
    // (not the turn, which re-reads its tile from B's transpose)
    constexpr bool kSkipB = SP >= 4 && WB == 2 && !TURN;
    // which optional steps this launch performs (compile-time where the mode decides)
    const bool phaseIn = MODE == kTurnPhase || (MODE == kFwd && (a.flags & kPhaseIn));
    const bool phaseOut = MODE == kTurnPhase || MODE == kBwdFuse || (MODE == kBwd && (a.flags & kPhaseOut));
    const bool wantE = TURN || (MODE == kFwd && (a.flags & kEOut));
    const bool wantB = MODE != kFwd;
    const bool wantG = phaseOut;
    double accB2 = 0.0;  // kBwdFuse: <lam|X|phi> terms of the second rotation's layer
    const bool costC = TURN || phaseOut || (MODE == kFwd && (a.flags & kEOut));
    // Two-vector passes of complex64 tiles (16 waves per CU, 128 registers)
    // load the cost entries where they are used, which keeps them out of the
    // register budget of the rotations; the other waves cover the latency.
    constexpr bool kLateCost = Tr<R>::NW == 8 && (MODE == kBwd || MODE == kBwdFuse);
    CT cin[NR], cv[NR];
    if (phaseIn) {
#pragma unroll
        for (int r = 0; r < NR; ++r) cin[r] = VA(r) ? ld(&cost[ZA(r)], strm) : (CT)0;
    }
    if (costC && !kLateCost) {
#pragma unroll
        for (int r = 0; r < NR; ++r) cv[r] = VC(r) ? ld(&cost[ZC(r)], strm) : (CT)0;
    }

    if constexpr (MODE == kFwd || TURN) {
        V v[NR];
        if (a.flags & kInit) {
            const V a0 = {(R)a.amp0, (R)0};
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = VA(r) ? a0 : zero;
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = VA(r) ? ld(&psi[ZA(r)], strm) : zero;
        }
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
        if (phaseIn) {
            const auto PK = phase_consts<R>(-a.gamma_in);
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (VA(r)) {
                    R c, s;
                    phase_cs<(SP >= 0)>(-a.gamma_in, cin[r], c, s, PK);
                    v[r] = cmul(v[r], c, s);
                }
        }
        // complex128 turn: the loaded tile (the state before the group, in
        // arrangement A) stays in registers for the terms of A's bits at the end
        constexpr bool kKeep0 = MODE == kTurn && WB == 2;
        V v0[kKeep0 ? NR : 1];
        if constexpr (kKeep0) {
#pragma unroll
            for (int r = 0; r < NR; ++r) v0[r] = v[r];
        }
        const R mf = (R)a.mul_f;
        mix_stage<0, TM, !TURN>(v, mf, tg);
        if constexpr (kSkipB) {
            xpose<0, 2>(v, lds, lane, wave);
        } else {
            xpose<0, 1>(v, lds, lane, wave);
            mix_stage<1, TM, !TURN>(v, mf, tg);
            xpose<1, 2>(v, lds, lane, wave);
        }
        mix_stage<2, TM, !TURN>(v, mf, tg);
        const R sf = (R)a.scl_f;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = vscale(v[r], sf);

        if constexpr (MODE == kFwd) {
            if (a.flags & kEOut) {
#pragma unroll
                for (int r = 0; r < NR; ++r) accE += (double)cv[r] * norm2(v[r]);
            }
            REDUCE();
            if (!(a.flags & kNoStore)) {
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (VC(r)) st(v[r], &psi[ZC(r)], strm);
            }
        } else {
            // v is the final state phi on this tile: E, lam = C phi, then undo the
            // group on both, visiting the register arrangements C, B, A; lam is
            // stored from A (from C when the phase is undone too).
            V l[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
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
                const int kA = popc(tg.tmask & owned<0, WB>()), kB = popc(tg.tmask & owned<1, WB>());
                const int kC = popc(tg.tmask & owned<2, WB>());
                const double ff = a.fac_f, fb = a.fac_b;
                beta_terms<2>(v, l, tg, 1.0, accB);
                mix_stage<2, TM>(l, mb, tg);
                {
                    const V *rd = lds + lds_slot<WB>(elem<1, WB>(lane, wave, 0));
#pragma unroll
                    for (int r = 0; r < NR; ++r) v[r] = rd[lds_slot<WB>(elem<1, WB>(0, 0, r))];
                    lds_barrier();
                }
                xpose<2, 1>(l, lds, lane, wave);
                // lam misses fb^kC, phi (forward stages A, B) misses ff^(kA+kB)
                beta_terms<1>(v, l, tg, upow(fb, kC) * upow(ff, kA + kB), accB);
                mix_stage<1, TM>(l, mb, tg);
                if constexpr (kKeep0) {
                    // A's bits at the point before the group: the loaded phi (exact)
                    // and lam with the whole group undone (missing fb^k)
                    xpose<1, 0>(l, lds, lane, wave);
                    mix_stage<0, TM>(l, mb, tg);
                    beta_terms<0>(v0, l, tg, upow(fb, kA + kB + kC), accB);
                } else {
                    mix_stage<1, TM>(v, mb, tg);
                    xpose<1, 0>(v, lds, lane, wave);
                    xpose<1, 0>(l, lds, lane, wave);
                    beta_terms<0>(v, l, tg, upow(fb, kC + 2 * kB) * upow(ff, kA + kB), accB);
                    mix_stage<0, TM>(l, mb, tg);
                }
                REDUCE();
                if (!(a.flags & kNoStore)) {
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        if (VA(r)) st(vscale(l[r], sb), &lam[ZA(r)], strm);
                }
            } else {
            const double f2 = a.fac_b * a.fac_b;
            double sig2 = 1.0;
            adj_stage<2, TM>(v, l, mb, tg, sig2, f2, accB);
            xpose<2, 1>(v, lds, lane, wave);
            xpose<2, 1>(l, lds, lane, wave);
            adj_stage<1, TM>(v, l, mb, tg, sig2, f2, accB);
            xpose<1, 0>(v, lds, lane, wave);
            xpose<1, 0>(l, lds, lane, wave);
            adj_stage<0, TM>(v, l, mb, tg, sig2, f2, accB);
                xpose<0, 2>(l, lds, lane, wave);
                xpose<0, 2>(v, lds, lane, wave);
                const auto PK = phase_consts<R>(a.gamma_out);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    l[r] = vscale(l[r], sb);
                    if (VC(r)) {
                        accG += (double)cv[r] * imcx(l[r], vscale(v[r], sb));
                        R c, s;
                        phase_cs<(SP >= 0)>(a.gamma_out, cv[r], c, s, PK);
                        l[r] = cmul(l[r], c, s);
                    }
                }
                REDUCE();
                if (!(a.flags & kNoStore)) {
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        if (VC(r)) st(l[r], &lam[ZC(r)], strm);
                }
            }
        }
    } else {
        V f[NR], l[NR];
        if (MODE == kBwd && (a.flags & kLamFromC)) {
            // the first pass of a reverse sweep from a stored final state: lam = C phi
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const bool ok = VA(r);
                const CT c = ok ? ld(&cost[ZA(r)], strm) : (CT)0;
                f[r] = ok ? ld(&psi[ZA(r)], strm) : zero;
                l[r] = vscale(f[r], (R)c);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const bool ok = VA(r);
                f[r] = ok ? ld(&psi[ZA(r)], strm) : zero;
                l[r] = ok ? ld(&lam[ZA(r)], strm) : zero;
            }
        }
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
        if constexpr (RES) __syncthreads();
        const R mb = (R)a.mul_b;
        const double f2 = a.fac_b * a.fac_b;
        double sig2 = 1.0;
        adj_stage<0, TM>(f, l, mb, tg, sig2, f2, accB);
        if constexpr (kSkipB) {
            xpose<0, 2>(f, lds, lane, wave);
            xpose<0, 2>(l, lds, lane, wave);
        } else {
            xpose<0, 1>(f, lds, lane, wave);
            xpose<0, 1>(l, lds, lane, wave);
            adj_stage<1, TM>(f, l, mb, tg, sig2, f2, accB);
            xpose<1, 2>(f, lds, lane, wave);
            xpose<1, 2>(l, lds, lane, wave);
        }
        adj_stage<2, TM>(f, l, mb, tg, sig2, f2, accB);
        const R sb = (R)a.scl_b;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            f[r] = vscale(f[r], sb);
            l[r] = vscale(l[r], sb);
        }
        if (phaseOut) {
            // the last sweep stores nothing, so it skips the phase undo
            const bool undo = MODE == kBwdFuse || !(a.flags & kNoStore);
            const auto PK = phase_consts<R>(a.gamma_out);
            // with late cost loads, eight entries at a time (fewer registers live)
            constexpr int H = kLateCost ? NR / 2 : NR;
#pragma unroll
            for (int h = 0; h < NR; h += H) {
                if constexpr (kLateCost) {
                    // addresses formed afresh from the thread index: kept from the
                    // start of the tile they would be spilled
                    uint32_t tid2 = threadIdx.x;
                    asm volatile("" : "+v"(tid2));
                    const uint64_t thrC2 = base | dep(elem<2, WB>(tid2 & 63u, tid2 >> 6, 0), g);
#pragma unroll
                    for (int r = h; r < h + H; ++r) cv[r] = VC(r) ? ld(&cost[thrC2 | offC(r)], strm) : (CT)0;
                }
#pragma unroll
                for (int r = h; r < h + H; ++r)
                    if (VC(r)) {
                        accG += (double)cv[r] * imcx(l[r], f[r]);
                        if (undo) {
                            R c, s;
                            phase_cs<(SP >= 0)>(a.gamma_out, cv[r], c, s, PK);
                            f[r] = cmul(f[r], c, s);
                            l[r] = cmul(l[r], c, s);
                        }
                    }
                if constexpr (kLateCost) {
                    asm volatile("" : "+v"(accG));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        if constexpr (MODE == kBwdFuse) {
            // the same group's rotations of the previous layer, undone from C back to A
            const R mb2 = (R)a.mul_b2;
            const double f22 = a.fac_b2 * a.fac_b2;
            double sig22 = 1.0;
            adj_stage<2, TM2>(f, l, mb2, tg, sig22, f22, accB2);
            if constexpr (kSkipB) {
                xpose<2, 0>(f, lds, lane, wave);
                xpose<2, 0>(l, lds, lane, wave);
            } else {
                xpose<2, 1>(f, lds, lane, wave);
                xpose<2, 1>(l, lds, lane, wave);
                adj_stage<1, TM2>(f, l, mb2, tg, sig22, f22, accB2);
                xpose<1, 0>(f, lds, lane, wave);
                xpose<1, 0>(l, lds, lane, wave);
            }
            adj_stage<0, TM2>(f, l, mb2, tg, sig22, f22, accB2);
            REDUCE();
            const R sb2 = (R)a.scl_b2;
            uint32_t tid3 = threadIdx.x;
            asm volatile("" : "+v"(tid3));
            const uint64_t thrA3 = kLateCost ? (base | dep(elem<0, WB>(tid3 & 63u, tid3 >> 6, 0), g)) : thrA;
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (VA(r)) {
                    st(vscale(f[r], sb2), &psi[thrA3 | offA(r)], strm);
                    st(vscale(l[r], sb2), &lam[thrA3 | offA(r)], strm);
                }
        } else {
            REDUCE();
            if (!(a.flags & kNoStore)) {
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (VC(r)) {
                        st(f[r], &psi[ZC(r)], strm);
                        st(l[r], &lam[ZC(r)], strm);
                    }
            }
        }
    }
#undef ZA
#undef ZC
#undef VA
#undef VC
#undef REDUCE
}

// Layer-boundary forward pass on tile t: the group's rotations with layer l's
// angle (arrangements A, B, C), layer l+1's phase (in C), the same group's
// rotations with layer l+1's angle (C, B, A); loaded and stored in A.
template <typename R, bool TM, bool TM2, int SP = -1>
__device__ __forceinline__ void tile_pass_fwd_fuse(const PassArgs &a, uint64_t t, typename Tr<R>::V *lds)
{
    using V = typename Tr<R>::V;
    using CT = typename Tr<R>::CT;
    constexpr int WB = Tr<R>::WB, NR = Tr<R>::NR;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const Geometry &g = a.geo;
    const uint64_t base = tile_base(t, g);
    const bool full = g.tbits == (uint32_t)Tr<R>::TB;
    const uint32_t lim = 1u << g.tbits;
    const Targets<SP> tg{g.tmask};
    const bool strm = SP >= 0 ? stream_class(SP) : (a.flags & kStream) != 0;
    V *psi = (V *)a.psi;
    const CT *cost = (const CT *)a.cost;
    const uint64_t thrA = base | dep(elem<0, WB>(lane, wave, 0), g);
    const uint64_t thrC = base | dep(elem<2, WB>(lane, wave, 0), g);
    const RegOffsets<0, WB> offA(g);
    const RegOffsets<2, WB> offC(g);
    const V zero = {(R)0, (R)0};
    CT cv[NR];
    V v[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        cv[r] = (full || elem<2, WB>(lane, wave, r) < lim) ? ld(&cost[thrC | offC(r)], strm) : (CT)0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        v[r] = (full || elem<0, WB>(lane, wave, r) < lim) ? ld(&psi[thrA | offA(r)], strm) : zero;
    const R m1 = (R)a.mul_f, m2 = (R)a.mul_f2;
    // complex128 passes whose B arrangement holds no target bit go from A to C
    // (and back) with one transpose
    constexpr bool kSkipB = SP >= 4 && WB == 2;
    mix_stage<0, TM, true>(v, m1, tg);
    if constexpr (kSkipB) {
        xpose<0, 2>(v, lds, lane, wave);
    } else {
        xpose<0, 1>(v, lds, lane, wave);
        mix_stage<1, TM, true>(v, m1, tg);
        xpose<1, 2>(v, lds, lane, wave);
    }
    mix_stage<2, TM, true>(v, m1, tg);
    const R s1 = (R)a.scl_f;
    const auto PK = phase_consts<R>(-a.gamma_in);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        R c, s;
        phase_cs<(SP >= 0)>(-a.gamma_in, cv[r], c, s, PK);
        v[r] = cmul(vscale(v[r], s1), c, s);
    }
    mix_stage<2, TM2, true>(v, m2, tg);
    if constexpr (kSkipB) {
        xpose<2, 0>(v, lds, lane, wave);
    } else {
        xpose<2, 1>(v, lds, lane, wave);
        mix_stage<1, TM2, true>(v, m2, tg);
        xpose<1, 0>(v, lds, lane, wave);
    }
    mix_stage<0, TM2, true>(v, m2, tg);
    const R s2 = (R)a.scl_f2;
    uint64_t thrS = thrA;  // see tile_pass_bwd_fuse
    asm volatile("" : "+v"(thrS));
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (full || elem<0, WB>(lane, wave, r) < lim) st(vscale(v[r], s2), &psi[thrS | offA(r)], strm);
}

}  // namespace
}  // namespace qk
