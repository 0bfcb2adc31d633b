// gfx950 kernels of the QAOA statevector path.
//
// Streaming pass kernel (k_pass)
//   The mixer U_M(b) = prod_j exp(-i b X_j) is a product of commuting
//   single-qubit rotations (Eq. (1); Sec. IV-B applies them gate by gate).
//   Instead of one full-state sweep per qubit, a pass loads a tile of 2^TB
//   amplitudes whose index bits cover a group of qubits, applies every rotation
//   of that group in registers, and writes the tile back once (TB = 12 for
//   complex128, 13 for complex64: 64 KiB of state per tile either way).  A
//   tile is the set of indices with bits [0,S) and [h,h+k) free (S + k = TB);
//   the other n-TB bits are fixed by the workgroup.  Each thread holds 16
//   amplitudes (256 threads for complex128, 512 for complex64); three register
//   arrangements (A, B, C) each put four different tile bits into the register
//   index, and two LDS transposes move between them, so every tile bit up to
//   11 is a register bit once.  For TB = 12:
//     A: lane = bits 0-5,        reg = bits 6-9,         wave = bits 10-11
//     B: reg = bits 0-3,         lane = bits 4-9,        wave = bits 10-11
//     C: lane = bits 0-3,6,7,    reg = bits 4,5,10,11,   wave = bits 8-9
//   For TB = 13 bit 12 is a third wave bit in B and C and lane bit 5 in A,
//   where its rotation pairs each lane with the lane 32 away.
//   Global loads happen in A and stores in C; with k = 10 every access is a
//   64 B run of consecutive amplitudes, with S >= 6 a run of >= 512 B.
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
#include "tile_device.h"

namespace qk {
namespace {

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

// Gradient outputs in device memory from the summed slots (p <= 64 threads).
__global__ void k_gradient_out(const double *res, int p, double *E, double *dg, double *db)
{
    const int i = threadIdx.x;
    if (i == 0 && E) E[0] = res[0];
    if (i < p) {
        db[i] = 2.0 * res[1 + i];
        dg[i] = 2.0 * res[1 + p + i];
    }
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

// A workgroup builds 4096 consecutive entries of the cost diagonal per
// iteration.  Thread (lane, wave) holds the 16 entries z = base | q << 6 |
// lane | wave << 10, q < 16, so every store of a wave is 64 consecutive
// entries, and z bits >= 10 are the same for the whole wavefront.  The terms
// arrive as pieces (cost_terms.cpp): a piece whose wave-bit literals fail is
// skipped by the whole wavefront with a scalar branch, lanes that fail its
// lane-bit literals sit it out under the execution mask, and the rest add to
// entry q the piece's wq[q]: its weight where the piece covers q, -0.0 where
// it does not (x + (-0.0) == x exactly in round-to-nearest, signed zeros
// included).  Each entry thus receives exactly the weights of its active
// terms, added one by one in the given term order, as the definition sums
// them.
constexpr int kCostTileBits = 12;

template <typename CT>
__device__ __forceinline__ void store_costs(CT *__restrict__ C, uint64_t N, uint64_t zt, const double (&acc)[16])
{
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint64_t z = zt | ((uint64_t)q << 6);
        if (z < N) C[z] = (CT)acc[q];
    }
}

template <typename CT>
__global__ __launch_bounds__(kThreads) void k_cost_pieces(CT *__restrict__ C, uint64_t N,
                                                          const CostPiece *__restrict__ P,
                                                          int64_t count, double offset)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t tile = blockIdx.x; (tile << kCostTileBits) < N; tile += gridDim.x) {
        const uint64_t zw = (tile << kCostTileBits) | ((uint64_t)wave << 10);
        double acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = offset;
        for (int64_t k = 0; k < count; ++k) {
            const CostPiece &pc = P[k];
            const uint64_t um = pc.umask, uv = pc.uval;
            const uint32_t ln = pc.lanes;
            if ((zw & um) != uv) continue;  // the whole wavefront skips the piece
            double wq[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) wq[q] = pc.wq[q];
            if ((lane & ln & 63u) == (ln >> 8)) {  // lanes failing the test sit it out
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[q] += wq[q];
            }
        }
        store_costs(C, N, zw | lane, acc);
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

// One thread per shot (grid-stride): u -> target t = u * total, binary search over the
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
    const double T = pre[nsub];
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t s = (uint64_t)blockIdx.x * kThreads + threadIdx.x; s < (uint64_t)shots; s += stride) {
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
}

// Workgroups of a cost-diagonal launch: one per 4096 entries, at most 2^20.
inline unsigned cost_grid(uint64_t N)
{
    const uint64_t t = (N + (1ull << kCostTileBits) - 1) >> kCostTileBits;
    return (unsigned)(t < (1ull << 20) ? t : (1ull << 20));
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

int static_spectators(const Geometry &g, bool c64, int mode)
{
    const int TB = tile_bits(c64);
    const uint32_t t = g.tmask;
    if ((int)g.tbits != TB || t == 0) return -1;
    const int S = __builtin_ctz(t);
    if (t != (((1u << TB) - 1u) & ~((1u << S) - 1u))) return -1;  // not "every bit from S up"
    if (S == 0) return 0;
    return (S >= 2 && S <= 7 && mode != kTurnPhase) ? S : -1;
}

// A pass with a spectator class that has its own kernels (every full-tile pass
// whose S lowest tile bits are spectators, S = 0 or 2..7) runs them;
// any other pass runs the kernels that read the target mask at run time.
hipError_t launch_pass(int mode, bool c64, const PassArgs &a, uint64_t nblocks, hipStream_t s)
{
    int sp = static_spectators(a.geo, c64, mode);
    // a class's kernels fix whether their accesses stream, and take every phase
    // argument in the fast reduction's range
    if (sp >= 0 && stream_class(sp) != ((a.flags & kStream) != 0)) sp = -1;
    if (a.flags & kFarPhase) sp = -1;
    if (!c64) {
        switch (sp) {
        case 0: return launch_pass_sp<double, 0>(mode, a, nblocks, s);
        case 2: return launch_pass_sp<double, 2>(mode, a, nblocks, s);
        case 3: return launch_pass_sp<double, 3>(mode, a, nblocks, s);
        case 4: return launch_pass_sp<double, 4>(mode, a, nblocks, s);
        case 5: return launch_pass_sp<double, 5>(mode, a, nblocks, s);
        case 6: return launch_pass_sp<double, 6>(mode, a, nblocks, s);
        case 7: return launch_pass_sp<double, 7>(mode, a, nblocks, s);
        default: return launch_pass_sp<double, -1>(mode, a, nblocks, s);
        }
    }
    switch (sp) {
    case 0: return launch_pass_sp<float, 0>(mode, a, nblocks, s);
    case 2: return launch_pass_sp<float, 2>(mode, a, nblocks, s);
    case 3: return launch_pass_sp<float, 3>(mode, a, nblocks, s);
    case 4: return launch_pass_sp<float, 4>(mode, a, nblocks, s);
    case 5: return launch_pass_sp<float, 5>(mode, a, nblocks, s);
    case 6: return launch_pass_sp<float, 6>(mode, a, nblocks, s);
    case 7: return launch_pass_sp<float, 7>(mode, a, nblocks, s);
    default: return launch_pass_sp<float, -1>(mode, a, nblocks, s);
    }
}

hipError_t launch_sum_slots(const double *parts, uint64_t count, uint64_t stride, int nslots,
                            double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_slots, dim3(nslots), dim3(kThreads), 0, s, parts, count, stride, out);
    return hipGetLastError();
}

hipError_t launch_gradient_out(const double *res, int p, double *E, double *dgamma, double *dbeta,
                               hipStream_t s)
{
    if (p > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gradient_out, dim3(1), dim3(64), 0, s, res, p, E, dgamma, dbeta);
    return hipGetLastError();
}

hipError_t launch_cost_pieces(bool c64, void *C, int n, const CostPiece *pieces, int64_t count,
                              double offset, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (c64)
        hipLaunchKernelGGL(k_cost_pieces<float>, dim3(cost_grid(N)), dim3(kThreads), 0, s,
                           (float *)C, N, pieces, count, offset);
    else
        hipLaunchKernelGGL(k_cost_pieces<double>, dim3(cost_grid(N)), dim3(kThreads), 0, s,
                           (double *)C, N, pieces, count, offset);
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
    // one thread per shot up to 2^20 workgroups; beyond that each thread takes several
    const unsigned nb = grid_for((uint64_t)shots);
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
