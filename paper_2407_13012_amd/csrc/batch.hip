// Batched engine: thousands of small MaxCut instances of uneven size, each
// optimised with Adam on its QAOA angles, in one persistent launch.
//
// A fixed grid of workgroups pops instances from a work queue (largest n
// first).  A workgroup owns one instance at a time and runs everything for it
// in its own scratch slot: the cost diagonal (Sec. IV-A, cut indicator per
// edge), then for every Adam step one expectation + adjoint gradient (the
// same tiled passes as the single-instance path, Sec. II-B / IV-C, with the
// tiles of a pass processed in order by the workgroup) and the Adam update of
// the 2p angles, and finally E at the optimised angles.  Every wave reaches
// the end of the queue, so the launch always drains.  The queue counter is
// reset by a kernel, and the pair (reset, engine) is captured in a hipGraph.
#include "qaoa.h"
#include "tile_device.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

namespace qk {
namespace {

constexpr int kMaxP = 16;       // depth limit of the batched engine
constexpr int kMaxPasses = 16;  // passes per mixer layer
constexpr int kMaxBatchN = QAOA_BATCH_MAX_QUBITS;

struct BatchArgs {
    int32_t count;
    int32_t begin, end;     // this launch's range of the processing order
    const int32_t *order;   // processing order (largest n first)
    const int32_t *nq;      // [count] qubits
    const int64_t *eoff;    // [count + 1] edge offsets
    const int32_t *edges;   // [E][2]
    const double *w;        // [E] (NULL: unit weights)
    const double *scale;    // [count] objective scale (1 / sum |w|)
    double *gamma, *beta;   // [count][p] start in, optimum out
    double *e_first;        // [count] E at the start angles
    double *e_last;         // [count] E at the final angles
    int32_t p, steps;
    double lr, b1, b2, eps;
    const Geometry *geo;    // [(kMaxBatchN + 1) * kMaxPasses]
    const int32_t *npass;   // [kMaxBatchN + 1]
    double2 *psi, *lam;     // slot arrays, `slot` amplitudes each
    double *cost;
    uint64_t slot;
    uint32_t *counter;      // this launch's queue counter
    uint64_t *ticks;        // [count][2] device wall clock at an instance's start and end
};

// Values every lane of the workgroup holds alike (read from LDS or loaded from
// a uniform address), moved to scalar registers so the tile code keeps its
// addressing and coefficients there.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni(uint64_t x)
{
    return (uint64_t)uni((uint32_t)x) | ((uint64_t)uni((uint32_t)(x >> 32)) << 32);
}
__device__ __forceinline__ int64_t uni(int64_t x) { return (int64_t)uni((uint64_t)x); }
__device__ __forceinline__ double uni(double x) { return __longlong_as_double((long long)uni((uint64_t)__double_as_longlong(x))); }

// Kernel arguments of pass gi of an n-qubit instance with mixer angle beta.
__device__ __forceinline__ void make_args(PassArgs &a, const BatchArgs &B, int n, int gi, double beta,
                                          double2 *psi, double2 *lam, double *cost)
{
    a.psi = psi;
    a.lam = lam;
    a.cost = cost;
    a.part_e = a.part_b = a.part_g = nullptr;
    const Geometry &gs = B.geo[n * kMaxPasses + gi];
#pragma unroll
    for (int r = 0; r < kTileRuns; ++r) {
        a.geo.t_src[r] = uni(gs.t_src[r]);
        a.geo.t_dst[r] = uni(gs.t_dst[r]);
        a.geo.t_len[r] = uni(gs.t_len[r]);
    }
#pragma unroll
    for (int r = 0; r < kFreeRuns; ++r) {
        a.geo.f_src[r] = uni(gs.f_src[r]);
        a.geo.f_dst[r] = uni(gs.f_dst[r]);
        a.geo.f_len[r] = uni(gs.f_len[r]);
    }
    a.geo.tmask = uni(gs.tmask);
    a.geo.tbits = uni(gs.tbits);
    a.xcd_g = 0;
    a.flags = 0;
    a.amp0 = 1.0 / sqrt((double)(1ull << n));
    a.gamma_in = a.gamma_out = 0.0;
    double s, c;
    sincos(beta, &s, &c);
    const int k = __builtin_popcount(a.geo.tmask);
    const bool tm = fabs(c) >= fabs(s);
    a.tan_mode = tm ? 1u : 0u;
    double mf = tm ? s / c : c / s, ff = tm ? c : s, fb = tm ? c : -s;
    double sf = 1.0, sb = 1.0;
    for (int i = 0; i < k; ++i) {
        sf *= ff;
        sb *= fb;
    }
    a.tan_mode = uni(a.tan_mode);
    a.mul_f = uni(mf);
    a.mul_b = -a.mul_f;
    a.fac_f = uni(ff);
    a.fac_b = uni(fb);
    a.scl_f = uni(sf);
    a.scl_b = uni(sb);
}

// Hides a value's origin from the optimiser, so that what the tile code
// derives from it is recomputed per tile instead of being hoisted out of the
// tile loop and kept live (the derived addresses and masks do not fit in
// registers alongside the tile's amplitudes).
__device__ __forceinline__ void opaque(uint32_t &x) { asm volatile("" : "+s"(x)); }

// All tiles of one pass, in order; sums accumulate in thread 0.
template <int MODE, bool RES = false>
__device__ __forceinline__ void run_tiles(const PassArgs &a, uint64_t T, double2 *lds, double (&acc)[3])
{
    for (uint64_t t = 0; t < T; ++t) {
        PassArgs b = a;
#pragma unroll
        for (int r = 0; r < kTileRuns; ++r) {
            opaque(b.geo.t_src[r]);
            opaque(b.geo.t_dst[r]);
            opaque(b.geo.t_len[r]);
        }
        opaque(b.geo.tmask);
        opaque(b.geo.tbits);
        double s[4];
        if (b.tan_mode) tile_pass<double, MODE, true, true, -1, RES>(b, t, lds, s);
        else tile_pass<double, MODE, false, false, -1, RES>(b, t, lds, s);
        acc[0] += s[0];
        acc[1] += s[1];
        acc[2] += s[2];
    }
    __syncthreads();  // this pass's stores are visible to the next pass
}

// Second rotation of a layer-boundary pass (the other layer's angle).
__device__ __forceinline__ void make_second(PassArgs &a, double beta2)
{
    double s, c;
    sincos(beta2, &s, &c);
    const int k = __builtin_popcount(a.geo.tmask);
    const bool tm = fabs(c) >= fabs(s);
    const double mf = tm ? s / c : c / s, ff = tm ? c : s, fb = tm ? c : -s;
    double sf = 1.0, sb = 1.0;
    for (int i = 0; i < k; ++i) {
        sf *= ff;
        sb *= fb;
    }
    a.tan_mode2 = uni(tm ? 1u : 0u);
    a.mul_f2 = uni(mf);
    a.mul_b2 = -a.mul_f2;
    a.fac_b2 = uni(fb);
    a.scl_f2 = uni(sf);
    a.scl_b2 = uni(sb);
}

// All tiles of one layer-boundary pass; for kBwdFuse acc gets the X terms of
// the later layer ([1]), the C term ([2]) and the X terms of the earlier layer ([3]).
template <int MODE>
__device__ __forceinline__ void run_tiles_fuse(const PassArgs &a, uint64_t T, double2 *lds, double (&acc)[4])
{
    for (uint64_t t = 0; t < T; ++t) {
        PassArgs b = a;
#pragma unroll
        for (int r = 0; r < kTileRuns; ++r) {
            opaque(b.geo.t_src[r]);
            opaque(b.geo.t_dst[r]);
            opaque(b.geo.t_len[r]);
        }
        opaque(b.geo.tmask);
        opaque(b.geo.tbits);
        const int sel = (b.tan_mode ? 2 : 0) + (b.tan_mode2 ? 1 : 0);
        if constexpr (MODE == kFwdFuse) {
            if (sel == 3) tile_pass_fwd_fuse<double, true, true>(b, t, lds);
            else if (sel == 2) tile_pass_fwd_fuse<double, true, false>(b, t, lds);
            else if (sel == 1) tile_pass_fwd_fuse<double, false, true>(b, t, lds);
            else tile_pass_fwd_fuse<double, false, false>(b, t, lds);
        } else {
            double s[4];
            if (sel == 3) tile_pass<double, kBwdFuse, true, true>(b, t, lds, s);
            else if (sel == 2) tile_pass<double, kBwdFuse, true, false>(b, t, lds, s);
            else if (sel == 1) tile_pass<double, kBwdFuse, false, true>(b, t, lds, s);
            else tile_pass<double, kBwdFuse, false, false>(b, t, lds, s);
            acc[1] += s[1];
            acc[2] += s[2];
            acc[3] += s[3];
        }
    }
    __syncthreads();
}

// Mixer group at position idx of layer l (even layers ascending, odd descending).
__device__ __forceinline__ int group_at(int l, int idx, int P) { return (l % 2 == 0) ? idx : P - 1 - idx; }

// E (out[0]) and, with grad, dE/dgamma (out[1 .. p]) and dE/dbeta (out[p+1 ..])
// of the instance in the workgroup's slot; th = (gamma, beta).  out is shared
// memory written by thread 0.  Schedule (Sec. II-B / IV-C), the one of the
// single-instance gradient: the layers forward, except the last group of the
// last layer; the turn pass, which applies that group, takes E, forms
// lam = C psi and undoes the group on lam; then per layer, last first, the
// mixer groups undone on (phi, lam) with the <lam|X_j|phi> terms, a layer's
// first group also undoing its phase with the <lam|C|phi> term.  Layers visit
// their groups in alternating order, so that with two or more groups per
// layer the groups meeting at a layer boundary share one sweep.  Without
// grad the forward runs through every group and its last pass takes E.
__device__ __forceinline__ void wg_eval(const BatchArgs &B, int n, bool grad, const double *th,
                                        double2 *lds, double2 *psi, double2 *lam, double *cost,
                                        double *out)
{
    const int p = B.p, P = uni(B.npass[n]);
    const uint64_t T = n > kTileBits ? 1ull << (n - kTileBits) : 1ull;
    const uint32_t tid = threadIdx.x;
    if (tid == 0)
        for (int i = 0; i <= 2 * p; ++i) out[i] = 0.0;
    PassArgs a;
    for (int l = 0; l < p; ++l) {
        for (int idx = 0; idx < P; ++idx) {
            if (P > 1 && l > 0 && idx == 0) continue;  // applied by layer l - 1's boundary sweep
            const bool lastg = idx == P - 1;
            if (grad && lastg && l == p - 1) break;   // the turn pass
            const int gi = P > 1 ? group_at(l, idx, P) : 0;
            make_args(a, B, n, gi, uni(th[p + l]), psi, lam, cost);
            if (P > 1 && lastg && l < p - 1) {
                make_second(a, uni(th[p + l + 1]));
                a.gamma_in = uni(th[l + 1]);
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                run_tiles_fuse<kFwdFuse>(a, T, lds, acc);
                continue;
            }
            if (idx == 0) {
                a.flags |= kPhaseIn;
                a.gamma_in = uni(th[l]);
                if (l == 0) a.flags |= kInit;
            }
            if (lastg && l == p - 1) a.flags |= kEOut;
            double acc[3] = {0.0, 0.0, 0.0};
            run_tiles<kFwd>(a, T, lds, acc);
            if (tid == 0 && lastg && l == p - 1) out[0] = acc[0];
        }
    }
    if (!grad) return;
    {
        const int l = p - 1;
        make_args(a, B, n, P > 1 ? group_at(l, P - 1, P) : 0, uni(th[p + l]), psi, lam, cost);
        double acc[3] = {0.0, 0.0, 0.0};
        if (P == 1) {
            a.flags |= kPhaseIn | kPhaseOut;
            a.gamma_in = a.gamma_out = uni(th[l]);
            if (l == 0) a.flags |= kInit | kNoStore;
            run_tiles<kTurnPhase>(a, T, lds, acc);
        } else {
            run_tiles<kTurn>(a, T, lds, acc);
        }
        if (tid == 0) {
            out[0] = acc[0];
            out[1 + p + l] += acc[1];
            out[1 + l] += acc[2];
        }
    }
    for (int l = p - 1; l >= 0; --l) {
        for (int j = 0; j < P; ++j) {
            const int idx = P - 1 - j;
            if (j == 0 && (l == p - 1 || P > 1)) continue;  // the turn pass, or layer l + 1's boundary sweep
            const int gi = P > 1 ? group_at(l, idx, P) : 0;
            make_args(a, B, n, gi, uni(th[p + l]), psi, lam, cost);
            if (P > 1 && idx == 0 && l > 0) {
                make_second(a, uni(th[p + l - 1]));
                a.gamma_out = uni(th[l]);
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                run_tiles_fuse<kBwdFuse>(a, T, lds, acc);
                if (tid == 0) {
                    out[1 + p + l] += acc[1];
                    out[1 + l] += acc[2];
                    out[p + l] += acc[3];
                }
                continue;
            }
            if (idx == 0) {
                a.flags |= kPhaseOut;
                a.gamma_out = uni(th[l]);
                if (l == 0) a.flags |= kNoStore;
            }
            double acc[3] = {0.0, 0.0, 0.0};
            run_tiles<kBwd>(a, T, lds, acc);
            if (tid == 0) {
                out[1 + p + l] += acc[1];
                out[1 + l] += acc[2];
            }
        }
    }
    if (tid == 0)
        for (int i = 1; i <= 2 * p; ++i) out[i] *= 2.0;
}

// wg_eval for an instance of at most kTileBits qubits whose state and adjoint
// vector live in LDS (psi, lam): every mixer layer is one pass over the single
// tile, as in wg_eval with one group per layer.  The passes that hold one vector
// transpose through lam's LDS (lam is dead then, or written at the pass's end),
// the two-vector passes through psi's, after both vectors are in registers.
__device__ __forceinline__ void wg_eval_res(const BatchArgs &B, int n, bool grad, const double *th,
                                            double2 *psi, double2 *lam, double *cost, double *out)
{
    const int p = B.p;
    const uint32_t tid = threadIdx.x;
    if (tid == 0)
        for (int i = 0; i <= 2 * p; ++i) out[i] = 0.0;
    PassArgs a;
    for (int l = 0; l < p; ++l) {
        if (grad && l == p - 1) break;  // the turn pass
        make_args(a, B, n, 0, uni(th[p + l]), psi, lam, cost);
        a.flags |= kPhaseIn;
        a.gamma_in = uni(th[l]);
        if (l == 0) a.flags |= kInit;
        if (l == p - 1) a.flags |= kEOut;
        double acc[3] = {0.0, 0.0, 0.0};
        run_tiles<kFwd, true>(a, 1, lam, acc);
        if (tid == 0 && l == p - 1) out[0] = acc[0];
    }
    if (!grad) return;
    {
        const int l = p - 1;
        make_args(a, B, n, 0, uni(th[p + l]), psi, lam, cost);
        a.flags |= kPhaseIn | kPhaseOut;
        a.gamma_in = a.gamma_out = uni(th[l]);
        if (l == 0) a.flags |= kInit | kNoStore;
        double acc[3] = {0.0, 0.0, 0.0};
        run_tiles<kTurnPhase, true>(a, 1, lam, acc);
        if (tid == 0) {
            out[0] = acc[0];
            out[1 + p + l] += acc[1];
            out[1 + l] += acc[2];
        }
    }
    for (int l = p - 2; l >= 0; --l) {
        make_args(a, B, n, 0, uni(th[p + l]), psi, lam, cost);
        a.flags |= kPhaseOut;
        a.gamma_out = uni(th[l]);
        if (l == 0) a.flags |= kNoStore;
        double acc[3] = {0.0, 0.0, 0.0};
        run_tiles<kBwd, true>(a, 1, psi, acc);
        if (tid == 0) {
            out[1 + p + l] += acc[1];
            out[1 + l] += acc[2];
        }
    }
    if (tid == 0)
        for (int i = 1; i <= 2 * p; ++i) out[i] *= 2.0;
}

__global__ __launch_bounds__(kThreads) void k_reset(uint32_t *c)
{
    c[0] = 0u;
    c[1] = 0u;
}

// The queue loop of one launch.  RES: the instances are one tile each and their
// state and adjoint vector stay in the LDS arrays lds0 / lds1 for the whole
// optimisation; otherwise they live in the workgroup's slot and lds0 takes the
// transposes.  The cost diagonal is in the slot either way.
template <bool RES>
__device__ __forceinline__ void engine(const BatchArgs &B, double2 *lds0, double2 *lds1)
{
    __shared__ double th[2 * kMaxP], am[2 * kMaxP], av[2 * kMaxP], gr[2 * kMaxP + 1];
    __shared__ int sh_idx;
    const uint32_t tid = threadIdx.x;
    double2 *psi = RES ? lds0 : B.psi + (uint64_t)blockIdx.x * B.slot;
    double2 *lam = RES ? lds1 : B.lam + (uint64_t)blockIdx.x * B.slot;
    double *cost = B.cost + (uint64_t)blockIdx.x * B.slot;
    const int p = B.p;
    for (;;) {
        if (tid == 0) sh_idx = B.begin + (int)atomicAdd(B.counter, 1u);
        __syncthreads();
        const int idx = uni(sh_idx);
        __syncthreads();
        if (idx >= B.end) return;
        const int i = uni(B.order[idx]);
        if (tid == 0) B.ticks[2 * (int64_t)i] = wall_clock64();
        const int n = uni(B.nq[i]);
        const uint64_t N = 1ull << n;
        // cost diagonal: sum of cut edge weights in edge order
        const int64_t e0 = uni(B.eoff[i]), e1 = uni(B.eoff[i + 1]);
        for (uint64_t z = tid; z < N; z += kThreads) {
            double acc = 0.0;
            for (int64_t k = e0; k < e1; ++k) {
                const int u = B.edges[2 * k], v = B.edges[2 * k + 1];
                const double wk = B.w ? B.w[k] : 1.0;
                acc = (((z >> u) ^ (z >> v)) & 1ull) ? acc + wk : acc;
            }
            cost[z] = acc;
        }
        if (tid < 2 * p) {
            th[tid] = tid < p ? B.gamma[(int64_t)i * p + tid] : B.beta[(int64_t)i * p + tid - p];
            am[tid] = 0.0;
            av[tid] = 0.0;
        }
        __syncthreads();
        const double sc = B.scale[i];
        // steps gradient evaluations with an Adam update each, then one
        // evaluation of E at the final angles (one call site keeps a single
        // copy of the pass code in the kernel)
        for (int step = 0;; ++step) {
            const bool last = step == B.steps;
            if constexpr (RES) wg_eval_res(B, n, !last, th, psi, lam, cost, gr);
            else wg_eval(B, n, !last, th, lds0, psi, lam, cost, gr);
            __syncthreads();
            if (tid == 0 && step == 0) B.e_first[i] = gr[0];
            if (last) {
                if (tid == 0) B.e_last[i] = gr[0];
                break;
            }
            if (tid < 2 * p) {
                // Adam ascent on sc * E
                const double g = sc * gr[1 + tid];
                am[tid] = B.b1 * am[tid] + (1.0 - B.b1) * g;
                av[tid] = B.b2 * av[tid] + (1.0 - B.b2) * g * g;
                const double mh = am[tid] / (1.0 - pow(B.b1, (double)(step + 1)));
                const double vh = av[tid] / (1.0 - pow(B.b2, (double)(step + 1)));
                th[tid] += B.lr * mh / (sqrt(vh) + B.eps);
            }
            __syncthreads();
        }
        if (tid < 2 * p) {
            if (tid < p) B.gamma[(int64_t)i * p + tid] = th[tid];
            else B.beta[(int64_t)i * p + tid - p] = th[tid];
        }
        if (tid == 0) B.ticks[2 * (int64_t)i + 1] = wall_clock64();
        __syncthreads();
    }
}

// WPE = waves per SIMD the register allocation is held to: 1 leaves room for
// every value of the tile code, 2 hides more memory latency at the cost of a
// few spilled registers.  The tuner measures both.
template <int WPE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_batch(BatchArgs B)
{
    __shared__ double2 lds[kLdsTotal<double>];
    engine<false>(B, lds, lds);
}

// Instances of at most kTileBits qubits with both vectors resident in LDS
// (2 x 68 KiB: one workgroup per compute unit).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_batch_res(BatchArgs B)
{
    __shared__ double2 lds_psi[kLdsTotal<double>], lds_lam[kLdsTotal<double>];
    engine<true>(B, lds_psi, lds_lam);
}

}  // namespace
}  // namespace qk

// ------------------------------------------------------------------ C ABI

struct qaoa_batch_s {
    int count = 0, p = 0, nmax = 0, device = 0, workgroups = 0, wpe = 1;
    int split = 0;            // instances [0, split) of the order are streamed, the rest LDS-resident
    int res_workgroups = 0;   // grid of the LDS-resident launch
    int resident_max_n = 0;
    bool ran = false;
    int64_t edges_total = 0;
    hipStream_t stream = nullptr;
    std::vector<void *> allocs;
    std::vector<int32_t> order, nq;
    qk::BatchArgs args{}, args_res{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = true;
    bool poisoned = false;
};

namespace {

qaoa_status bfail(qaoa_status st, const char *msg)
{
    qk::set_error_message(msg);
    return st;
}

#define BCHECK(b, call)                                                        \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            if (b) (b)->poisoned = true;                                       \
            qk::set_error_message(std::string(#call " failed: ") + hipGetErrorString(e_)); \
            return QAOA_ERR_DEVICE;                                            \
        }                                                                      \
    } while (0)

template <typename T>
qaoa_status upload(qaoa_batch b, T **dst, const T *src, size_t count)
{
    BCHECK(b, hipMalloc((void **)dst, std::max<size_t>(count, 1) * sizeof(T)));
    b->allocs.push_back(*dst);
    if (src && count) BCHECK(b, hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, b->stream));
    return QAOA_OK;
}

qaoa_status launch_engine(qaoa_batch b)
{
    hipLaunchKernelGGL(qk::k_reset, dim3(1), dim3(1), 0, b->stream, b->args.counter);
    BCHECK(b, hipGetLastError());
    if (b->split > 0) {
        const dim3 grid(std::min(b->workgroups, b->split));
        if (b->wpe == 2) hipLaunchKernelGGL(qk::k_batch<2>, grid, dim3(qk::kThreads), 0, b->stream, b->args);
        else hipLaunchKernelGGL(qk::k_batch<1>, grid, dim3(qk::kThreads), 0, b->stream, b->args);
        BCHECK(b, hipGetLastError());
    }
    if (b->split < b->count) {
        hipLaunchKernelGGL(qk::k_batch_res, dim3(b->res_workgroups), dim3(qk::kThreads), 0, b->stream,
                           b->args_res);
        BCHECK(b, hipGetLastError());
    }
    return QAOA_OK;
}

}  // namespace

extern "C" {

qaoa_status qaoa_batch_create(int32_t count, const int32_t *n, const int64_t *edge_offsets,
                              const int32_t *edges, const double *w, int32_t p,
                              const qaoa_batch_options *opt, qaoa_batch *out)
{
    if (!out) return bfail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    if (count < 1 || !n || !edge_offsets) return bfail(QAOA_ERR_INVALID_ARGUMENT, "count, n or offsets invalid");
    if (p < 1 || p > qk::kMaxP) return bfail(QAOA_ERR_INVALID_ARGUMENT, "p must be in [1, 16]");
    qaoa_batch_options o;
    std::memset(&o, 0, sizeof o);
    o.steps = 100;
    o.lr = 0.05;
    o.beta1 = 0.9;
    o.beta2 = 0.999;
    o.eps = 1e-8;
    o.max_group = 10;
    o.use_graph = 1;
    if (opt) o = *opt;
    for (int m = 0; m <= qk::kMaxBatchN; ++m)
        if (o.group_by_n[m] < 0 || o.group_by_n[m] > 10)
            return bfail(QAOA_ERR_INVALID_ARGUMENT, "group_by_n entries must be in [0, 10]");
    if (o.steps < 0 || !(o.lr > 0.0) || !(o.beta1 >= 0.0 && o.beta1 < 1.0) ||
        !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps > 0.0) || o.workgroups < 0 ||
        o.max_group < 1 || o.max_group > 10 || o.waves_per_simd < 0 || o.waves_per_simd > 2 ||
        o.resident_max_n < 0 || o.resident_max_n > qk::kTileBits)
        return bfail(QAOA_ERR_INVALID_ARGUMENT, "invalid options");
    if (edge_offsets[0] != 0) return bfail(QAOA_ERR_INVALID_ARGUMENT, "edge_offsets[0] must be 0");
    int nmax = 0;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 2 || n[i] > qk::kMaxBatchN) return bfail(QAOA_ERR_INVALID_ARGUMENT, "n out of [2, 24]");
        if (edge_offsets[i + 1] < edge_offsets[i]) return bfail(QAOA_ERR_INVALID_ARGUMENT, "offsets decrease");
        nmax = std::max(nmax, (int)n[i]);
    }
    const int64_t E = edge_offsets[count];
    if (E > 0 && !edges) return bfail(QAOA_ERR_INVALID_ARGUMENT, "edges is NULL");
    std::vector<double> scale(count, 1.0);
    for (int i = 0; i < count; ++i) {
        double s = 0.0;
        for (int64_t k = edge_offsets[i]; k < edge_offsets[i + 1]; ++k) {
            const int u = edges[2 * k], v = edges[2 * k + 1];
            if (u < 0 || v < 0 || u >= n[i] || v >= n[i] || u == v)
                return bfail(QAOA_ERR_INVALID_ARGUMENT, "edge index out of range or self-loop");
            const double wk = w ? w[k] : 1.0;
            if (!std::isfinite(wk)) return bfail(QAOA_ERR_INVALID_ARGUMENT, "weights must be finite");
            s += std::fabs(wk);
        }
        if (s > 0.0) scale[i] = 1.0 / s;
    }

    qaoa_batch b = new (std::nothrow) qaoa_batch_s();
    if (!b) return bfail(QAOA_ERR_OUT_OF_MEMORY, "host allocation");
    b->count = count;
    b->p = p;
    b->nmax = nmax;
    b->edges_total = E;
    b->use_graph = o.use_graph != 0;
    b->wpe = o.waves_per_simd == 2 ? 2 : 1;
    b->resident_max_n = o.resident_max_n;
    auto cleanup = [&](qaoa_status st) {
        std::string keep = qk::error_message();
        qaoa_batch_destroy(b);
        qk::set_error_message(keep);
        return st;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return cleanup(bfail(QAOA_ERR_DEVICE, "hipGetDevice failed"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess)
        return cleanup(bfail(QAOA_ERR_DEVICE, "hipGetDeviceProperties failed"));
    int per_cu = 0;
    const hipError_t oe = b->wpe == 2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, qk::k_batch<2>, qk::kThreads, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, qk::k_batch<1>, qk::kThreads, 0);
    if (oe != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    b->workgroups = o.workgroups > 0 ? o.workgroups : per_cu * prop.multiProcessorCount;
    b->workgroups = std::min(b->workgroups, count);
    int per_cu_res = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_res, qk::k_batch_res, qk::kThreads, 0) !=
            hipSuccess ||
        per_cu_res < 1)
        per_cu_res = 1;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return cleanup(bfail(QAOA_ERR_DEVICE, "stream creation failed"));

    const uint64_t slot = 1ull << nmax;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return cleanup(bfail(QAOA_ERR_DEVICE, "hipMemGetInfo failed"));
    const double need = (double)b->workgroups * (double)slot * 40.0 + (double)E * 16.0 + count * 64.0;
    if (need > (double)fr) return cleanup(bfail(QAOA_ERR_OUT_OF_MEMORY, "scratch slots do not fit"));

    // pass plans of every size in the batch
    std::vector<qk::Geometry> geo((qk::kMaxBatchN + 1) * qk::kMaxPasses);
    std::vector<int32_t> npass(qk::kMaxBatchN + 1, 0);
    for (int m = 2; m <= nmax; ++m) {
        const int kg = o.group_by_n[m] ? o.group_by_n[m] : o.max_group;
        const std::vector<qk::PassPlan> pl = qk::plan_passes(m, false, kg);
        if ((int)pl.size() > qk::kMaxPasses) return cleanup(bfail(QAOA_ERR_UNSUPPORTED, "too many passes"));
        npass[m] = (int32_t)pl.size();
        for (size_t j = 0; j < pl.size(); ++j) qk::make_geometry(m, pl[j], &geo[m * qk::kMaxPasses + j]);
    }
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return n[a] > n[c]; });
    // the largest-first order puts the LDS-resident instances (one pass per layer) at its end
    b->split = count;
    while (b->split > 0 && n[order[b->split - 1]] <= o.resident_max_n) --b->split;
    for (int i = b->split; i < count; ++i)
        if (npass[n[order[i]]] != 1) return cleanup(bfail(QAOA_ERR_UNSUPPORTED, "resident instance with several passes"));
    // the resident launch uses the first res_workgroups slots' cost areas
    b->res_workgroups = std::min({per_cu_res * prop.multiProcessorCount, b->workgroups, std::max(count - b->split, 1)});
    b->order = order;
    b->nq.assign(n, n + count);

    qk::BatchArgs &A = b->args;
    qaoa_status st;
    int32_t *d_order, *d_n, *d_edges, *d_npass;
    int64_t *d_eoff;
    double *d_w = nullptr, *d_scale, *d_g, *d_b, *d_e0, *d_e1, *d_cost;
    qk::Geometry *d_geo;
    double2 *d_psi, *d_lam;
    uint32_t *d_cnt;
    uint64_t *d_ticks;
    if ((st = upload(b, &d_order, order.data(), count)) != QAOA_OK ||
        (st = upload(b, &d_n, n, count)) != QAOA_OK ||
        (st = upload(b, &d_eoff, edge_offsets, (size_t)count + 1)) != QAOA_OK ||
        (st = upload(b, &d_edges, edges, (size_t)E * 2)) != QAOA_OK ||
        (w && (st = upload(b, &d_w, w, (size_t)E)) != QAOA_OK) ||
        (st = upload(b, &d_scale, scale.data(), count)) != QAOA_OK ||
        (st = upload<double>(b, &d_g, nullptr, (size_t)count * p)) != QAOA_OK ||
        (st = upload<double>(b, &d_b, nullptr, (size_t)count * p)) != QAOA_OK ||
        (st = upload<double>(b, &d_e0, nullptr, count)) != QAOA_OK ||
        (st = upload<double>(b, &d_e1, nullptr, count)) != QAOA_OK ||
        (st = upload(b, &d_geo, geo.data(), geo.size())) != QAOA_OK ||
        (st = upload(b, &d_npass, npass.data(), npass.size())) != QAOA_OK ||
        (st = upload<double2>(b, &d_psi, nullptr, (size_t)b->workgroups * slot)) != QAOA_OK ||
        (st = upload<double2>(b, &d_lam, nullptr, (size_t)b->workgroups * slot)) != QAOA_OK ||
        (st = upload<double>(b, &d_cost, nullptr, (size_t)b->workgroups * slot)) != QAOA_OK ||
        (st = upload<uint32_t>(b, &d_cnt, nullptr, 2)) != QAOA_OK ||
        (st = upload<uint64_t>(b, &d_ticks, nullptr, (size_t)count * 2)) != QAOA_OK)
        return cleanup(st);
    A.count = count;
    A.begin = 0;
    A.end = b->split;
    A.ticks = d_ticks;
    A.order = d_order;
    A.nq = d_n;
    A.eoff = d_eoff;
    A.edges = d_edges;
    A.w = d_w;
    A.scale = d_scale;
    A.gamma = d_g;
    A.beta = d_b;
    A.e_first = d_e0;
    A.e_last = d_e1;
    A.p = p;
    A.steps = o.steps;
    A.lr = o.lr;
    A.b1 = o.beta1;
    A.b2 = o.beta2;
    A.eps = o.eps;
    A.geo = d_geo;
    A.npass = d_npass;
    A.psi = d_psi;
    A.lam = d_lam;
    A.cost = d_cost;
    A.slot = slot;
    A.counter = d_cnt;
    b->args_res = A;
    b->args_res.begin = b->split;
    b->args_res.end = count;
    b->args_res.counter = d_cnt + 1;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return cleanup(bfail(QAOA_ERR_DEVICE, "upload failed"));

    if (b->use_graph) {
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return cleanup(bfail(QAOA_ERR_DEVICE, "graph capture failed"));
        st = launch_engine(b);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(b->stream, &gr);
        b->graph = gr;
        if (st != QAOA_OK) return cleanup(st);
        if (e != hipSuccess || hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
            return cleanup(bfail(QAOA_ERR_DEVICE, "graph instantiation failed"));
    }
    *out = b;
    return QAOA_OK;
}

qaoa_status qaoa_batch_run(qaoa_batch b, const double *gamma0, const double *beta0, double *gamma,
                           double *beta, double *e_first, double *e_last)
{
    if (!b) return bfail(QAOA_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (b->poisoned) return bfail(QAOA_ERR_DEVICE, "batch is unusable after an earlier device error");
    if (!gamma0 || !beta0) return bfail(QAOA_ERR_INVALID_ARGUMENT, "start angles are NULL");
    const size_t np = (size_t)b->count * b->p;
    for (size_t i = 0; i < np; ++i)
        if (!std::isfinite(gamma0[i]) || !std::isfinite(beta0[i]))
            return bfail(QAOA_ERR_INVALID_ARGUMENT, "angles must be finite");
    // the batch's device is current for the call and the caller's restored after it
    struct DeviceScope {
        int old = -1;
        explicit DeviceScope(int dev)
        {
            if (hipGetDevice(&old) != hipSuccess) old = -1;
            if (old != dev) (void)hipSetDevice(dev);
        }
        ~DeviceScope()
        {
            int cur = -1;
            if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
        }
    } scope(b->device);
    qk::BatchArgs &A = b->args;
    BCHECK(b, hipMemcpyAsync(A.gamma, gamma0, np * 8, hipMemcpyHostToDevice, b->stream));
    BCHECK(b, hipMemcpyAsync(A.beta, beta0, np * 8, hipMemcpyHostToDevice, b->stream));
    if (b->use_graph) {
        BCHECK(b, hipGraphLaunch(b->exec, b->stream));
    } else {
        qaoa_status st = launch_engine(b);
        if (st != QAOA_OK) return st;
    }
    if (gamma) BCHECK(b, hipMemcpyAsync(gamma, A.gamma, np * 8, hipMemcpyDeviceToHost, b->stream));
    if (beta) BCHECK(b, hipMemcpyAsync(beta, A.beta, np * 8, hipMemcpyDeviceToHost, b->stream));
    if (e_first) BCHECK(b, hipMemcpyAsync(e_first, A.e_first, b->count * 8, hipMemcpyDeviceToHost, b->stream));
    if (e_last) BCHECK(b, hipMemcpyAsync(e_last, A.e_last, b->count * 8, hipMemcpyDeviceToHost, b->stream));
    BCHECK(b, hipStreamSynchronize(b->stream));
    b->ran = true;
    return QAOA_OK;
}

qaoa_status qaoa_batch_timeline(qaoa_batch b, double *start_s, double *end_s, int32_t *which_launch)
{
    if (!b) return bfail(QAOA_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (!b->ran) return bfail(QAOA_ERR_INVALID_ARGUMENT, "the batch has not run yet");
    if (b->poisoned) return bfail(QAOA_ERR_DEVICE, "batch is unusable after an earlier device error");
    int rate_khz = 0;
    BCHECK(b, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->device));
    if (rate_khz <= 0) return bfail(QAOA_ERR_DEVICE, "device wall clock rate unknown");
    std::vector<uint64_t> t((size_t)b->count * 2);
    BCHECK(b, hipMemcpyAsync(t.data(), b->args.ticks, t.size() * 8, hipMemcpyDeviceToHost, b->stream));
    BCHECK(b, hipStreamSynchronize(b->stream));
    uint64_t t0 = ~0ull;
    for (int i = 0; i < b->count; ++i) t0 = std::min(t0, t[2 * (size_t)i]);
    const double tick = 1.0 / (1e3 * (double)rate_khz);
    std::vector<int32_t> which(b->count, 0);
    for (int k = b->split; k < b->count; ++k) which[b->order[k]] = 1;
    for (int i = 0; i < b->count; ++i) {
        if (start_s) start_s[i] = (double)(int64_t)(t[2 * (size_t)i] - t0) * tick;
        if (end_s) end_s[i] = (double)(int64_t)(t[2 * (size_t)i + 1] - t0) * tick;
        if (which_launch) which_launch[i] = which[i];
    }
    return QAOA_OK;
}

qaoa_status qaoa_batch_destroy(qaoa_batch b)
{
    if (!b) return QAOA_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : b->allocs) (void)hipFree(p);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return QAOA_OK;
}

}  // extern "C"
