// C ABI of the QAOA statevector library (declared in include/qaoa.h).
//
// Host runtime: argument validation (always before any HIP call), the handle
// and its lazily allocated buffers (Sec. IV-B), the pass plan that groups the
// n mixer rotations of a layer into tile passes, and the launch sequences for
// the state, the expectation, the adjoint gradient and sampling.
#include "qaoa.h"
#include "qaoa_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

void set_err(const char *fmt, const char *a = "", long long b = 0)
{
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    g_err = buf;
}

qaoa_status fail(qaoa_status st, const char *msg)
{
    g_err = msg;
    return st;
}

}  // namespace

namespace qk {
void set_error_message(const std::string &m) { g_err = m; }
std::string error_message() { return g_err; }
}  // namespace qk

struct qaoa_handle_s {
    int n = 0;
    int prec = QAOA_C128;
    int device = 0;
    uint64_t N = 0;
    qaoa_allocator alloc{};  // device-memory provider (alloc == NULL: hipMalloc / hipFree)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *psi = nullptr;   // state, 2^n amplitudes
    void *lam = nullptr;   // adjoint vector, allocated on first gradient
    void *cost = nullptr;  // cost diagonal, fp64 (c128) or fp32 (c64)
    double cost_bound = 0; // |offset| + sum of |weights|: bounds |C(z)|
    double *parts = nullptr;
    size_t parts_cap = 0;  // doubles
    double *res = nullptr;
    size_t res_cap = 0;    // doubles
    std::vector<qk::PassPlan> plan;  // mixer sweeps of one layer (fixed by n and precision)
    bool state_valid = false;
    std::vector<double> state_angles;  // (gamma, beta) of the current state
    bool poisoned = false;
    bool extrema_valid = false;
    double cmin = 0, cmax = 0;
    // Kernel timing: event pairs bracketing pass launches, drained on read.
    bool profiling = false;
    struct Pending {
        int kind;
        double bytes;
        hipEvent_t t0, t1;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    // per pass kind: forward, turn, backward, layer-boundary forward, layer-boundary backward
    int64_t prof_launches[5] = {0, 0, 0, 0, 0};
    double prof_ms[5] = {0, 0, 0, 0, 0};
    double prof_bytes[5] = {0, 0, 0, 0, 0};
};

namespace {

thread_local qaoa_allocator g_alloc{};  // allocator for handles created on this thread

// Device allocation through the handle's allocator.
hipError_t dev_alloc(qaoa_handle h, void **p, size_t bytes)
{
    if (!h->alloc.alloc) return hipMalloc(p, bytes);
    *p = h->alloc.alloc(bytes, (void *)h->stream, h->alloc.user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(qaoa_handle h, void *p, size_t bytes)
{
    if (!p) return;
    if (!h->alloc.alloc) (void)hipFree(p);
    else h->alloc.free(p, bytes, (void *)h->stream, h->alloc.user);
}

// Free device memory for a buffer of `bytes`, or true when an allocator
// provides the memory (it reports failure itself).
bool fits(qaoa_handle h, double bytes, size_t fr) { return h->alloc.alloc || bytes <= (double)fr; }

}  // namespace


namespace {

struct DeviceGuard {
    int old = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) {
            ok = false;
            return;
        }
        if (old != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

qaoa_status device_fail(qaoa_handle h, const char *what, hipError_t e)
{
    if (h) h->poisoned = true;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
    g_err = buf;
    return QAOA_ERR_DEVICE;
}

#define HIPCHECK(h, call)                                              \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return device_fail((h), #call, e_);      \
    } while (0)

inline size_t amp_bytes(int prec) { return prec == QAOA_C64 ? 8 : 16; }
inline size_t cost_bytes(int prec) { return prec == QAOA_C64 ? 4 : 8; }
inline bool c64(const qaoa_handle h) { return h->prec == QAOA_C64; }
// Workgroups (tiles) of a pass kernel launch.
inline uint64_t nblocks(int n, bool c64)
{
    const int tb = qk::tile_bits(c64);
    return n <= tb ? 1ull : (1ull << (n - tb));
}
inline uint64_t nblocks(const qaoa_handle h) { return nblocks(h->n, c64(h)); }

qaoa_status check_handle(qaoa_handle h)
{
    if (!h) return fail(QAOA_ERR_INVALID_ARGUMENT, "handle is NULL");
    if (h->poisoned) return fail(QAOA_ERR_DEVICE, "handle is unusable after an earlier device error");
    return QAOA_OK;
}

qaoa_status check_angles(int32_t p, const double *gamma, const double *beta)
{
    if (p < 0) return fail(QAOA_ERR_INVALID_ARGUMENT, "p must be >= 0");
    if (p > 0 && (!gamma || !beta)) return fail(QAOA_ERR_INVALID_ARGUMENT, "gamma/beta is NULL");
    for (int i = 0; i < p; ++i)
        if (!std::isfinite(gamma[i]) || !std::isfinite(beta[i]))
            return fail(QAOA_ERR_INVALID_ARGUMENT, "angles must be finite");
    return QAOA_OK;
}

qaoa_status check_terms(int32_t n, int64_t m, const int32_t *idx, const double *w, bool w_required)
{
    if (n < 1 || n > QAOA_MAX_QUBITS)
        return fail(QAOA_ERR_INVALID_ARGUMENT, "n must be in [1, QAOA_MAX_QUBITS]");
    if (m < 0) return fail(QAOA_ERR_INVALID_ARGUMENT, "m must be >= 0");
    if (m > 0 && !idx) return fail(QAOA_ERR_INVALID_ARGUMENT, "index array is NULL");
    if (m > 0 && w_required && !w) return fail(QAOA_ERR_INVALID_ARGUMENT, "weight array is NULL");
    for (int64_t k = 0; k < m; ++k) {
        const int32_t i = idx[2 * k], j = idx[2 * k + 1];
        if (i < 0 || i >= n || j < 0 || j >= n) {
            set_err("term %s%lld has a variable index outside [0, n)", "", (long long)k);
            return QAOA_ERR_INVALID_ARGUMENT;
        }
        if (i == j) {
            set_err("term %s%lld joins a variable to itself", "", (long long)k);
            return QAOA_ERR_INVALID_ARGUMENT;
        }
        if (w && !std::isfinite(w[k])) return fail(QAOA_ERR_INVALID_ARGUMENT, "weights must be finite");
    }
    return QAOA_OK;
}

// Ensure `*buf` holds at least `count` doubles.
qaoa_status ensure_doubles(qaoa_handle h, double **buf, size_t *cap, size_t count)
{
    if (*cap >= count) return QAOA_OK;
    if (*buf) {
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        dev_free(h, *buf, *cap * sizeof(double));
    }
    *buf = nullptr;
    *cap = 0;
    size_t fr = 0, tot = 0;
    HIPCHECK(h, hipMemGetInfo(&fr, &tot));
    if (!fits(h, (double)count * sizeof(double), fr))
        return fail(QAOA_ERR_OUT_OF_MEMORY, "scratch buffer does not fit");
    if (dev_alloc(h, (void **)buf, count * sizeof(double)) != hipSuccess)
        return fail(QAOA_ERR_OUT_OF_MEMORY, "scratch buffer allocation failed");
    *cap = count;
    return QAOA_OK;
}

// Kernel arguments of one pass over plan entry `pp` with mixer angle `beta`.
qk::PassArgs pass_args(qaoa_handle h, const qk::PassPlan &pp, double beta)
{
    qk::PassArgs a;
    std::memset(&a, 0, sizeof a);
    a.psi = h->psi;
    a.lam = h->lam;
    a.cost = h->cost;
    qk::make_geometry(h->n, pp, &a.geo);  // plans are validated when made
    // Nontemporal accesses pay off for runs of >= 64 consecutive amplitudes; for
    // short runs the L2 must keep each line for the neighbouring tile.
    if (a.geo.t_dst[0] == 0 && a.geo.t_len[0] >= 6) a.flags |= qk::kStream;
    // Send 16 consecutive tiles (adjacent runs, shared lines and DRAM rows) to one XCD.
    a.xcd_g = qk::xcd_group_bits(nblocks(h), 4);
    a.amp0 = 1.0 / std::sqrt((double)h->N);
    // Factored rotations: exp(-i b X) = f (p I - i q X) with the larger of
    // |cos b|, |sin b| as f, so the non-unit coefficient has magnitude <= 1.
    const double c = std::cos(beta), s = std::sin(beta);
    const int k = __builtin_popcount(a.geo.tmask);
    a.tan_mode = std::fabs(c) >= std::fabs(s) ? 1u : 0u;
    if (a.tan_mode) {
        a.mul_f = s / c;
        a.mul_b = -s / c;
        a.fac_f = c;
        a.fac_b = c;
    } else {
        a.mul_f = c / s;
        a.mul_b = -c / s;
        a.fac_f = s;
        a.fac_b = -s;
    }
    a.scl_f = a.scl_b = 1.0;
    for (int i = 0; i < k; ++i) {
        a.scl_f *= a.fac_f;
        a.scl_b *= a.fac_b;
    }
    return a;
}

// Second rotation of a layer-boundary pass (kFwdFuse / kBwdFuse): the same
// factored form for the other layer's angle on the same target qubits.
void set_second(qk::PassArgs &a, double beta2)
{
    const double c = std::cos(beta2), s = std::sin(beta2);
    const int k = __builtin_popcount(a.geo.tmask);
    a.tan_mode2 = std::fabs(c) >= std::fabs(s) ? 1u : 0u;
    double ff, fb;
    if (a.tan_mode2) {
        a.mul_f2 = s / c;
        a.mul_b2 = -s / c;
        ff = fb = c;
    } else {
        a.mul_f2 = c / s;
        a.mul_b2 = -c / s;
        ff = s;
        fb = -s;
    }
    a.fac_b2 = fb;
    a.scl_f2 = a.scl_b2 = 1.0;
    for (int i = 0; i < k; ++i) {
        a.scl_f2 *= ff;
        a.scl_b2 *= fb;
    }
}

// Mixer group visited at position idx of layer l: even layers ascending, odd
// layers descending, so that consecutive layers meet on one shared group.
int group_at(int l, int idx, int P) { return (l % 2 == 0) ? idx : P - 1 - idx; }

// Bytes a pass must move at minimum: each amplitude vector it reads and/or
// writes once, plus one read of the cost diagonal when it applies or measures C.
double pass_bytes(qaoa_handle h, int mode, const qk::PassArgs &a)
{
    const double N = (double)h->N, s = (double)amp_bytes(h->prec), c = (double)cost_bytes(h->prec);
    const bool store = !(a.flags & qk::kNoStore);
    const bool initd = (a.flags & qk::kInit) != 0;
    if (mode == qk::kFwd)
        return N * ((initd ? 0 : s) + (store ? s : 0) +
                    ((a.flags & (qk::kPhaseIn | qk::kEOut)) ? c : 0));
    if (mode == qk::kTurn || mode == qk::kTurnPhase) return N * ((initd ? 0 : s) + c + (store ? s : 0));
    if (mode == qk::kFwdFuse) return N * (2 * s + c);
    if (mode == qk::kBwdFuse) return N * (4 * s + c);
    return N * (2 * s + (store ? 2 * s : 0) + ((a.flags & qk::kPhaseOut) ? c : 0));
}

qaoa_status take_event(qaoa_handle h, hipEvent_t *ev)
{
    if (!h->event_pool.empty()) {
        *ev = h->event_pool.back();
        h->event_pool.pop_back();
        return QAOA_OK;
    }
    HIPCHECK(h, hipEventCreate(ev));
    return QAOA_OK;
}

qaoa_status run_pass(qaoa_handle h, int mode, const qk::PassArgs &args)
{
    // passes whose phase arguments |gamma C| could leave the fast reduction's
    // range are marked (the unused gamma fields are 0)
    qk::PassArgs a = args;
    if (std::max(std::fabs(a.gamma_in), std::fabs(a.gamma_out)) * h->cost_bound >= qk::near_phase_limit(c64(h)))
        a.flags |= qk::kFarPhase;
    if (!h->profiling) {
        HIPCHECK(h, qk::launch_pass(mode, c64(h), a, nblocks(h), h->stream));
        return QAOA_OK;
    }
    // reported kinds: 0 forward, 1 turn, 2 backward, 3 / 4 layer-boundary forward / backward
    const int kind = mode == qk::kFwd ? 0 : (mode == qk::kTurn || mode == qk::kTurnPhase) ? 1
                     : mode == qk::kBwd ? 2 : mode == qk::kFwdFuse ? 3 : 4;
    qaoa_handle_s::Pending pd{kind, pass_bytes(h, mode, a), nullptr, nullptr};
    qaoa_status st = take_event(h, &pd.t0);
    if (st == QAOA_OK) st = take_event(h, &pd.t1);
    if (st != QAOA_OK) return st;
    HIPCHECK(h, hipEventRecord(pd.t0, h->stream));
    HIPCHECK(h, qk::launch_pass(mode, c64(h), a, nblocks(h), h->stream));
    HIPCHECK(h, hipEventRecord(pd.t1, h->stream));
    h->pending.push_back(pd);
    return QAOA_OK;
}

qaoa_status drain_profile(qaoa_handle h)
{
    if (h->pending.empty()) return QAOA_OK;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    for (auto &pd : h->pending) {
        float ms = 0.f;
        HIPCHECK(h, hipEventElapsedTime(&ms, pd.t0, pd.t1));
        h->prof_launches[pd.kind] += 1;
        h->prof_ms[pd.kind] += ms;
        h->prof_bytes[pd.kind] += pd.bytes;
        h->event_pool.push_back(pd.t0);
        h->event_pool.push_back(pd.t1);
    }
    h->pending.clear();
    return QAOA_OK;
}

// Forward evolution through layers [0, p); the last `skip_last` groups of the
// last layer are left out (the gradient's turn pass runs the last group).
// With `e_out`, the final pass accumulates E into partial slot 0.
qaoa_status run_forward(qaoa_handle h, int p, const double *gamma, const double *beta,
                        bool skip_last, bool e_out)
{
    const std::vector<qk::PassPlan> &G = h->plan;
    const int P = (int)G.size();
    for (int l = 0; l < p; ++l) {
        for (int idx = 0; idx < P; ++idx) {
            // with P >= 2, a layer's first group was applied by the previous
            // layer's last (layer-boundary) pass
            if (P > 1 && l > 0 && idx == 0) continue;
            const bool last = idx == P - 1;
            if (last && l == p - 1 && skip_last) break;  // the gradient's turn pass
            const int gi = P > 1 ? group_at(l, idx, P) : 0;
            qk::PassArgs a = pass_args(h, G[gi], beta[l]);
            if (P > 1 && last && l < p - 1) {
                set_second(a, beta[l + 1]);
                a.gamma_in = gamma[l + 1];
                qaoa_status st = run_pass(h, qk::kFwdFuse, a);
                if (st != QAOA_OK) return st;
                continue;
            }
            if (idx == 0) {
                a.flags |= qk::kPhaseIn;
                a.gamma_in = gamma[l];
                if (l == 0) a.flags |= qk::kInit;
            }
            if (e_out && l == p - 1 && last) {
                a.flags |= qk::kEOut;
                a.part_e = h->parts;
            }
            qaoa_status st = run_pass(h, qk::kFwd, a);
            if (st != QAOA_OK) return st;
        }
    }
    return QAOA_OK;
}

// Partial-sum slots of a gradient: (2p + 1) x nblocks doubles, slot 0 E,
// slots 1 .. p the <lam|X|phi> terms of layers 0 .. p-1, slots p+1 .. 2p their
// <lam|C|phi> terms.
struct Slots {
    double *parts;
    uint64_t T;
    int p;
    double *E() const { return parts; }
    double *B(int l) const { return parts + (uint64_t)(1 + l) * T; }
    double *G(int l) const { return parts + (uint64_t)(1 + p + l) * T; }
};

// Backward sweep after the last group of layer p-1 has been undone (by the
// turn pass or by the first pass of a reverse sweep from a stored state): each
// layer undoes its groups in the reverse of the forward order; a layer's first
// group also undoes its phase and, for P >= 2 and l > 0, shares its sweep with
// the last group of layer l - 1.  Partials of <lam|X|phi>: with P >= 2 a
// layer's slot has already been written when its own passes run (by the pass
// that undid layer p-1's last group, or by the layer-boundary sweep of layer
// l+1), so they add to it, and a layer-boundary sweep is always the first to
// touch layer l-1's slot, so it overwrites it; with P = 1 every layer but the
// last has one pass, which overwrites.
qaoa_status enqueue_backward(qaoa_handle h, int p, const double *gamma, const double *beta, void *lam,
                             const Slots &sl)
{
    const std::vector<qk::PassPlan> &G = h->plan;
    const int P = (int)G.size();
    for (int l = p - 1; l >= 0; --l) {
        for (int j = 0; j < P; ++j) {
            const int idx = P - 1 - j;
            if (j == 0 && (l == p - 1 || P > 1)) continue;  // undone already, or fused into layer l+1
            const int gi = P > 1 ? group_at(l, idx, P) : 0;
            qk::PassArgs a = pass_args(h, G[gi], beta[l]);
            a.lam = lam;
            a.part_b = sl.B(l);
            if (P > 1) a.flags |= qk::kBetaAcc;
            int mode = qk::kBwd;
            if (idx == 0) {
                a.gamma_out = gamma[l];
                a.part_g = sl.G(l);
                if (P > 1 && l > 0) {
                    mode = qk::kBwdFuse;
                    set_second(a, beta[l - 1]);
                    a.part_b2 = sl.B(l - 1);
                } else {
                    a.flags |= qk::kPhaseOut;
                    if (l == 0) a.flags |= qk::kNoStore;
                }
            }
            qaoa_status st = run_pass(h, mode, a);
            if (st != QAOA_OK) return st;
        }
    }
    return QAOA_OK;
}

// Launch sequence of the expectation and its adjoint gradient (Sec. II-B,
// IV-C) on the handle's stream: forward sweeps, the turn sweep, backward
// sweeps.  `lam` is the adjoint vector (2^n amplitudes) and `parts` holds the
// (2p + 1) x nblocks partial sums (Slots).  Every slot is overwritten before it
// is added to, so neither buffer needs clearing.  Only enqueues kernels
// (p >= 1); allocates nothing.
qaoa_status enqueue_gradient(qaoa_handle h, int p, const double *gamma, const double *beta, void *lam,
                             double *parts)
{
    qaoa_status st;
    const Slots sl{parts, nblocks(h), p};
    const std::vector<qk::PassPlan> &G = h->plan;
    const int P = (int)G.size();

    // Forward through every group except the last group of the last layer.
    if ((st = run_forward(h, p, gamma, beta, true, false)) != QAOA_OK) return st;

    // Turn pass: last group of layer p-1 forward, E, lam = C phi, group undone on lam.
    {
        const int l = p - 1;
        qk::PassArgs a = pass_args(h, G[P > 1 ? group_at(l, P - 1, P) : 0], beta[l]);
        a.lam = lam;
        a.part_e = sl.E();
        a.part_b = sl.B(l);
        if (P == 1) {
            a.flags |= qk::kPhaseIn | qk::kPhaseOut;
            a.gamma_in = a.gamma_out = gamma[l];
            a.part_g = sl.G(l);
            if (l == 0) a.flags |= qk::kInit | qk::kNoStore;
        }
        if ((st = run_pass(h, P == 1 ? qk::kTurnPhase : qk::kTurn, a)) != QAOA_OK) return st;
    }
    return enqueue_backward(h, p, gamma, beta, lam, sl);
}

// Reverse sweep from the final state phi(gamma, beta) held in psi: the first
// backward pass forms lam = C phi as it loads phi, undoes the last group of
// layer p-1 on both vectors with its <lam|X|phi> terms (and, with one group
// per layer, the phase with the <lam|C|phi> term) and stores both; the rest is
// the gradient's backward sweep.  Slot 0 (E) is not written.
qaoa_status enqueue_reverse(qaoa_handle h, int p, const double *gamma, const double *beta, void *lam,
                            double *parts)
{
    const Slots sl{parts, nblocks(h), p};
    const std::vector<qk::PassPlan> &G = h->plan;
    const int P = (int)G.size();
    const int l = p - 1;
    qk::PassArgs a = pass_args(h, G[P > 1 ? group_at(l, P - 1, P) : 0], beta[l]);
    a.lam = lam;
    a.part_b = sl.B(l);
    a.flags |= qk::kLamFromC;
    if (P == 1) {
        a.flags |= qk::kPhaseOut;
        a.gamma_out = gamma[l];
        a.part_g = sl.G(l);
        if (l == 0) a.flags |= qk::kNoStore;
    }
    qaoa_status st = run_pass(h, qk::kBwd, a);
    if (st != QAOA_OK) return st;
    return enqueue_backward(h, p, gamma, beta, lam, sl);
}

// Records the angles of the state just computed (qaoa_gradient_from_state
// checks them).
qaoa_status keep_angles(qaoa_handle h, int p, const double *gamma, const double *beta)
{
    try {
        h->state_angles.assign(gamma, gamma + p);
        h->state_angles.insert(h->state_angles.end(), beta, beta + p);
    } catch (...) {
        return fail(QAOA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    return QAOA_OK;
}

// Adjoint vector of the handle, allocated on first use.
qaoa_status ensure_lam(qaoa_handle h)
{
    if (h->lam) return QAOA_OK;
    size_t fr = 0, tot = 0;
    HIPCHECK(h, hipMemGetInfo(&fr, &tot));
    if (!fits(h, (double)h->N * amp_bytes(h->prec), fr))
        return fail(QAOA_ERR_OUT_OF_MEMORY, "adjoint vector does not fit in free device memory");
    if (dev_alloc(h, &h->lam, h->N * amp_bytes(h->prec)) != hipSuccess)
        return fail(QAOA_ERR_OUT_OF_MEMORY, "adjoint vector allocation failed");
    return QAOA_OK;
}

qaoa_status fetch_results(qaoa_handle h, int nslots, uint64_t count, double *host)
{
    HIPCHECK(h, qk::launch_sum_slots(h->parts, count, count, nslots, h->res, h->stream));
    HIPCHECK(h, hipMemcpyAsync(host, h->res, (size_t)nslots * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return QAOA_OK;
}

qaoa_status create_common(int32_t n, int32_t precision, void *stream, qaoa_handle *out,
                          qaoa_handle *hh)
{
    if (!out) return fail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    if (precision != QAOA_C128 && precision != QAOA_C64)
        return fail(QAOA_ERR_INVALID_ARGUMENT, "unknown precision");
    qaoa_handle h = new (std::nothrow) qaoa_handle_s();
    if (!h) return fail(QAOA_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->n = n;
    h->prec = precision;
    h->N = 1ull << n;
    h->alloc = g_alloc;
    try {
        h->plan = qk::plan_passes(n, precision == QAOA_C64);
    } catch (...) {
        delete h;
        return fail(QAOA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return device_fail(nullptr, "hipGetDevice", e);
    }
    size_t fr = 0, tot = 0;
    e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) {
        delete h;
        return device_fail(nullptr, "hipMemGetInfo", e);
    }
    const double need = (double)h->N * (double)(amp_bytes(precision) + cost_bytes(precision)) +
                        (double)nblocks(n, precision == QAOA_C64) * 8.0 * 2 + (1 << 20);
    if (!fits(h, need, fr)) {
        delete h;
        return fail(QAOA_ERR_OUT_OF_MEMORY, "state and cost diagonal do not fit in free device memory");
    }
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return device_fail(nullptr, "hipStreamCreateWithFlags", e);
        }
        h->own_stream = true;
    }
    *hh = h;
    if ((e = dev_alloc(h, &h->psi, h->N * amp_bytes(precision))) != hipSuccess ||
        (e = dev_alloc(h, &h->cost, h->N * cost_bytes(precision))) != hipSuccess) {
        qaoa_destroy(h);
        *hh = nullptr;
        if (e == hipErrorOutOfMemory) return fail(QAOA_ERR_OUT_OF_MEMORY, "state or cost allocation failed");
        return device_fail(nullptr, "hipMalloc", e);
    }
    qaoa_status st = ensure_doubles(h, &h->parts, &h->parts_cap, 2 * nblocks(n, precision == QAOA_C64) + 2);
    if (st == QAOA_OK) st = ensure_doubles(h, &h->res, &h->res_cap, 64);
    if (st != QAOA_OK) {
        std::string keep = g_err;
        qaoa_destroy(h);
        *hh = nullptr;
        g_err = keep;
        return st;
    }
    return QAOA_OK;
}

// Uploads the cost pieces (through the handle's allocator), builds the cost
// diagonal, frees the upload once the stream has drained.
qaoa_status build_cost(qaoa_handle h, const std::vector<qk::CostPiece> &pieces, double offset)
{
    h->cost_bound = std::fabs(offset);
    for (const qk::CostPiece &pc : pieces) h->cost_bound += std::fabs(pc.w);
    const size_t bytes = pieces.size() * sizeof(qk::CostPiece);
    void *dev = nullptr;
    if (bytes) {
        hipError_t e = dev_alloc(h, &dev, bytes);
        if (e == hipErrorOutOfMemory || (e == hipSuccess && !dev))
            return fail(QAOA_ERR_OUT_OF_MEMORY, "term upload buffer allocation failed");
        if (e != hipSuccess) return device_fail(h, "term upload allocation", e);
    }
    qaoa_status st = QAOA_OK;
    hipError_t e = hipSuccess;
    if (bytes) e = hipMemcpyAsync(dev, pieces.data(), bytes, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = qk::launch_cost_pieces(c64(h), h->cost, h->n, (const qk::CostPiece *)dev,
                                   (int64_t)pieces.size(), offset, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        st = device_fail(h, "cost diagonal", e);
        (void)hipStreamSynchronize(h->stream);  // queued work must finish before the free
    }
    dev_free(h, dev, bytes);
    return st;
}

// Builds the pieces of a cost (host vectors; a failed allocation is reported).
template <typename Make>
qaoa_status make_pieces(std::vector<qk::CostPiece> *out, Make make)
{
    try {
        *out = make();
    } catch (...) {
        return fail(QAOA_ERR_OUT_OF_MEMORY, "host allocation of the cost terms failed");
    }
    return QAOA_OK;
}

// Creates the handle and its cost diagonal from pieces; on error nothing is left.
qaoa_status create_with_pieces(int32_t n, int32_t precision, void *stream, qaoa_handle *out,
                               const std::vector<qk::CostPiece> &pieces, double offset)
{
    qaoa_handle h = nullptr;
    qaoa_status st = create_common(n, precision, stream, out, &h);
    if (st != QAOA_OK) return st;
    st = build_cost(h, pieces, offset);
    if (st != QAOA_OK) {
        std::string keep = g_err;
        qaoa_destroy(h);
        g_err = keep;
        return st;
    }
    *out = h;
    return QAOA_OK;
}

}  // namespace

namespace qk {

int handle_device(qaoa_handle h) { return h->device; }

size_t noalloc_need(qaoa_handle h, int p)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    if (p == 0) return al((size_t)((h->N + kTile - 1) / kTile) * sizeof(double)) + sizeof(double);
    const size_t nslots = 2 * (size_t)p + 1;
    return al(h->N * amp_bytes(h->prec)) + al(nslots * nblocks(h) * sizeof(double)) + nslots * sizeof(double);
}

qaoa_status noalloc_check(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                          const double *dgamma, const double *dbeta, size_t cap)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if ((st = check_angles(p, gamma, beta)) != QAOA_OK) return st;
    if (p > kNoAllocMaxLayers) return fail(QAOA_ERR_INVALID_ARGUMENT, "p exceeds the no-allocation limit of 32 layers");
    if (p > 0 && (!dgamma || !dbeta)) return fail(QAOA_ERR_INVALID_ARGUMENT, "gradient output is NULL");
    if (noalloc_need(h, p) > cap) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "n = %d needs %zu bytes of scratch, more than the %zu of the no-allocation gradient",
                      h->n, noalloc_need(h, p), cap);
        g_err = buf;
        return QAOA_ERR_INVALID_ARGUMENT;
    }
    return QAOA_OK;
}

qaoa_status gradient_on_scratch(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                                double *E, double *dgamma, double *dbeta, int32_t out_is_device,
                                void *scratch)
{
    DeviceGuard dg(h->device);
    if (!dg.ok) return device_fail(h, "hipSetDevice", hipErrorInvalidDevice);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *base = (char *)scratch;
    h->state_valid = false;
    // No timing events here (creating them may allocate); restored on every path.
    struct ProfOff {
        qaoa_handle h;
        bool was;
        ~ProfOff() { h->profiling = was; }
    } prof{h, h->profiling};
    h->profiling = false;
    double *res;
    int nslots;
    if (p == 0) {
        const uint64_t T0 = (h->N + kTile - 1) / kTile;
        double *parts = (double *)base;
        res = (double *)(base + al(T0 * sizeof(double)));
        nslots = 1;
        HIPCHECK(h, launch_fill_plus(c64(h), h->psi, h->n, h->stream));
        HIPCHECK(h, launch_expect(c64(h), h->psi, h->cost, h->n, parts, h->stream));
        HIPCHECK(h, launch_sum_slots(parts, T0, T0, 1, res, h->stream));
    } else {
        const uint64_t T = nblocks(h);
        nslots = 2 * p + 1;
        void *lam = base;
        double *parts = (double *)(base + al(h->N * amp_bytes(h->prec)));
        res = (double *)((char *)parts + al((size_t)nslots * T * sizeof(double)));
        qaoa_status st = enqueue_gradient(h, p, gamma, beta, lam, parts);
        if (st != QAOA_OK) return st;
        HIPCHECK(h, launch_sum_slots(parts, T, T, nslots, res, h->stream));
    }
    if (out_is_device) {
        HIPCHECK(h, launch_gradient_out(res, p, E, dgamma, dbeta, h->stream));
        return QAOA_OK;
    }
    double r[2 * kNoAllocMaxLayers + 1];
    HIPCHECK(h, hipMemcpyAsync(r, res, (size_t)nslots * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    if (E) *E = r[0];
    for (int l = 0; l < p; ++l) {
        dbeta[l] = 2.0 * r[1 + l];
        dgamma[l] = 2.0 * r[1 + p + l];
    }
    return QAOA_OK;
}

}  // namespace qk

extern "C" {

qaoa_status qaoa_create_maxcut(int32_t n, int64_t m, const int32_t *edges, const double *w,
                               int32_t precision, void *stream, qaoa_handle *out)
{
    qaoa_status st = check_terms(n, m, edges, w, false);
    if (st != QAOA_OK) return st;
    if (!out) return fail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    std::vector<qk::CostPiece> pieces;
    if ((st = make_pieces(&pieces, [&] { return qk::cost_pieces_maxcut(m, edges, w); })) != QAOA_OK)
        return st;
    return create_with_pieces(n, precision, stream, out, pieces, 0.0);
}

qaoa_status qaoa_create_qubo(int32_t n, int64_t m, const int32_t *pairs, const double *J,
                             const double *hl, double offset, int32_t precision, void *stream,
                             qaoa_handle *out)
{
    qaoa_status st = check_terms(n, m, pairs, J, true);
    if (st != QAOA_OK) return st;
    if (!std::isfinite(offset)) return fail(QAOA_ERR_INVALID_ARGUMENT, "offset must be finite");
    if (hl)
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(hl[i])) return fail(QAOA_ERR_INVALID_ARGUMENT, "h must be finite");
    if (!out) return fail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    std::vector<qk::CostPiece> pieces;
    if ((st = make_pieces(&pieces, [&] { return qk::cost_pieces_qubo(n, m, pairs, J, hl); })) != QAOA_OK)
        return st;
    return create_with_pieces(n, precision, stream, out, pieces, offset);
}

qaoa_status qaoa_create_poly(int32_t n, int64_t L, const uint64_t *masks, const double *w,
                             double offset, int32_t precision, void *stream, qaoa_handle *out)
{
    if (n < 1 || n > QAOA_MAX_QUBITS)
        return fail(QAOA_ERR_INVALID_ARGUMENT, "n must be in [1, QAOA_MAX_QUBITS]");
    if (L < 0) return fail(QAOA_ERR_INVALID_ARGUMENT, "L must be >= 0");
    if (L > 0 && (!masks || !w)) return fail(QAOA_ERR_INVALID_ARGUMENT, "mask or weight array is NULL");
    if (!std::isfinite(offset)) return fail(QAOA_ERR_INVALID_ARGUMENT, "offset must be finite");
    const uint64_t lim = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    for (int64_t k = 0; k < L; ++k) {
        if (masks[k] & ~lim) {
            set_err("term %s%lld uses a variable outside [0, n)", "", (long long)k);
            return QAOA_ERR_INVALID_ARGUMENT;
        }
        if (!std::isfinite(w[k])) return fail(QAOA_ERR_INVALID_ARGUMENT, "weights must be finite");
    }
    if (!out) return fail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    std::vector<qk::CostPiece> pieces;
    qaoa_status st = make_pieces(&pieces, [&] { return qk::cost_pieces_poly(L, masks, w); });
    if (st != QAOA_OK) return st;
    return create_with_pieces(n, precision, stream, out, pieces, offset);
}

qaoa_status qaoa_destroy(qaoa_handle h)
{
    if (!h) return QAOA_OK;
    DeviceGuard dg(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    dev_free(h, h->psi, h->N * amp_bytes(h->prec));
    dev_free(h, h->lam, h->N * amp_bytes(h->prec));
    dev_free(h, h->cost, h->N * cost_bytes(h->prec));
    dev_free(h, h->parts, h->parts_cap * sizeof(double));
    dev_free(h, h->res, h->res_cap * sizeof(double));
    for (auto &pd : h->pending) {
        (void)hipEventDestroy(pd.t0);
        (void)hipEventDestroy(pd.t1);
    }
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return QAOA_OK;
}

qaoa_status qaoa_get_info(qaoa_handle h, int32_t *n, int32_t *precision)
{
    if (!h) return fail(QAOA_ERR_INVALID_ARGUMENT, "handle is NULL");
    if (n) *n = h->n;
    if (precision) *precision = h->prec;
    return QAOA_OK;
}

qaoa_status qaoa_cost_diagonal(qaoa_handle h, double *out, int32_t out_is_device)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if (!out) return fail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    DeviceGuard dg(h->device);
    if (!c64(h)) {
        HIPCHECK(h, hipMemcpyAsync(out, h->cost, h->N * 8,
                                   out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                   h->stream));
        if (!out_is_device) HIPCHECK(h, hipStreamSynchronize(h->stream));
        return QAOA_OK;
    }
    if (out_is_device) {
        HIPCHECK(h, qk::launch_widen_cost((const float *)h->cost, out, h->N, h->stream));
        return QAOA_OK;
    }
    std::vector<float> tmp;
    try {
        tmp.resize(h->N);
    } catch (...) {
        return fail(QAOA_ERR_OUT_OF_MEMORY, "host staging buffer");
    }
    HIPCHECK(h, hipMemcpyAsync(tmp.data(), h->cost, h->N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    for (uint64_t z = 0; z < h->N; ++z) out[z] = (double)tmp[z];
    return QAOA_OK;
}

qaoa_status qaoa_cost_extrema(qaoa_handle h, double *cmin, double *cmax)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if (!cmin || !cmax) return fail(QAOA_ERR_INVALID_ARGUMENT, "output is NULL");
    if (!h->extrema_valid) {
        DeviceGuard dg(h->device);
        const uint64_t T = (h->N + qk::kTile - 1) / qk::kTile;
        if ((st = ensure_doubles(h, &h->parts, &h->parts_cap, 2 * T)) != QAOA_OK) return st;
        HIPCHECK(h, qk::launch_minmax(c64(h), h->cost, h->n, h->parts, h->parts + T, h->stream));
        HIPCHECK(h, qk::launch_minmax_final(h->parts, h->parts + T, T, h->res, h->stream));
        double r[2];
        HIPCHECK(h, hipMemcpyAsync(r, h->res, sizeof r, hipMemcpyDeviceToHost, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        h->cmin = r[0];
        h->cmax = r[1];
        h->extrema_valid = true;
    }
    *cmin = h->cmin;
    *cmax = h->cmax;
    return QAOA_OK;
}

qaoa_status qaoa_statevector(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                             void *out, int32_t out_is_device)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if ((st = check_angles(p, gamma, beta)) != QAOA_OK) return st;
    DeviceGuard dg(h->device);
    h->state_valid = false;
    if (p == 0) {
        HIPCHECK(h, qk::launch_fill_plus(c64(h), h->psi, h->n, h->stream));
    } else if ((st = run_forward(h, p, gamma, beta, false, false)) != QAOA_OK) {
        return st;
    }
    if ((st = keep_angles(h, p, gamma, beta)) != QAOA_OK) return st;
    h->state_valid = true;
    if (out) {
        HIPCHECK(h, hipMemcpyAsync(out, h->psi, h->N * amp_bytes(h->prec),
                                   out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                   h->stream));
        if (!out_is_device) HIPCHECK(h, hipStreamSynchronize(h->stream));
    }
    return QAOA_OK;
}

qaoa_status qaoa_expectation(qaoa_handle h, double *E)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if (!E) return fail(QAOA_ERR_INVALID_ARGUMENT, "E is NULL");
    if (!h->state_valid) return fail(QAOA_ERR_NO_STATE, "no current state");
    DeviceGuard dg(h->device);
    const uint64_t T = (h->N + qk::kTile - 1) / qk::kTile;
    if ((st = ensure_doubles(h, &h->parts, &h->parts_cap, T)) != QAOA_OK) return st;
    HIPCHECK(h, qk::launch_expect(c64(h), h->psi, h->cost, h->n, h->parts, h->stream));
    return fetch_results(h, 1, T, E);
}

qaoa_status qaoa_evaluate(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                          double *E)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if ((st = check_angles(p, gamma, beta)) != QAOA_OK) return st;
    if (!E) return fail(QAOA_ERR_INVALID_ARGUMENT, "E is NULL");
    if (p == 0) {
        if ((st = qaoa_statevector(h, 0, nullptr, nullptr, nullptr, 0)) != QAOA_OK) return st;
        return qaoa_expectation(h, E);
    }
    DeviceGuard dg(h->device);
    h->state_valid = false;
    const uint64_t T = nblocks(h);
    if ((st = ensure_doubles(h, &h->parts, &h->parts_cap, T)) != QAOA_OK) return st;
    if ((st = run_forward(h, p, gamma, beta, false, true)) != QAOA_OK) return st;
    if ((st = keep_angles(h, p, gamma, beta)) != QAOA_OK) return st;
    h->state_valid = true;
    return fetch_results(h, 1, T, E);
}

qaoa_status qaoa_gradient(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                          double *E, double *dgamma, double *dbeta)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if ((st = check_angles(p, gamma, beta)) != QAOA_OK) return st;
    if (p > 0 && (!dgamma || !dbeta)) return fail(QAOA_ERR_INVALID_ARGUMENT, "gradient output is NULL");
    if (p == 0) {
        double e0;
        if ((st = qaoa_evaluate(h, 0, nullptr, nullptr, &e0)) != QAOA_OK) return st;
        if (E) *E = e0;
        h->state_valid = false;
        return QAOA_OK;
    }
    DeviceGuard dg(h->device);
    if ((st = ensure_lam(h)) != QAOA_OK) return st;
    const uint64_t T = nblocks(h);
    const int nslots = 2 * p + 1;
    if ((st = ensure_doubles(h, &h->parts, &h->parts_cap, (size_t)nslots * T)) != QAOA_OK) return st;
    if ((st = ensure_doubles(h, &h->res, &h->res_cap, (size_t)nslots)) != QAOA_OK) return st;
    h->state_valid = false;

    if ((st = enqueue_gradient(h, p, gamma, beta, h->lam, h->parts)) != QAOA_OK) return st;
    std::vector<double> r((size_t)nslots);
    if ((st = fetch_results(h, nslots, T, r.data())) != QAOA_OK) return st;
    if (E) *E = r[0];
    for (int l = 0; l < p; ++l) {
        dbeta[l] = 2.0 * r[1 + l];
        dgamma[l] = 2.0 * r[1 + p + l];
    }
    return QAOA_OK;
}

qaoa_status qaoa_gradient_from_state(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                                     double *dgamma, double *dbeta)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if ((st = check_angles(p, gamma, beta)) != QAOA_OK) return st;
    if (p > 0 && (!dgamma || !dbeta)) return fail(QAOA_ERR_INVALID_ARGUMENT, "gradient output is NULL");
    if (!h->state_valid) return fail(QAOA_ERR_NO_STATE, "no current state (run qaoa_evaluate or qaoa_statevector first)");
    bool same = h->state_angles.size() == (size_t)(2 * p);
    for (int l = 0; same && l < p; ++l)
        same = h->state_angles[l] == gamma[l] && h->state_angles[p + l] == beta[l];
    if (!same) return fail(QAOA_ERR_NO_STATE, "the current state was computed at other angles");
    if (p == 0) return QAOA_OK;
    DeviceGuard dg(h->device);
    if ((st = ensure_lam(h)) != QAOA_OK) return st;
    const uint64_t T = nblocks(h);
    const int nslots = 2 * p + 1;
    if ((st = ensure_doubles(h, &h->parts, &h->parts_cap, (size_t)nslots * T)) != QAOA_OK) return st;
    if ((st = ensure_doubles(h, &h->res, &h->res_cap, (size_t)nslots)) != QAOA_OK) return st;
    h->state_valid = false;
    if ((st = enqueue_reverse(h, p, gamma, beta, h->lam, h->parts)) != QAOA_OK) return st;
    // slots 1 .. 2p (slot 0, E, is not written by the reverse sweep)
    HIPCHECK(h, qk::launch_sum_slots(h->parts + T, T, T, 2 * p, h->res, h->stream));
    std::vector<double> r((size_t)(2 * p));
    HIPCHECK(h, hipMemcpyAsync(r.data(), h->res, (size_t)(2 * p) * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    for (int l = 0; l < p; ++l) {
        dbeta[l] = 2.0 * r[l];
        dgamma[l] = 2.0 * r[p + l];
    }
    return QAOA_OK;
}

qaoa_status qaoa_sample(qaoa_handle h, int64_t shots, uint64_t seed, uint64_t *z, double *cost,
                        int32_t out_is_device)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if (shots < 0) return fail(QAOA_ERR_INVALID_ARGUMENT, "shots must be >= 0");
    // bounds the staging arithmetic below far from overflow (2^40 shots = 16 TiB of output)
    if (shots > ((int64_t)1 << 40)) return fail(QAOA_ERR_INVALID_ARGUMENT, "shots must be <= 2^40");
    if (shots > 0 && !z) return fail(QAOA_ERR_INVALID_ARGUMENT, "z is NULL");
    if (!h->state_valid) return fail(QAOA_ERR_NO_STATE, "no current state");
    if (shots == 0) return QAOA_OK;
    DeviceGuard dg(h->device);
    const int sbits = qk::sample_subblock_bits(h->n);
    const uint64_t nsub = h->N >> sbits;
    const uint64_t nscr = qk::scan_scratch_doubles(nsub);
    // layout: sub[nsub] | pre[nsub + 1] | scratch[nscr] | (host output staging)
    const size_t base = 2 * nsub + 1 + nscr;
    const size_t stage = out_is_device ? 0 : (size_t)shots * 2;
    if ((st = ensure_doubles(h, &h->parts, &h->parts_cap, base + stage)) != QAOA_OK) return st;
    double *sub = h->parts, *pre = sub + nsub, *scr = pre + nsub + 1;
    HIPCHECK(h, qk::launch_submass(c64(h), h->psi, h->n, sbits, sub, h->stream));
    HIPCHECK(h, qk::launch_exclusive_scan(sub, nsub, pre, scr, h->stream));
    double T = 0;
    HIPCHECK(h, hipMemcpyAsync(&T, pre + nsub, sizeof T, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(QAOA_ERR_INVALID_ARGUMENT, "state has zero norm");
    uint64_t *dz = z;
    double *dc = cost;
    if (!out_is_device) {
        dz = (uint64_t *)(h->parts + base);
        dc = cost ? h->parts + base + shots : nullptr;
    }
    HIPCHECK(h, qk::launch_shots(c64(h), h->psi, h->cost, h->n, sbits, pre, nsub, shots, seed, dz,
                                 dc, h->stream));
    if (!out_is_device) {
        HIPCHECK(h, hipMemcpyAsync(z, dz, (size_t)shots * 8, hipMemcpyDeviceToHost, h->stream));
        if (cost)
            HIPCHECK(h, hipMemcpyAsync(cost, dc, (size_t)shots * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        // a large staging area is given back; later calls allocate what they need
        if (stage * sizeof(double) > (64ull << 20)) {
            dev_free(h, h->parts, h->parts_cap * sizeof(double));
            h->parts = nullptr;
            h->parts_cap = 0;
        }
    }
    return QAOA_OK;
}

qaoa_status qaoa_profile_enable(qaoa_handle h, int32_t on)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    DeviceGuard dg(h->device);
    if ((st = drain_profile(h)) != QAOA_OK) return st;
    h->profiling = on != 0;
    for (int k = 0; k < 5; ++k) {
        h->prof_launches[k] = 0;
        h->prof_ms[k] = 0;
        h->prof_bytes[k] = 0;
    }
    return QAOA_OK;
}

qaoa_status qaoa_profile_read(qaoa_handle h, int32_t kind, int64_t *launches, double *ms,
                              double *bytes)
{
    qaoa_status st = check_handle(h);
    if (st != QAOA_OK) return st;
    if (kind < 0 || kind > 4) return fail(QAOA_ERR_INVALID_ARGUMENT, "kind must be in [0, 4]");
    DeviceGuard dg(h->device);
    if ((st = drain_profile(h)) != QAOA_OK) return st;
    if (launches) *launches = h->prof_launches[kind];
    if (ms) *ms = h->prof_ms[kind];
    if (bytes) *bytes = h->prof_bytes[kind];
    return QAOA_OK;
}

qaoa_status qaoa_pass_plan(int32_t n, int32_t precision, int32_t cap, int32_t *npasses,
                           uint64_t *tile_bits, uint64_t *target_bits)
{
    if (n < 1 || n > QAOA_MAX_QUBITS)
        return fail(QAOA_ERR_INVALID_ARGUMENT, "n must be in [1, QAOA_MAX_QUBITS]");
    if (precision != QAOA_C128 && precision != QAOA_C64)
        return fail(QAOA_ERR_INVALID_ARGUMENT, "unknown precision");
    if (!npasses || !tile_bits || !target_bits) return fail(QAOA_ERR_INVALID_ARGUMENT, "output is NULL");
    const std::vector<qk::PassPlan> pl = qk::plan_passes(n, precision == QAOA_C64);
    if ((int32_t)pl.size() > cap) return fail(QAOA_ERR_INVALID_ARGUMENT, "cap is too small");
    *npasses = (int32_t)pl.size();
    for (size_t i = 0; i < pl.size(); ++i) {
        tile_bits[i] = pl[i].tile_bits;
        target_bits[i] = pl[i].target_bits;
    }
    return QAOA_OK;
}

const char *qaoa_status_string(qaoa_status s)
{
    switch (s) {
    case QAOA_OK: return "success";
    case QAOA_ERR_INVALID_ARGUMENT: return "invalid argument";
    case QAOA_ERR_OUT_OF_MEMORY: return "out of device memory";
    case QAOA_ERR_DEVICE: return "device error";
    case QAOA_ERR_NO_STATE: return "no current state";
    case QAOA_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *qaoa_last_error_message(void) { return g_err.c_str(); }

qaoa_status qaoa_set_allocator(const qaoa_allocator *a)
{
    if (!a) {
        g_alloc = qaoa_allocator{};
        return QAOA_OK;
    }
    if (!a->alloc || !a->free) return fail(QAOA_ERR_INVALID_ARGUMENT, "allocator needs both alloc and free");
    g_alloc = *a;
    return QAOA_OK;
}

}  // extern "C"
