// Warm-start network: a message-passing network that maps a weighted graph to
// QAOA angles, trained and evaluated entirely with the kernels below.
//
// Network (hidden width 128, three message-passing layers, depth-p output):
//   x_v = (deg_v / 8, wdeg_v / 8, 1, sqdeg_v / 8, 0 ... 0)      (32 features)
//   H'  = ReLU([H | A H] W_l^T + b_l)                            (l = 0, 1, 2)
//   g   = mean of H over the graph's nodes
//   Y   = ReLU(g W_h1^T + b_h1) W_h2^T + b_h2                    (2p outputs)
//   gamma_i = i/p + Y_i,  beta_i = 1 - i/p + Y_{p+i}              (i = 1..p)
// A is the symmetric weighted adjacency.  Loss: mean squared angle error.
//
// Every matrix product runs on the bf16 matrix cores (16x16x32 MFMA, fp32
// accumulation) with bf16 operands: activations, aggregated messages, the bf16
// copy of the fp32 master weights, and the gradients fed to the
// weight-gradient products.  Aggregation, pooling, the loss, bias gradients
// and Adam run in fp32.  Every reduction has a fixed order, so results do not
// depend on scheduling.
#include "qaoa.h"
#include "qaoa_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace qm {
namespace {

constexpr int kHid = 128;
constexpr int kFin = 32;
constexpr int kLayers = 3;
constexpr int kOutPad = 32;  // 2p outputs padded to one MFMA K step

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (inputs are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

union Frag {
    uint4 u;
    uint16_t h[8];
    bf16x8 v;
};

// Eight consecutive-k bf16 values of one row (A) or column (B) of an operand:
// element (outer, k) sits at P[outer * s_outer + k * s_k].  Out-of-range
// entries read as zero.
__device__ __forceinline__ bf16x8 load_frag(const uint16_t *P, int64_t s_outer, int64_t s_k, int outer,
                                            int OUT, int k, int kend, bool contig)
{
    Frag r;
    if (contig && outer < OUT && k + 8 <= kend) {
        r.u = *(const uint4 *)(P + (int64_t)outer * s_outer + k);
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            r.h[j] = (outer < OUT && k + j < kend) ? P[(int64_t)outer * s_outer + (int64_t)(k + j) * s_k] : 0;
    }
    return r.v;
}

struct GemmArgs {
    const uint16_t *A;  // op(A)[m][k] = A[m * sam + k * sak]
    int64_t sam, sak;
    const uint16_t *B;  // op(B)[k][n] = B[k * sbk + n * sbn]
    int64_t sbk, sbn;
    int M, N, K;
    int kchunk;          // K range of one blockIdx.z (a multiple of 32)
    float *C32;          // fp32 result (split: partial of slice z at C32 + z * split_stride)
    int64_t ldc32, split_stride;
    uint16_t *C16;       // optional bf16 copy of the (ReLU'd if relu) result
    int64_t ldc16;
    const float *bias;   // optional [N]
    const float *mask;   // optional: result multiplied by (mask[m][n] > 0)
    int64_t ldmask;
    int relu;
    int contigA, contigB;
};

// C = op(A) op(B) on 64 x 64 output tiles: four waves of 32 x 32, each a 2 x 2
// grid of 16x16x32 bf16 MFMAs accumulating in fp32.  Per MFMA, lane l holds
// row l % 16 of A and column l % 16 of B over k = 8 (l / 16) .. + 8, and
// receives C rows 4 (l / 16) .. + 4 of column l % 16.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m_base = blockIdx.x * 64 + (wave >> 1) * 32;
    const int n_base = blockIdx.y * 64 + (wave & 1) * 32;
    const int k_begin = blockIdx.z * g.kchunk;
    const int k_end = min(g.K, k_begin + g.kchunk);
    const int r = lane & 15, kq = (lane >> 4) * 8;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = k_begin; k0 < k_end; k0 += 32) {
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = load_frag(g.A, g.sam, g.sak, m_base + 16 * i + r, g.M, k0 + kq, k_end, g.contigA);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = load_frag(g.B, g.sbn, g.sbk, n_base + 16 * j + r, g.N, k0 + kq, k_end, g.contigB);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    const bool split = gridDim.z > 1;
    float *C32 = g.C32 + (split ? (int64_t)blockIdx.z * g.split_stride : 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m_base + 16 * i + 4 * (lane >> 4) + q;
                const int n = n_base + 16 * j + r;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][q];
                if (!split) {
                    if (g.bias) v += g.bias[n];
                    if (g.mask && !(g.mask[(int64_t)m * g.ldmask + n] > 0.f)) v = 0.f;
                }
                if (C32) C32[(int64_t)m * g.ldc32 + n] = v;
                if (!split && g.C16) g.C16[(int64_t)m * g.ldc16 + n] = f2bf(g.relu ? fmaxf(v, 0.f) : v);
            }
}

// out[m][n] (ld ldo) = sum over z = 0 .. S-1 of part[z][m][n] (row length N), in order.
__global__ __launch_bounds__(256) void k_split_sum(const float *part, int S, int64_t stride, int M, int N,
                                                   float *out, int64_t ldo)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[z * stride + i];
    out[(i / N) * ldo + i % N] = s;
}

// Column sums of X [R][C] (ld ldx): stage 1 writes per-chunk partials [S][C].
__global__ __launch_bounds__(256) void k_colsum_part(const float *X, int R, int C, int64_t ldx, int rows_per,
                                                     float *part)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    const int r0 = blockIdx.y * rows_per, r1 = min(R, r0 + rows_per);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += X[(int64_t)r * ldx + c];
    part[(int64_t)blockIdx.y * C + c] = s;
}

__global__ __launch_bounds__(256) void k_colsum_final(const float *part, int S, int C, float *out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * C + c];
    out[c] = s;
}

// Node input features into the left half of XC0 [N][2 * kFin] (bf16).
__global__ __launch_bounds__(256) void k_features(const int32_t *rowp, const float *val, int N, uint16_t *XC0)
{
    const int v = blockIdx.x * 8 + (threadIdx.x >> 5), f = threadIdx.x & 31;
    if (v >= N) return;
    float x = 0.f;
    if (f == 0) x = (float)(rowp[v + 1] - rowp[v]) / 8.f;
    if (f == 1 || f == 3) {
        float s = 0.f;
        for (int j = rowp[v]; j < rowp[v + 1]; ++j) s += f == 1 ? val[j] : val[j] * val[j];
        x = s / 8.f;
    }
    if (f == 2) x = 1.f;
    XC0[(int64_t)v * 2 * kFin + f] = f2bf(x);
}

// Messages: XC[v][d + f] = bf16(sum_j val[j] * XC[col[j]][f]) (left half = H, bf16).
template <int D>
__global__ __launch_bounds__(256) void k_aggregate(const int32_t *rowp, const int32_t *col, const float *val,
                                                   int N, uint16_t *XC)
{
    constexpr int PER = 256 / D;
    const int v = blockIdx.x * PER + threadIdx.x / D, f = threadIdx.x % D;
    if (v >= N) return;
    float s = 0.f;
    for (int j = rowp[v]; j < rowp[v + 1]; ++j) s += val[j] * bf2f(XC[(int64_t)col[j] * 2 * D + f]);
    XC[(int64_t)v * 2 * D + D + f] = f2bf(s);
}

// Backward of [H | A H]: dH[v][f] = dXC[v][f] + sum_j val[j] dXC[col[j]][d + f]
// (A is symmetric), then dZ = dH * (Z > 0) in fp32 and bf16.
template <int D>
__global__ __launch_bounds__(256) void k_aggregate_bwd(const int32_t *rowp, const int32_t *col, const float *val,
                                                       int N, const float *dXC, const float *Zprev,
                                                       float *dZ, uint16_t *dZ16)
{
    constexpr int PER = 256 / D;
    const int v = blockIdx.x * PER + threadIdx.x / D, f = threadIdx.x % D;
    if (v >= N) return;
    float s = dXC[(int64_t)v * 2 * D + f];
    for (int j = rowp[v]; j < rowp[v + 1]; ++j) s += val[j] * dXC[(int64_t)col[j] * 2 * D + D + f];
    const float d = Zprev[(int64_t)v * kHid + f] > 0.f ? s : 0.f;
    dZ[(int64_t)v * kHid + f] = d;
    dZ16[(int64_t)v * kHid + f] = f2bf(d);
}

// Readout: g[G][f] = mean over the graph's nodes of ReLU(Z3), fp32 and bf16.
__global__ __launch_bounds__(kHid) void k_pool(const int32_t *noff, const float *Z3, float *g, uint16_t *g16)
{
    const int gi = blockIdx.x, f = threadIdx.x;
    const int v0 = noff[gi], v1 = noff[gi + 1];
    float s = 0.f;
    for (int v = v0; v < v1; ++v) s += fmaxf(Z3[(int64_t)v * kHid + f], 0.f);
    const float m = v1 > v0 ? s / (float)(v1 - v0) : 0.f;
    g[(int64_t)gi * kHid + f] = m;
    g16[(int64_t)gi * kHid + f] = f2bf(m);
}

// Backward of the readout and the last ReLU: dZ3[v] = dg[graph(v)] / n * (Z3 > 0).
__global__ __launch_bounds__(256) void k_unpool(const int32_t *node_graph, const int32_t *noff, const float *dg,
                                                const float *Z3, int N, float *dZ, uint16_t *dZ16)
{
    const int v = blockIdx.x * 2 + threadIdx.x / kHid, f = threadIdx.x % kHid;
    if (v >= N) return;
    const int gi = node_graph[v];
    const float cnt = (float)(noff[gi + 1] - noff[gi]);
    const int64_t o = (int64_t)v * kHid + f;
    const float d = Z3[o] > 0.f ? dg[(int64_t)gi * kHid + f] / cnt : 0.f;
    dZ[o] = d;
    dZ16[o] = f2bf(d);
}

// Angles from the head output Y [G][kOutPad]; optional loss terms against targets.
__global__ __launch_bounds__(256) void k_angles(const float *Y, int G, int p, double *gamma, double *beta,
                                                const double *gt, const double *bt, float *dY, uint16_t *dY16,
                                                double *sq)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= G * kOutPad) return;
    const int gi = i / kOutPad, o = i % kOutPad;
    if (o >= 2 * p) {
        if (dY) {
            dY[i] = 0.f;
            dY16[i] = 0;
        }
        return;
    }
    const int k = o < p ? o : o - p;
    const double ramp = (double)(k + 1) / p;
    const double a = (double)Y[i] + (o < p ? ramp : 1.0 - ramp);
    if (gamma && o < p) gamma[(int64_t)gi * p + k] = a;
    if (beta && o >= p) beta[(int64_t)gi * p + k] = a;
    if (dY) {
        const double t = o < p ? gt[(int64_t)gi * p + k] : bt[(int64_t)gi * p + k];
        const double d = a - t;
        sq[(int64_t)gi * 2 * p + o] = d * d;
        const float dy = (float)(2.0 * d / (2.0 * p * G));
        dY[i] = dy;
        dY16[i] = f2bf(dy);
    }
}

// Fixed-order sum of n doubles by one block.
__global__ __launch_bounds__(256) void k_sum(const double *x, int64_t n, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam descent on the fp32 master parameters; refreshes their bf16 copy.
__global__ __launch_bounds__(256) void k_adam(float *theta, const float *grad, float *m, float *v, uint16_t *t16,
                                              int64_t n, float lr, float b1, float b2, float eps, float c1,
                                              float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = th;
    t16[i] = f2bf(th);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *x, uint16_t *y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

}  // namespace
}  // namespace qm

// ------------------------------------------------------------------ host side

namespace {

// Offsets of the parameter blocks in the flat vector (see qaoa.h).
struct Layout {
    int64_t W[3], b[3], Wh1, bh1, Wh2, bh2, total;
    int din[3];
    explicit Layout(int p)
    {
        int64_t o = 0;
        int d = qm::kFin;
        for (int l = 0; l < 3; ++l) {
            din[l] = d;
            W[l] = o;
            o += (int64_t)qm::kHid * 2 * d;
            b[l] = o;
            o += qm::kHid;
            d = qm::kHid;
        }
        Wh1 = o;
        o += (int64_t)qm::kHid * qm::kHid;
        bh1 = o;
        o += qm::kHid;
        Wh2 = o;
        o += (int64_t)2 * p * qm::kHid;
        bh2 = o;
        o += 2 * p;
        total = o;
    }
};

struct GraphBatch {
    int G = 0, N = 0, E2 = 0;
    std::vector<int32_t> rowp, col, noff, node_graph;
    std::vector<float> val;
};

qaoa_status mfail(qaoa_status st, const std::string &m)
{
    qk::set_error_message(m);
    return st;
}

// Validate a graph batch and build its symmetric CSR (entries of a row in edge order).
qaoa_status build_batch(int32_t count, const int32_t *n, const int64_t *off, const int32_t *edges,
                        const double *w, GraphBatch &B)
{
    if (count < 1 || !n || !off) return mfail(QAOA_ERR_INVALID_ARGUMENT, "count, n or edge_offsets invalid");
    if (off[0] != 0) return mfail(QAOA_ERR_INVALID_ARGUMENT, "edge_offsets[0] must be 0");
    B.G = count;
    B.noff.assign(count + 1, 0);
    int64_t N = 0;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 1 || n[i] > 4096) return mfail(QAOA_ERR_INVALID_ARGUMENT, "n out of [1, 4096]");
        if (off[i + 1] < off[i]) return mfail(QAOA_ERR_INVALID_ARGUMENT, "edge_offsets decrease");
        N += n[i];
        if (N > (1 << 24)) return mfail(QAOA_ERR_INVALID_ARGUMENT, "too many nodes in one batch");
        B.noff[i + 1] = (int32_t)N;
    }
    const int64_t E = off[count];
    if (E > (1 << 26)) return mfail(QAOA_ERR_INVALID_ARGUMENT, "too many edges in one batch");
    if (E > 0 && !edges) return mfail(QAOA_ERR_INVALID_ARGUMENT, "edges is NULL");
    B.N = (int)N;
    B.E2 = (int)(2 * E);
    std::vector<int32_t> deg(N + 1, 0);
    for (int i = 0; i < count; ++i)
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            const int u = edges[2 * k], v = edges[2 * k + 1];
            if (u < 0 || v < 0 || u >= n[i] || v >= n[i] || u == v)
                return mfail(QAOA_ERR_INVALID_ARGUMENT, "edge index out of range or self-loop");
            if (w && !std::isfinite(w[k])) return mfail(QAOA_ERR_INVALID_ARGUMENT, "weights must be finite");
            ++deg[B.noff[i] + u];
            ++deg[B.noff[i] + v];
        }
    B.rowp.assign(N + 1, 0);
    for (int64_t v = 0; v < N; ++v) B.rowp[v + 1] = B.rowp[v] + deg[v];
    B.col.assign(B.E2, 0);
    B.val.assign(B.E2, 0.f);
    std::vector<int32_t> fill(B.rowp.begin(), B.rowp.end() - 1);
    for (int i = 0; i < count; ++i)
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            const int u = B.noff[i] + edges[2 * k], v = B.noff[i] + edges[2 * k + 1];
            const float wk = w ? (float)w[k] : 1.f;
            B.col[fill[u]] = v;
            B.val[fill[u]++] = wk;
            B.col[fill[v]] = u;
            B.val[fill[v]++] = wk;
        }
    B.node_graph.assign(N, 0);
    for (int i = 0; i < count; ++i)
        for (int v = B.noff[i]; v < B.noff[i + 1]; ++v) B.node_graph[v] = i;
    return QAOA_OK;
}

}  // namespace

struct qaoa_mpnn_s {
    int p = 0, device = 0;
    Layout lay{1};
    hipStream_t stream = nullptr;
    bool poisoned = false;
    int64_t step = 0;
    // parameters (fp32 master, bf16 copy), gradient, Adam moments
    float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
    uint16_t *theta16 = nullptr;
    // per-batch workspace (grown on demand)
    std::vector<std::pair<void **, size_t>> ws_list;
    size_t ws_nodes = 0, ws_edges = 0, ws_graphs = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int32_t *rowp, *col, *noff, *node_graph;
    float *val;
    uint16_t *XC[3];        // [N][2 d_l]
    float *Z[3];            // [N][128]
    float *g, *Z1, *Y, *dY, *dZ1, *dg, *dZ, *dXC, *part, *loss_sq_f;
    uint16_t *g16, *A1, *dY16, *dZ116, *dZ16;
    double *gam, *bet, *gt, *bt, *sq, *loss;
};

namespace {

#define MCHECK(m, call)                                                                \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (m)->poisoned = true;                                                      \
            return mfail(QAOA_ERR_DEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)

constexpr int kSplitMax = 64;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carve the workspace for G graphs, N nodes and E2 CSR entries.
qaoa_status ensure_ws(qaoa_mpnn m, int G, int N, int E2)
{
    if ((size_t)G <= m->ws_graphs && (size_t)N <= m->ws_nodes && (size_t)E2 <= m->ws_edges) return QAOA_OK;
    const size_t Gc = std::max<size_t>(G, m->ws_graphs), Nc = std::max<size_t>(N, m->ws_nodes),
                 Ec = std::max<size_t>(std::max(E2, 1), m->ws_edges);
    const int p2 = 2 * m->p;
    struct Item {
        void **ptr;
        size_t bytes;
    };
    const size_t partN = (size_t)kSplitMax * qm::kHid * 2 * qm::kHid;
    std::vector<Item> items = {
        {(void **)&m->rowp, (Nc + 1) * 4}, {(void **)&m->col, Ec * 4}, {(void **)&m->val, Ec * 4},
        {(void **)&m->noff, (Gc + 1) * 4}, {(void **)&m->node_graph, Nc * 4},
        {(void **)&m->XC[0], Nc * 2 * qm::kFin * 2}, {(void **)&m->XC[1], Nc * 2 * qm::kHid * 2},
        {(void **)&m->XC[2], Nc * 2 * qm::kHid * 2}, {(void **)&m->Z[0], Nc * qm::kHid * 4},
        {(void **)&m->Z[1], Nc * qm::kHid * 4}, {(void **)&m->Z[2], Nc * qm::kHid * 4},
        {(void **)&m->g, Gc * qm::kHid * 4}, {(void **)&m->g16, Gc * qm::kHid * 2},
        {(void **)&m->Z1, Gc * qm::kHid * 4}, {(void **)&m->A1, Gc * qm::kHid * 2},
        {(void **)&m->Y, Gc * qm::kOutPad * 4}, {(void **)&m->dY, Gc * qm::kOutPad * 4},
        {(void **)&m->dY16, Gc * qm::kOutPad * 2}, {(void **)&m->dZ1, Gc * qm::kHid * 4},
        {(void **)&m->dZ116, Gc * qm::kHid * 2}, {(void **)&m->dg, Gc * qm::kHid * 4},
        {(void **)&m->dZ, Nc * qm::kHid * 4}, {(void **)&m->dZ16, Nc * qm::kHid * 2},
        {(void **)&m->dXC, Nc * 2 * qm::kHid * 4}, {(void **)&m->part, partN * 4},
        {(void **)&m->gam, Gc * m->p * 8}, {(void **)&m->bet, Gc * m->p * 8},
        {(void **)&m->gt, Gc * m->p * 8}, {(void **)&m->bt, Gc * m->p * 8},
        {(void **)&m->sq, Gc * p2 * 8}, {(void **)&m->loss, 8},
    };
    size_t total = 0;
    for (const Item &it : items) total += align256(it.bytes);
    size_t fr = 0, tot = 0;
    MCHECK(m, hipMemGetInfo(&fr, &tot));
    if (m->ws) {
        MCHECK(m, hipStreamSynchronize(m->stream));
        (void)hipFree(m->ws);
        m->ws = nullptr;
        fr += m->ws_bytes;
        // no workspace until the new one is carved: a failed allocation below
        // must not leave the old capacities pointing at freed memory
        m->ws_bytes = 0;
        m->ws_graphs = m->ws_nodes = m->ws_edges = 0;
    }
    if (total > fr) return mfail(QAOA_ERR_OUT_OF_MEMORY, "workspace does not fit in device memory");
    MCHECK(m, hipMalloc(&m->ws, total));
    m->ws_bytes = total;
    char *c = (char *)m->ws;
    for (const Item &it : items) {
        *it.ptr = c;
        c += align256(it.bytes);
    }
    m->ws_graphs = Gc;
    m->ws_nodes = Nc;
    m->ws_edges = Ec;
    return QAOA_OK;
}

// Launch one product; K splits (when > 1) go to m->part and are summed into C32.
qaoa_status gemm(qaoa_mpnn m, const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
                 int64_t sbn, int M, int N, int K, float *C32, int64_t ldc32, uint16_t *C16 = nullptr,
                 int64_t ldc16 = 0, const float *bias = nullptr, const float *mask = nullptr,
                 int64_t ldmask = 0, bool relu = false, int splits = 1)
{
    if (M <= 0 || N <= 0) return QAOA_OK;
    qm::GemmArgs g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.M = M;
    g.N = N;
    g.K = K;
    auto aligned = [](const void *p, int64_t s_outer) {
        return ((uintptr_t)p % 16 == 0) && (s_outer % 8 == 0);
    };
    g.contigA = (sak == 1 && aligned(A, sam)) ? 1 : 0;
    g.contigB = (sbk == 1 && aligned(B, sbn)) ? 1 : 0;
    const int kblocks = std::max(1, (K + 31) / 32);
    splits = std::max(1, std::min(splits, std::min(kSplitMax, kblocks)));
    if ((size_t)M * N > (size_t)qm::kHid * 2 * qm::kHid) splits = 1;  // partial buffer bound
    g.kchunk = ((kblocks + splits - 1) / splits) * 32;
    splits = std::max(1, (K + g.kchunk - 1) / g.kchunk);
    dim3 grid((M + 63) / 64, (N + 63) / 64, splits);
    if (splits > 1) {
        g.C32 = m->part;
        g.ldc32 = N;
        g.split_stride = (int64_t)M * N;
    } else {
        g.C32 = C32;
        g.ldc32 = ldc32;
        g.C16 = C16;
        g.ldc16 = ldc16;
        g.bias = bias;
        g.mask = mask;
        g.ldmask = ldmask;
        g.relu = relu ? 1 : 0;
    }
    hipLaunchKernelGGL(qm::k_gemm, grid, dim3(256), 0, m->stream, g);
    MCHECK(m, hipGetLastError());
    if (splits > 1) {
        const int64_t tot = (int64_t)M * N;
        hipLaunchKernelGGL(qm::k_split_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, m->stream,
                           (const float *)m->part, splits, (int64_t)M * N, M, N, C32, ldc32);
        MCHECK(m, hipGetLastError());
    }
    return QAOA_OK;
}

qaoa_status colsum(qaoa_mpnn m, const float *X, int R, int C, int64_t ldx, float *out)
{
    const int S = std::max(1, std::min(kSplitMax, (R + 127) / 128));
    const int rows_per = (R + S - 1) / S;
    hipLaunchKernelGGL(qm::k_colsum_part, dim3((C + 255) / 256, S), dim3(256), 0, m->stream, X, R, C, ldx,
                       rows_per, m->part);
    MCHECK(m, hipGetLastError());
    hipLaunchKernelGGL(qm::k_colsum_final, dim3((C + 255) / 256), dim3(256), 0, m->stream, (const float *)m->part,
                       S, C, out);
    MCHECK(m, hipGetLastError());
    return QAOA_OK;
}

#define MTRY(x)                               \
    do {                                      \
        qaoa_status s_ = (x);                 \
        if (s_ != QAOA_OK) return s_;         \
    } while (0)

qaoa_status upload_batch(qaoa_mpnn m, const GraphBatch &B)
{
    MTRY(ensure_ws(m, B.G, B.N, B.E2));
    MCHECK(m, hipMemcpyAsync(m->rowp, B.rowp.data(), (B.N + 1) * 4, hipMemcpyHostToDevice, m->stream));
    if (B.E2) {
        MCHECK(m, hipMemcpyAsync(m->col, B.col.data(), (size_t)B.E2 * 4, hipMemcpyHostToDevice, m->stream));
        MCHECK(m, hipMemcpyAsync(m->val, B.val.data(), (size_t)B.E2 * 4, hipMemcpyHostToDevice, m->stream));
    }
    MCHECK(m, hipMemcpyAsync(m->noff, B.noff.data(), (B.G + 1) * 4, hipMemcpyHostToDevice, m->stream));
    MCHECK(m, hipMemcpyAsync(m->node_graph, B.node_graph.data(), (size_t)B.N * 4, hipMemcpyHostToDevice,
                             m->stream));
    return QAOA_OK;
}

// Forward pass on the uploaded batch; Y [G][kOutPad] and every intermediate kept.
qaoa_status forward(qaoa_mpnn m, const GraphBatch &B)
{
    const Layout &L = m->lay;
    const int N = B.N, G = B.G;
    hipLaunchKernelGGL(qm::k_features, dim3((N + 7) / 8), dim3(256), 0, m->stream, (const int32_t *)m->rowp,
                       (const float *)m->val, N, m->XC[0]);
    MCHECK(m, hipGetLastError());
    for (int l = 0; l < qm::kLayers; ++l) {
        const int d = L.din[l];
        if (d == qm::kFin)
            hipLaunchKernelGGL(qm::k_aggregate<qm::kFin>, dim3((N + 7) / 8), dim3(256), 0, m->stream,
                               (const int32_t *)m->rowp, (const int32_t *)m->col, (const float *)m->val, N,
                               m->XC[l]);
        else
            hipLaunchKernelGGL(qm::k_aggregate<qm::kHid>, dim3((N + 1) / 2), dim3(256), 0, m->stream,
                               (const int32_t *)m->rowp, (const int32_t *)m->col, (const float *)m->val, N,
                               m->XC[l]);
        MCHECK(m, hipGetLastError());
        // Z = XC W^T + b;  next layer's H = bf16(ReLU(Z))
        uint16_t *next = l + 1 < qm::kLayers ? m->XC[l + 1] : nullptr;
        MTRY(gemm(m, m->XC[l], 2 * d, 1, m->theta16 + L.W[l], 1, 2 * d, N, qm::kHid, 2 * d, m->Z[l], qm::kHid,
                  next, 2 * qm::kHid, m->theta + L.b[l], nullptr, 0, true));
    }
    hipLaunchKernelGGL(qm::k_pool, dim3(G), dim3(qm::kHid), 0, m->stream, (const int32_t *)m->noff,
                       (const float *)m->Z[2], m->g, m->g16);
    MCHECK(m, hipGetLastError());
    MTRY(gemm(m, m->g16, qm::kHid, 1, m->theta16 + L.Wh1, 1, qm::kHid, G, qm::kHid, qm::kHid, m->Z1, qm::kHid,
              m->A1, qm::kHid, m->theta + L.bh1, nullptr, 0, true));
    MTRY(gemm(m, m->A1, qm::kHid, 1, m->theta16 + L.Wh2, 1, qm::kHid, G, 2 * m->p, qm::kHid, m->Y, qm::kOutPad,
              nullptr, 0, m->theta + L.bh2));
    return QAOA_OK;
}

// Backward pass from dY (set by k_angles); gradient into m->grad.
qaoa_status backward(qaoa_mpnn m, const GraphBatch &B)
{
    const Layout &L = m->lay;
    const int N = B.N, G = B.G, p2 = 2 * m->p;
    // head
    MTRY(gemm(m, m->dY16, 1, qm::kOutPad, m->A1, qm::kHid, 1, p2, qm::kHid, G, m->grad + L.Wh2, qm::kHid, nullptr,
              0, nullptr, nullptr, 0, false, 8));
    MTRY(colsum(m, m->dY, G, p2, qm::kOutPad, m->grad + L.bh2));
    MTRY(gemm(m, m->dY16, qm::kOutPad, 1, m->theta16 + L.Wh2, qm::kHid, 1, G, qm::kHid, p2, m->dZ1, qm::kHid,
              m->dZ116, qm::kHid, nullptr, m->Z1, qm::kHid));
    MTRY(gemm(m, m->dZ116, 1, qm::kHid, m->g16, qm::kHid, 1, qm::kHid, qm::kHid, G, m->grad + L.Wh1, qm::kHid,
              nullptr, 0, nullptr, nullptr, 0, false, 8));
    MTRY(colsum(m, m->dZ1, G, qm::kHid, qm::kHid, m->grad + L.bh1));
    MTRY(gemm(m, m->dZ116, qm::kHid, 1, m->theta16 + L.Wh1, qm::kHid, 1, G, qm::kHid, qm::kHid, m->dg, qm::kHid));
    // readout and the last layer's ReLU
    hipLaunchKernelGGL(qm::k_unpool, dim3((N + 1) / 2), dim3(256), 0, m->stream, (const int32_t *)m->node_graph,
                       (const int32_t *)m->noff, (const float *)m->dg, (const float *)m->Z[2], N, m->dZ, m->dZ16);
    MCHECK(m, hipGetLastError());
    for (int l = qm::kLayers - 1; l >= 0; --l) {
        const int d = L.din[l];
        const int splits = std::max(1, std::min(kSplitMax, N / 256));
        MTRY(gemm(m, m->dZ16, 1, qm::kHid, m->XC[l], 2 * d, 1, qm::kHid, 2 * d, N, m->grad + L.W[l], 2 * d, nullptr,
                  0, nullptr, nullptr, 0, false, splits));
        MTRY(colsum(m, m->dZ, N, qm::kHid, qm::kHid, m->grad + L.b[l]));
        if (l == 0) break;
        MTRY(gemm(m, m->dZ16, qm::kHid, 1, m->theta16 + L.W[l], 2 * d, 1, N, 2 * d, qm::kHid, m->dXC, 2 * d));
        hipLaunchKernelGGL(qm::k_aggregate_bwd<qm::kHid>, dim3((N + 1) / 2), dim3(256), 0, m->stream,
                           (const int32_t *)m->rowp, (const int32_t *)m->col, (const float *)m->val, N,
                           (const float *)m->dXC, (const float *)m->Z[l - 1], m->dZ, m->dZ16);
        MCHECK(m, hipGetLastError());
    }
    return QAOA_OK;
}

// Angles, and with targets the loss and dY; optional host copies of the angles.
qaoa_status angles_and_loss(qaoa_mpnn m, const GraphBatch &B, const double *gt, const double *bt, double *gamma,
                            double *beta, double *loss)
{
    const int G = B.G, p = m->p;
    const bool tgt = gt != nullptr;
    if (tgt) {
        MCHECK(m, hipMemcpyAsync(m->gt, gt, (size_t)G * p * 8, hipMemcpyHostToDevice, m->stream));
        MCHECK(m, hipMemcpyAsync(m->bt, bt, (size_t)G * p * 8, hipMemcpyHostToDevice, m->stream));
    }
    const int tot = G * qm::kOutPad;
    hipLaunchKernelGGL(qm::k_angles, dim3((tot + 255) / 256), dim3(256), 0, m->stream, (const float *)m->Y, G, p,
                       m->gam, m->bet, tgt ? (const double *)m->gt : nullptr,
                       tgt ? (const double *)m->bt : nullptr, tgt ? m->dY : nullptr, tgt ? m->dY16 : nullptr,
                       tgt ? m->sq : nullptr);
    MCHECK(m, hipGetLastError());
    if (tgt) {
        hipLaunchKernelGGL(qm::k_sum, dim3(1), dim3(256), 0, m->stream, (const double *)m->sq, (int64_t)G * 2 * p,
                           m->loss);
        MCHECK(m, hipGetLastError());
    }
    if (gamma) MCHECK(m, hipMemcpyAsync(gamma, m->gam, (size_t)G * p * 8, hipMemcpyDeviceToHost, m->stream));
    if (beta) MCHECK(m, hipMemcpyAsync(beta, m->bet, (size_t)G * p * 8, hipMemcpyDeviceToHost, m->stream));
    if (loss && tgt) {
        double s = 0.0;
        MCHECK(m, hipMemcpyAsync(&s, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
        MCHECK(m, hipStreamSynchronize(m->stream));
        *loss = s / (2.0 * p * G);
    }
    MCHECK(m, hipStreamSynchronize(m->stream));
    return QAOA_OK;
}

qaoa_status check_model(qaoa_mpnn m)
{
    if (!m) return mfail(QAOA_ERR_INVALID_ARGUMENT, "model is NULL");
    if (m->poisoned) return mfail(QAOA_ERR_DEVICE, "model is unusable after an earlier device error");
    return QAOA_OK;
}

qaoa_status check_targets(int32_t count, int p, const double *gt, const double *bt)
{
    if (!gt || !bt) return mfail(QAOA_ERR_INVALID_ARGUMENT, "targets are NULL");
    for (int64_t i = 0; i < (int64_t)count * p; ++i)
        if (!std::isfinite(gt[i]) || !std::isfinite(bt[i]))
            return mfail(QAOA_ERR_INVALID_ARGUMENT, "targets must be finite");
    return QAOA_OK;
}

struct MDevice {
    int old = -1;
    explicit MDevice(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) (void)hipSetDevice(dev);
    }
    ~MDevice()
    {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

}  // namespace

extern "C" {

qaoa_status qaoa_mpnn_num_params(int32_t p, int64_t *count)
{
    if (p < 1 || p > 16 || !count) return mfail(QAOA_ERR_INVALID_ARGUMENT, "p must be in [1, 16], count non-NULL");
    *count = Layout(p).total;
    return QAOA_OK;
}

qaoa_status qaoa_mpnn_create(int32_t p, qaoa_mpnn *out)
{
    if (!out) return mfail(QAOA_ERR_INVALID_ARGUMENT, "out is NULL");
    if (p < 1 || p > 16) return mfail(QAOA_ERR_INVALID_ARGUMENT, "p must be in [1, 16]");
    qaoa_mpnn m = new (std::nothrow) qaoa_mpnn_s();
    if (!m) return mfail(QAOA_ERR_OUT_OF_MEMORY, "host allocation");
    m->p = p;
    m->lay = Layout(p);
    auto bad = [&](const char *msg) {
        qaoa_mpnn_destroy(m);
        return mfail(QAOA_ERR_DEVICE, msg);
    };
    if (hipGetDevice(&m->device) != hipSuccess) return bad("hipGetDevice failed");
    if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) return bad("stream creation failed");
    const size_t P = (size_t)m->lay.total;
    if (hipMalloc((void **)&m->theta, P * 4) != hipSuccess || hipMalloc((void **)&m->grad, P * 4) != hipSuccess ||
        hipMalloc((void **)&m->am, P * 4) != hipSuccess || hipMalloc((void **)&m->av, P * 4) != hipSuccess ||
        hipMalloc((void **)&m->theta16, P * 2) != hipSuccess)
        return bad("parameter allocation failed");
    if (hipMemsetAsync(m->theta, 0, P * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->grad, 0, P * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->am, 0, P * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->av, 0, P * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->theta16, 0, P * 2, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return bad("parameter initialisation failed");
    *out = m;
    return QAOA_OK;
}

qaoa_status qaoa_mpnn_destroy(qaoa_mpnn m)
{
    if (!m) return QAOA_OK;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    for (void *p : {(void *)m->theta, (void *)m->grad, (void *)m->am, (void *)m->av, (void *)m->theta16, m->ws})
        if (p) (void)hipFree(p);
    if (m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return QAOA_OK;
}

qaoa_status qaoa_mpnn_set_params(qaoa_mpnn m, const float *theta)
{
    MTRY(check_model(m));
    if (!theta) return mfail(QAOA_ERR_INVALID_ARGUMENT, "theta is NULL");
    const int64_t P = m->lay.total;
    for (int64_t i = 0; i < P; ++i)
        if (!std::isfinite(theta[i])) return mfail(QAOA_ERR_INVALID_ARGUMENT, "parameters must be finite");
    MDevice dg(m->device);
    MCHECK(m, hipMemcpyAsync(m->theta, theta, P * 4, hipMemcpyHostToDevice, m->stream));
    MCHECK(m, hipMemsetAsync(m->am, 0, P * 4, m->stream));
    MCHECK(m, hipMemsetAsync(m->av, 0, P * 4, m->stream));
    hipLaunchKernelGGL(qm::k_to_bf16, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, m->stream,
                       (const float *)m->theta, m->theta16, P);
    MCHECK(m, hipGetLastError());
    MCHECK(m, hipStreamSynchronize(m->stream));
    m->step = 0;
    return QAOA_OK;
}

qaoa_status qaoa_mpnn_get_params(qaoa_mpnn m, float *theta)
{
    MTRY(check_model(m));
    if (!theta) return mfail(QAOA_ERR_INVALID_ARGUMENT, "theta is NULL");
    MDevice dg(m->device);
    MCHECK(m, hipMemcpyAsync(theta, m->theta, m->lay.total * 4, hipMemcpyDeviceToHost, m->stream));
    MCHECK(m, hipStreamSynchronize(m->stream));
    return QAOA_OK;
}

qaoa_status qaoa_mpnn_predict(qaoa_mpnn m, int32_t count, const int32_t *n, const int64_t *edge_offsets,
                              const int32_t *edges, const double *w, double *gamma, double *beta)
{
    MTRY(check_model(m));
    if (!gamma || !beta) return mfail(QAOA_ERR_INVALID_ARGUMENT, "outputs are NULL");
    GraphBatch B;
    MTRY(build_batch(count, n, edge_offsets, edges, w, B));
    MDevice dg(m->device);
    MTRY(upload_batch(m, B));
    MTRY(forward(m, B));
    return angles_and_loss(m, B, nullptr, nullptr, gamma, beta, nullptr);
}

qaoa_status qaoa_mpnn_loss_grad(qaoa_mpnn m, int32_t count, const int32_t *n, const int64_t *edge_offsets,
                                const int32_t *edges, const double *w, const double *gamma_t,
                                const double *beta_t, double *loss, float *grad)
{
    MTRY(check_model(m));
    MTRY(check_targets(count, m->p, gamma_t, beta_t));
    GraphBatch B;
    MTRY(build_batch(count, n, edge_offsets, edges, w, B));
    MDevice dg(m->device);
    MTRY(upload_batch(m, B));
    MTRY(forward(m, B));
    MTRY(angles_and_loss(m, B, gamma_t, beta_t, nullptr, nullptr, loss));
    MTRY(backward(m, B));
    if (grad) MCHECK(m, hipMemcpyAsync(grad, m->grad, m->lay.total * 4, hipMemcpyDeviceToHost, m->stream));
    MCHECK(m, hipStreamSynchronize(m->stream));
    return QAOA_OK;
}

qaoa_status qaoa_mpnn_train_step(qaoa_mpnn m, int32_t count, const int32_t *n, const int64_t *edge_offsets,
                                 const int32_t *edges, const double *w, const double *gamma_t,
                                 const double *beta_t, const qaoa_mpnn_adam *opt, double *loss)
{
    MTRY(check_model(m));
    qaoa_mpnn_adam o = {1e-3, 0.9, 0.999, 1e-8};
    if (opt) o = *opt;
    if (!(o.lr > 0.0) || !(o.beta1 >= 0.0 && o.beta1 < 1.0) || !(o.beta2 >= 0.0 && o.beta2 < 1.0) ||
        !(o.eps > 0.0))
        return mfail(QAOA_ERR_INVALID_ARGUMENT, "invalid Adam options");
    MTRY(check_targets(count, m->p, gamma_t, beta_t));
    GraphBatch B;
    MTRY(build_batch(count, n, edge_offsets, edges, w, B));
    MDevice dg(m->device);
    MTRY(upload_batch(m, B));
    MTRY(forward(m, B));
    MTRY(angles_and_loss(m, B, gamma_t, beta_t, nullptr, nullptr, loss));
    MTRY(backward(m, B));
    const int64_t t = m->step + 1;
    const float c1 = (float)(1.0 - std::pow(o.beta1, (double)t)), c2 = (float)(1.0 - std::pow(o.beta2, (double)t));
    const int64_t P = m->lay.total;
    hipLaunchKernelGGL(qm::k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, m->stream, m->theta,
                       (const float *)m->grad, m->am, m->av, m->theta16, P, (float)o.lr, (float)o.beta1,
                       (float)o.beta2, (float)o.eps, c1, c2);
    MCHECK(m, hipGetLastError());
    MCHECK(m, hipStreamSynchronize(m->stream));
    m->step = t;
    return QAOA_OK;
}

}  // extern "C"
