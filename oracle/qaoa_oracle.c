/*
 * qaoa_oracle.c -- plain, slow FP64 CPU reference for the QAOA hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the package's smoke check and the
 * benchmark's CPU-baseline leg load it (through oracle/__init__.py).  It shares
 * no code, header, table or helper with the GPU path.
 *
 * Every routine follows the paper's definitions directly, in the order the
 * paper states them, without blocking or fusion:
 *
 *   cost diagonal   Sec. IV-A, Eq. (2): f(x) = sum_k w_k [term k active in x],
 *                   a term being active iff every one of its variables is 1.
 *                   MaxCut uses the cut indicator x_i XOR x_j per edge.
 *   initial state   Sec. II-A (ground state of the X mixer) and Sec. IV-B:
 *                   every amplitude equals 1/sqrt(2^n).
 *   phase layer     Sec. IV-B: psi_z <- [cos(-g f_z) + i sin(-g f_z)] psi_z.
 *   mixer layer     Eq. (1), Sec. IV-B: one single-qubit rotation per qubit,
 *                   applied qubit after qubit, exp(-i b X_j)  (sign reading:
 *                   the Farhi form; the paper's H_M = -sum X gives b -> -b).
 *   expectation     Sec. IV-D: E = sum_z f(z) |psi_z|^2.
 *   gradient        Sec. II-B and IV-C (adjoint differentiation): with every
 *                   layer state stored, dE/dtheta_k = 2 Im <lam_k|H_k|phi_k>,
 *                   lam_k = U_{k+1}^dag ... U_{2p}^dag C psi.
 *   sampling        Sec. IV-D: draw z with probability |psi_z|^2 and return it
 *                   together with f(z).  Uniforms come from Philox-4x32-10
 *                   (Salmon et al., SC'11); the shot index is the counter.
 *
 * All arithmetic is IEEE fp64 round-to-nearest; the build uses
 * -ffp-contract=off so no multiply-add is fused behind the reader's back.
 * Sums over the 2^n basis states use Neumaier compensation in fixed chunks, so
 * results do not depend on the number of OpenMP threads.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ sums */

typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum *a) { return a->s + a->c; }

#define ORACLE_CHUNKS 256

/* Number of OpenMP threads the parallel loops below use. */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ cost */

/* MaxCut: f(z) = sum of w_k over edges (i,j) with bit i of z != bit j of z,
 * accumulated in edge order.  w == NULL means unit weights. */
double oracle_cost_maxcut_entry(uint64_t z, int64_t m, const int32_t *edges, const double *w)
{
    double acc = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        int i = edges[2 * k], j = edges[2 * k + 1];
        int xi = (int)((z >> i) & 1u), xj = (int)((z >> j) & 1u);
        if (xi != xj) acc = acc + (w ? w[k] : 1.0);
    }
    return acc;
}

void oracle_cost_maxcut(int n, int64_t m, const int32_t *edges, const double *w, double *C)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) C[z] = oracle_cost_maxcut_entry((uint64_t)z, m, edges, w);
}

/* 0-1 QUBO: f(z) = offset + sum_k J_k x_i x_j + sum_i h_i x_i with x_i = bit i of z.
 * Accumulated as: offset, then the pair terms in the given order, then the
 * linear terms in variable order; inactive terms are skipped.  h == NULL means
 * no linear terms. */
double oracle_cost_qubo_entry(uint64_t z, int n, int64_t m, const int32_t *pairs,
                              const double *J, const double *h, double offset)
{
    double acc = offset;
    for (int64_t k = 0; k < m; ++k) {
        int i = pairs[2 * k], j = pairs[2 * k + 1];
        if (((z >> i) & 1u) && ((z >> j) & 1u)) acc = acc + J[k];
    }
    if (h)
        for (int i = 0; i < n; ++i)
            if ((z >> i) & 1u) acc = acc + h[i];
    return acc;
}

void oracle_cost_qubo(int n, int64_t m, const int32_t *pairs, const double *J,
                      const double *h, double offset, double *C)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z)
        C[z] = oracle_cost_qubo_entry((uint64_t)z, n, m, pairs, J, h, offset);
}

/* General 0-1 polynomial of Eq. (2): term k carries the mask m_k = sum_{i in t_k} 2^i
 * and is active in z iff (z AND m_k) == m_k.  Terms are added in order. */
double oracle_cost_poly_entry(uint64_t z, int64_t L, const uint64_t *masks, const double *w)
{
    double acc = 0.0;
    for (int64_t k = 0; k < L; ++k)
        if ((z & masks[k]) == masks[k]) acc = acc + w[k];
    return acc;
}

void oracle_cost_poly(int n, int64_t L, const uint64_t *masks, const double *w, double *C)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) C[z] = oracle_cost_poly_entry((uint64_t)z, L, masks, w);
}

/* ------------------------------------------------------------- evolution */

void oracle_init_plus(int n, cplx *psi)
{
    const int64_t N = (int64_t)1 << n;
    const double a = 1.0 / sqrt((double)N);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) psi[z] = a;
}

/* psi_z <- exp(-i g C_z) psi_z, written with Euler's formula. */
void oracle_apply_phase(int n, const double *C, double g, cplx *psi)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) {
        double th = -g * C[z];
        psi[z] = (cos(th) + I * sin(th)) * psi[z];
    }
}

/* exp(-i b X) on qubit j: (a, b') <- (cos b a - i sin b b', -i sin b a + cos b b'). */
void oracle_apply_rx(int n, int j, double b, cplx *psi)
{
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t bit = (int64_t)1 << j;
    const double c = cos(b), s = sin(b);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < half; ++t) {
        /* t enumerates indices with bit j removed; re-insert a 0 at bit j. */
        int64_t z0 = ((t >> j) << (j + 1)) | (t & (bit - 1));
        int64_t z1 = z0 | bit;
        cplx a0 = psi[z0], a1 = psi[z1];
        psi[z0] = c * a0 - I * s * a1;
        psi[z1] = -I * s * a0 + c * a1;
    }
}

void oracle_apply_mixer(int n, double b, cplx *psi)
{
    for (int j = 0; j < n; ++j) oracle_apply_rx(n, j, b, psi);
}

/* psi = U_M(b_p) U_C(g_p) ... U_M(b_1) U_C(g_1) |+>^n   (Eq. (1)). */
void oracle_state(int n, const double *C, int p, const double *g, const double *b, cplx *psi)
{
    oracle_init_plus(n, psi);
    for (int l = 0; l < p; ++l) {
        oracle_apply_phase(n, C, g[l], psi);
        oracle_apply_mixer(n, b[l], psi);
    }
}

/* E = sum_z C_z |psi_z|^2 (Sec. IV-D), compensated, thread-count independent. */
double oracle_expectation(int n, const double *C, const cplx *psi)
{
    const int64_t N = (int64_t)1 << n;
    nsum part[ORACLE_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int q = 0; q < ORACLE_CHUNKS; ++q) {
        nsum a = {0.0, 0.0};
        int64_t lo = N * q / ORACLE_CHUNKS, hi = N * (q + 1) / ORACLE_CHUNKS;
        for (int64_t z = lo; z < hi; ++z) {
            double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
            nsum_add(&a, C[z] * pr);
        }
        part[q] = a;
    }
    nsum tot = {0.0, 0.0};
    for (int q = 0; q < ORACLE_CHUNKS; ++q) { nsum_add(&tot, part[q].s); nsum_add(&tot, part[q].c); }
    return nsum_value(&tot);
}

/* Im <lam| C |phi> = Im sum_z conj(lam_z) C_z phi_z */
static double im_inner_cost(int n, const double *C, const cplx *lam, const cplx *phi)
{
    const int64_t N = (int64_t)1 << n;
    nsum part[ORACLE_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int q = 0; q < ORACLE_CHUNKS; ++q) {
        nsum a = {0.0, 0.0};
        int64_t lo = N * q / ORACLE_CHUNKS, hi = N * (q + 1) / ORACLE_CHUNKS;
        for (int64_t z = lo; z < hi; ++z) nsum_add(&a, cimag(conj(lam[z]) * C[z] * phi[z]));
        part[q] = a;
    }
    nsum tot = {0.0, 0.0};
    for (int q = 0; q < ORACLE_CHUNKS; ++q) { nsum_add(&tot, part[q].s); nsum_add(&tot, part[q].c); }
    return nsum_value(&tot);
}

/* Im <lam| sum_j X_j |phi> = Im sum_z conj(lam_z) sum_j phi_{z xor 2^j} */
static double im_inner_mixer(int n, const cplx *lam, const cplx *phi)
{
    const int64_t N = (int64_t)1 << n;
    nsum part[ORACLE_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int q = 0; q < ORACLE_CHUNKS; ++q) {
        nsum a = {0.0, 0.0};
        int64_t lo = N * q / ORACLE_CHUNKS, hi = N * (q + 1) / ORACLE_CHUNKS;
        for (int64_t z = lo; z < hi; ++z)
            for (int j = 0; j < n; ++j)
                nsum_add(&a, cimag(conj(lam[z]) * phi[z ^ ((int64_t)1 << j)]));
        part[q] = a;
    }
    nsum tot = {0.0, 0.0};
    for (int q = 0; q < ORACLE_CHUNKS; ++q) { nsum_add(&tot, part[q].s); nsum_add(&tot, part[q].c); }
    return nsum_value(&tot);
}

/*
 * Adjoint gradient (Sec. II-B, Sec. IV-C).  The circuit has 2p layers
 * U_1 = U_C(g_1), U_2 = U_M(b_1), ..., U_2p = U_M(b_p).  All 2p+1 states
 * phi_k = U_k ... U_1 |+> are stored.  Starting from lam = C phi_2p the sweep
 * runs k = 2p..1:  g_k = 2 Im <lam|H_k|phi_k>, then lam <- U_k^dag lam, where
 * H_k is C for a phase layer and sum_j X_j for a mixer layer (the generator of
 * U_k = exp(-i theta_k H_k)).  Returns 0 on success, -1 if memory runs out.
 */
int oracle_gradient(int n, const double *C, int p, const double *g, const double *b,
                    double *E, double *dg, double *db)
{
    const int64_t N = (int64_t)1 << n;
    const int K = 2 * p;
    cplx **phi = (cplx **)calloc((size_t)K + 1, sizeof(cplx *));
    cplx *lam = (cplx *)malloc((size_t)N * sizeof(cplx));
    int ok = phi && lam;
    for (int k = 0; ok && k <= K; ++k) ok = (phi[k] = (cplx *)malloc((size_t)N * sizeof(cplx))) != NULL;
    if (!ok) {
        if (phi) for (int k = 0; k <= K; ++k) free(phi[k]);
        free(phi); free(lam);
        return -1;
    }

    oracle_init_plus(n, phi[0]);
    for (int k = 1; k <= K; ++k) {
        memcpy(phi[k], phi[k - 1], (size_t)N * sizeof(cplx));
        int l = (k - 1) / 2;
        if (k % 2 == 1) oracle_apply_phase(n, C, g[l], phi[k]);
        else            oracle_apply_mixer(n, b[l], phi[k]);
    }
    *E = oracle_expectation(n, C, phi[K]);

#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) lam[z] = C[z] * phi[K][z];

    for (int k = K; k >= 1; --k) {
        int l = (k - 1) / 2;
        if (k % 2 == 1) {
            dg[l] = 2.0 * im_inner_cost(n, C, lam, phi[k]);
            oracle_apply_phase(n, C, -g[l], lam);          /* U_C(g)^dag = U_C(-g) */
        } else {
            db[l] = 2.0 * im_inner_mixer(n, lam, phi[k]);
            oracle_apply_mixer(n, -b[l], lam);             /* U_M(b)^dag = U_M(-b) */
        }
    }

    for (int k = 0; k <= K; ++k) free(phi[k]);
    free(phi); free(lam);
    return 0;
}

/* ------------------------------------------------------------- sampling */

/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
 * (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
 * with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by the Weyl
 * constants (0x9E3779B9, 0xBB67AE85) before every round after the first. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in [0,1) for shot s: counter (s_lo, s_hi, 0, 0), key (seed_lo, seed_hi);
 * the top 53 bits of the 64-bit word (out1:out0) scaled by 2^-53. */
double oracle_uniform53(uint64_t seed, uint64_t s)
{
    uint32_t ctr[4] = {(uint32_t)s, (uint32_t)(s >> 32), 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    oracle_philox4x32_10(ctr, key, o);
    uint64_t x = ((uint64_t)o[1] << 32) | o[0];
    return (double)(x >> 11) * 0x1.0p-53;
}

/*
 * Sampling (Sec. IV-D).  S_z is the running (compensated) sum of |psi_y|^2 over
 * y <= z, made non-decreasing; T = S_{N-1}.  Shot s draws u_s, sets t = u_s T and
 * returns the smallest z with S_z > t, together with C_z.  A basis state with
 * zero probability is never returned.  C may be NULL (then cost is not written).
 * Returns 0, or -1 if memory runs out or the state has zero norm.
 */
int oracle_sample(int n, const cplx *psi, const double *C, int64_t shots, uint64_t seed,
                  uint64_t *zout, double *cost)
{
    const int64_t N = (int64_t)1 << n;
    double *S = (double *)malloc((size_t)N * sizeof(double));
    if (!S) return -1;
    nsum run = {0.0, 0.0};
    double prev = 0.0;
    for (int64_t z = 0; z < N; ++z) {
        double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
        nsum_add(&run, pr);
        double v = nsum_value(&run);
        if (v < prev) v = prev;     /* guard against a last-ulp step down */
        S[z] = prev = v;
    }
    const double T = S[N - 1];
    if (!(T > 0.0)) { free(S); return -1; }
    for (int64_t s = 0; s < shots; ++s) {
        double t = oracle_uniform53(seed, (uint64_t)s) * T;
        int64_t lo = 0, hi = N - 1;          /* first z with S_z > t; S_{N-1} = T > t */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (S[mid] > t) hi = mid; else lo = mid + 1;
        }
        zout[s] = (uint64_t)lo;
        if (cost) cost[s] = C[lo];
    }
    free(S);
    return 0;
}
