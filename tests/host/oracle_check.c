/* Host check of the CPU oracle (run under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py): every routine
 * on small MaxCut, QUBO and polynomial instances, n = 1..9 and p = 0..3, with
 * all buffers sized exactly.  Values are pinned elsewhere; this checks memory
 * and arithmetic safety only. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;
void oracle_cost_maxcut(int n, int64_t m, const int32_t *edges, const double *w, double *C);
void oracle_cost_qubo(int n, int64_t m, const int32_t *pairs, const double *J, const double *h,
                      double offset, double *C);
void oracle_cost_poly(int n, int64_t L, const uint64_t *masks, const double *w, double *C);
void oracle_state(int n, const double *C, int p, const double *g, const double *b, cplx *psi);
double oracle_expectation(int n, const double *C, const cplx *psi);
int oracle_gradient(int n, const double *C, int p, const double *g, const double *b, double *E,
                    double *dg, double *db);
int oracle_sample(int n, const cplx *psi, const double *C, int64_t shots, uint64_t seed, uint64_t *zout,
                  double *cost);

int main(void)
{
    for (int n = 1; n <= 9; ++n) {
        const int64_t N = (int64_t)1 << n;
        const int64_t m = n * (n - 1) / 2;
        int32_t *pairs = malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
        double *w = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
        double *h = malloc((size_t)n * sizeof(double));
        uint64_t *masks = malloc((size_t)n * sizeof(uint64_t));
        int64_t k = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                pairs[2 * k] = i;
                pairs[2 * k + 1] = j;
                w[k] = 0.25 * (double)((i + 2 * j) % 7) - 0.5;
                ++k;
            }
        for (int i = 0; i < n; ++i) {
            h[i] = 0.1 * i - 0.3;
            masks[i] = ((uint64_t)1 << i) | ((uint64_t)1 << ((i + 1) % n));
        }
        double *C = malloc((size_t)N * sizeof(double));
        cplx *psi = malloc((size_t)N * sizeof(cplx));
        oracle_cost_maxcut(n, m, pairs, w, C);
        oracle_cost_maxcut(n, m, pairs, NULL, C);
        oracle_cost_poly(n, n, masks, h, C);
        oracle_cost_qubo(n, m, pairs, w, h, 0.5, C);
        for (int p = 0; p <= 3; ++p) {
            double g[3] = {0.3, -0.7, 1.1}, b[3] = {0.4, 1.3, -0.2}, E, dg[3], db[3];
            oracle_state(n, C, p, g, b, psi);
            (void)oracle_expectation(n, C, psi);
            if (p > 0 && oracle_gradient(n, C, p, g, b, &E, dg, db) != 0) {
                printf("gradient failed: n=%d p=%d\n", n, p);
                return 1;
            }
            uint64_t z[64];
            double cost[64];
            if (oracle_sample(n, psi, C, 64, 7, z, cost) != 0) {
                printf("sampling failed: n=%d p=%d\n", n, p);
                return 1;
            }
        }
        free(pairs);
        free(w);
        free(h);
        free(masks);
        free(C);
        free(psi);
    }
    printf("oracle ok\n");
    return 0;
}
