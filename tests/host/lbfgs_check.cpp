// Host check of the L-BFGS driver (run under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py): Rosenbrock in
// 1..12 dimensions with several history lengths and full traces, an objective
// that turns non-finite, one that asks to stop, and a zero-iteration budget.
#include "qaoa.h"

#include <cmath>
#include <cstdio>
#include <vector>

// The library's qaoa_optimize calls qaoa_gradient; this check links the
// optimiser alone, so it provides a stand-in that is never reached.
extern "C" qaoa_status qaoa_gradient(qaoa_handle, int32_t, const double *, const double *, double *,
                                     double *, double *)
{
    return QAOA_ERR_UNSUPPORTED;
}

static int rosenbrock(const double *x, double *f, double *g, void *user)
{
    const int d = *(const int *)user;
    double s = 0.0;
    for (int i = 0; i < d; ++i) g[i] = 0.0;
    for (int i = 0; i + 1 < d; ++i) {
        const double a = x[i + 1] - x[i] * x[i], b = 1.0 - x[i];
        s += 100.0 * a * a + b * b;
        g[i] += -400.0 * a * x[i] - 2.0 * b;
        g[i + 1] += 200.0 * a;
    }
    *f = s;
    return 0;
}

static int turns_nan(const double *x, double *f, double *g, void *user)
{
    int *calls = (int *)user;
    *f = ++*calls > 3 ? NAN : x[0] * x[0];
    g[0] = 2.0 * x[0];
    return 0;
}

static int asks_stop(const double *x, double *f, double *g, void *user)
{
    *f = x[0];
    g[0] = 1.0;
    return ++*(int *)user > 2;
}

int main()
{
    for (int d = 1; d <= 12; ++d)
        for (int m = 1; m <= 11; m += 5) {
            std::vector<double> x((size_t)d, -1.2), tx((size_t)51 * d), tf(51);
            const qaoa_lbfgs_options o{50, m, 1e-10, 0.0, 400};
            double fx;
            int32_t it, ev;
            if (qaoa_lbfgs_minimize(d, x.data(), rosenbrock, &d, &o, &fx, &it, &ev, tx.data(),
                                    tf.data()) != QAOA_OK) {
                std::printf("rosenbrock failed: d=%d m=%d\n", d, m);
                return 1;
            }
        }
    double x1 = 3.0, fx;
    int32_t it, ev;
    int calls = 0;
    qaoa_lbfgs_minimize(1, &x1, turns_nan, &calls, nullptr, &fx, &it, &ev, nullptr, nullptr);
    calls = 0;
    x1 = 3.0;
    qaoa_lbfgs_minimize(1, &x1, asks_stop, &calls, nullptr, &fx, &it, &ev, nullptr, nullptr);
    const qaoa_lbfgs_options none{0, 1, 1e-8, 0.0, 1};
    int d1 = 1;
    x1 = 3.0;
    qaoa_lbfgs_minimize(1, &x1, rosenbrock, &d1, &none, &fx, &it, &ev, nullptr, nullptr);
    std::printf("lbfgs ok\n");
    return 0;
}
