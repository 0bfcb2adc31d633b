// Limited-memory BFGS (the optimiser the paper offers natively, Sec. V-B;
// Liu & Nocedal 1989) for the QAOA angles.
//
// Written from the textbook description (Nocedal & Wright, Numerical
// Optimization, 2nd ed.): the two-loop recursion for the search direction
// (Alg. 7.4) with the scaled identity H0 = (s.y)/(y.y) I, and a line search
// that enforces the strong Wolfe conditions by bracketing and zooming with
// safeguarded cubic interpolation (Alg. 3.5 / 3.6).  Every trial point costs
// one objective-and-gradient evaluation; for QAOA that is one qaoa_gradient
// call (expectation and all 2p partial derivatives).
#include "qaoa.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

namespace {

struct Eval {
    double a, f, d;  // step, objective, directional derivative
};

double dot(const std::vector<double> &a, const std::vector<double> &b)
{
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// Minimiser of the cubic through (a, fa, da), (b, fb, db); falls back to
// bisection when the cubic has no real minimiser inside the interval.
double cubic_min(const Eval &p, const Eval &q)
{
    const double d1 = p.d + q.d - 3.0 * (p.f - q.f) / (p.a - q.a);
    const double disc = d1 * d1 - p.d * q.d;
    if (disc < 0.0) return 0.5 * (p.a + q.a);
    const double d2 = std::copysign(std::sqrt(disc), q.a - p.a);
    const double den = q.d - p.d + 2.0 * d2;
    if (den == 0.0) return 0.5 * (p.a + q.a);
    return q.a - (q.a - p.a) * (q.d + d2 - d1) / den;
}

struct Problem {
    int dim;
    qaoa_objective_fn fn;
    void *user;
    int evals = 0;
    int max_evals;
    std::vector<double> x0, d, xt, gt;
    // f and g at x0 + a d
    bool eval(double a, Eval *e)
    {
        if (evals >= max_evals) return false;
        for (int i = 0; i < dim; ++i) xt[i] = x0[i] + a * d[i];
        double f = 0.0;
        ++evals;
        if (fn(xt.data(), &f, gt.data(), user) != 0 || !std::isfinite(f)) return false;
        e->a = a;
        e->f = f;
        e->d = dot(gt, d);
        return std::isfinite(e->d);
    }
};

// Strong-Wolfe line search; on success leaves the accepted point in
// pr.xt / pr.gt and its value in *acc.
bool wolfe_search(Problem &pr, const Eval &e0, double a1, Eval *acc)
{
    const double c1 = 1e-4, c2 = 0.9, amax = 1e10;
    Eval prev = e0, cur;
    double a = a1;
    auto zoom = [&](Eval lo, Eval hi) -> bool {
        for (int it = 0; it < 30; ++it) {
            double t = cubic_min(lo, hi);
            const double l = std::min(lo.a, hi.a), u = std::max(lo.a, hi.a);
            if (!(t > l + 0.1 * (u - l) && t < u - 0.1 * (u - l))) t = 0.5 * (lo.a + hi.a);
            Eval e;
            if (!pr.eval(t, &e)) return false;
            if (e.f > e0.f + c1 * t * e0.d || e.f >= lo.f) {
                hi = e;
            } else {
                if (std::fabs(e.d) <= -c2 * e0.d) {
                    *acc = e;
                    return true;
                }
                if (e.d * (hi.a - lo.a) >= 0.0) hi = lo;
                lo = e;
            }
            if (std::fabs(hi.a - lo.a) < 1e-16 * std::max(1.0, std::fabs(lo.a))) break;
        }
        // interval collapsed: accept the best point if it decreased f
        if (lo.a > 0.0 && lo.f < e0.f) {
            Eval e;
            if (!pr.eval(lo.a, &e)) return false;
            *acc = e;
            return true;
        }
        return false;
    };
    for (int i = 1; i <= 40; ++i) {
        if (!pr.eval(a, &cur)) return false;
        if (cur.f > e0.f + c1 * a * e0.d || (i > 1 && cur.f >= prev.f)) return zoom(prev, cur);
        if (std::fabs(cur.d) <= -c2 * e0.d) {
            *acc = cur;
            return true;
        }
        if (cur.d >= 0.0) return zoom(cur, prev);
        prev = cur;
        a = std::min(2.0 * a, amax);
    }
    return false;
}

}  // namespace

extern "C" qaoa_status qaoa_lbfgs_minimize(int32_t dim, double *x, qaoa_objective_fn fn, void *user,
                                           const qaoa_lbfgs_options *opt, double *fx,
                                           int32_t *iters, int32_t *evals, double *trace_x,
                                           double *trace_f)
{
    if (dim < 1 || !x || !fn) return QAOA_ERR_INVALID_ARGUMENT;
    qaoa_lbfgs_options o = {100, 10, 1e-8, 0.0, 1000};
    if (opt) o = *opt;
    if (o.max_iter < 0 || o.history < 1 || o.max_evals < 1 || !(o.gtol >= 0.0) || !(o.ftol >= 0.0))
        return QAOA_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < dim; ++i)
        if (!std::isfinite(x[i])) return QAOA_ERR_INVALID_ARGUMENT;

    Problem pr;
    pr.dim = dim;
    pr.fn = fn;
    pr.user = user;
    pr.max_evals = o.max_evals;
    pr.x0.assign(x, x + dim);
    pr.d.assign(dim, 0.0);
    pr.xt.assign(dim, 0.0);
    pr.gt.assign(dim, 0.0);

    std::vector<double> g(dim);
    double f = 0.0;
    pr.evals = 1;
    if (fn(pr.x0.data(), &f, g.data(), user) != 0 || !std::isfinite(f)) return QAOA_ERR_DEVICE;
    std::deque<std::vector<double>> S, Y;
    std::deque<double> rho;
    int k = 0;
    if (trace_x) std::memcpy(trace_x, pr.x0.data(), sizeof(double) * dim);
    if (trace_f) trace_f[0] = f;
    auto gnorm = [&] {
        double m = 0.0;
        for (double v : g) m = std::max(m, std::fabs(v));
        return m;
    };
    while (k < o.max_iter && gnorm() > o.gtol) {
        // two-loop recursion: d = -H g
        std::vector<double> q = g, al(S.size());
        for (int i = (int)S.size() - 1; i >= 0; --i) {
            al[i] = rho[i] * dot(S[i], q);
            for (int j = 0; j < dim; ++j) q[j] -= al[i] * Y[i][j];
        }
        double h0 = 1.0;
        if (!S.empty()) h0 = dot(S.back(), Y.back()) / dot(Y.back(), Y.back());
        for (int j = 0; j < dim; ++j) q[j] *= h0;
        for (size_t i = 0; i < S.size(); ++i) {
            const double b = rho[i] * dot(Y[i], q);
            for (int j = 0; j < dim; ++j) q[j] += S[i][j] * (al[i] - b);
        }
        for (int j = 0; j < dim; ++j) pr.d[j] = -q[j];
        double d0 = dot(g, pr.d);
        if (!(d0 < 0.0)) {  // not a descent direction: restart from steepest descent
            S.clear();
            Y.clear();
            rho.clear();
            for (int j = 0; j < dim; ++j) pr.d[j] = -g[j];
            d0 = dot(g, pr.d);
        }
        const double a1 = S.empty() ? std::min(1.0, 1.0 / std::max(gnorm(), 1e-300)) : 1.0;
        Eval e0{0.0, f, d0}, acc;
        if (!wolfe_search(pr, e0, a1, &acc)) break;
        std::vector<double> s(dim), y(dim);
        for (int j = 0; j < dim; ++j) {
            s[j] = pr.xt[j] - pr.x0[j];
            y[j] = pr.gt[j] - g[j];
        }
        const double f_old = f;
        pr.x0 = pr.xt;
        g = pr.gt;
        f = acc.f;
        ++k;
        if (trace_x) std::memcpy(trace_x + (size_t)k * dim, pr.x0.data(), sizeof(double) * dim);
        if (trace_f) trace_f[k] = f;
        const double sy = dot(s, y);
        if (sy > 1e-12 * std::sqrt(dot(s, s) * dot(y, y))) {
            S.push_back(s);
            Y.push_back(y);
            rho.push_back(1.0 / sy);
            if ((int)S.size() > o.history) {
                S.pop_front();
                Y.pop_front();
                rho.pop_front();
            }
        }
        if (o.ftol > 0.0 && std::fabs(f_old - f) <= o.ftol * std::max(1.0, std::fabs(f))) break;
    }
    std::memcpy(x, pr.x0.data(), sizeof(double) * dim);
    if (fx) *fx = f;
    if (iters) *iters = k;
    if (evals) *evals = pr.evals;
    return QAOA_OK;
}

namespace {

struct QaoaObjective {
    qaoa_handle h;
    int32_t p;
    qaoa_status status;
};

// f = -E(gamma, beta), g = -(dE/dgamma, dE/dbeta); x = (gamma, beta).
int qaoa_negated_objective(const double *x, double *f, double *g, void *user)
{
    QaoaObjective *o = (QaoaObjective *)user;
    double E = 0.0;
    o->status = qaoa_gradient(o->h, o->p, x, x + o->p, &E, g, g + o->p);
    if (o->status != QAOA_OK) return 1;
    *f = -E;
    for (int i = 0; i < 2 * o->p; ++i) g[i] = -g[i];
    return 0;
}

}  // namespace

extern "C" qaoa_status qaoa_optimize(qaoa_handle h, int32_t p, double *gamma, double *beta,
                                     const qaoa_lbfgs_options *opt, double *E, int32_t *iters,
                                     int32_t *evals, double *trace_x, double *trace_f)
{
    if (!h || p < 1 || !gamma || !beta) return QAOA_ERR_INVALID_ARGUMENT;
    std::vector<double> x(2 * (size_t)p);
    for (int i = 0; i < p; ++i) {
        x[i] = gamma[i];
        x[p + i] = beta[i];
    }
    QaoaObjective obj{h, p, QAOA_OK};
    double fx = 0.0;
    qaoa_status st = qaoa_lbfgs_minimize(2 * p, x.data(), qaoa_negated_objective, &obj, opt, &fx,
                                         iters, evals, trace_x, trace_f);
    if (obj.status != QAOA_OK) return obj.status;
    if (st != QAOA_OK) return st;
    for (int i = 0; i < p; ++i) {
        gamma[i] = x[i];
        beta[i] = x[p + i];
    }
    if (trace_f) {
        const int k = iters ? *iters : 0;
        for (int i = 0; i <= k; ++i) trace_f[i] = -trace_f[i];
    }
    if (E) *E = -fx;
    return QAOA_OK;
}
