"""Host-side L-BFGS (the library's optimiser) on functions with known minima,
and against scipy's L-BFGS-B on a smooth problem.  CPU only: the objective is
a Python callback through the C ABI."""
import numpy as np
import pytest
import scipy.optimize


def rosen(x):
    f = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)
    g = np.zeros_like(x)
    g[:-1] = -400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2 * (1 - x[:-1])
    g[1:] += 200.0 * (x[1:] - x[:-1] ** 2)
    return f, g


@pytest.mark.parametrize("dim", [2, 5, 10])
def test_rosenbrock(dim):
    from paper_2407_13012_amd import qaoa_lbfgs_minimize
    x0 = np.full(dim, -1.2)
    x0[1::2] = 1.0
    x, f, it, ev = qaoa_lbfgs_minimize(rosen, x0, max_iter=500, gtol=1e-9, max_evals=5000)
    assert np.allclose(x, 1.0, atol=1e-6), (x, f, it)
    assert f < 1e-12
    assert ev >= it


def test_quadratic_converges_fast():
    from paper_2407_13012_amd import qaoa_lbfgs_minimize
    rng = np.random.default_rng(0)
    A = rng.normal(size=(6, 6))
    A = A @ A.T + 6 * np.eye(6)
    b = rng.normal(size=6)

    def fq(x):
        return 0.5 * x @ A @ x - b @ x, A @ x - b

    x, f, it, ev = qaoa_lbfgs_minimize(fq, np.zeros(6), max_iter=100, gtol=1e-12)
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)
    assert it <= 20


def test_matches_scipy_on_smooth_problem():
    from paper_2407_13012_amd import qaoa_lbfgs_minimize

    def fs(x):
        f = np.sum(np.cos(x) * np.exp(0.1 * x)) + 0.05 * np.sum(x ** 2)
        g = -np.sin(x) * np.exp(0.1 * x) + 0.1 * np.cos(x) * np.exp(0.1 * x) + 0.1 * x
        return f, g

    x0 = np.linspace(-1, 1, 8)
    x, f, it, ev = qaoa_lbfgs_minimize(fs, x0, max_iter=200, gtol=1e-10)
    ref = scipy.optimize.minimize(fs, x0, jac=True, method="L-BFGS-B",
                                  options=dict(gtol=1e-12, ftol=1e-15, maxiter=1000))
    assert abs(f - ref.fun) < 1e-10
    assert np.allclose(x, ref.x, atol=1e-6)


def test_trace_and_monotone_decrease():
    from paper_2407_13012_amd import qaoa_lbfgs_minimize
    x, f, it, ev, tx, tf = qaoa_lbfgs_minimize(rosen, np.array([-1.2, 1.0]), max_iter=100,
                                               gtol=1e-10, trace=True)
    assert tx.shape == (it + 1, 2) and tf.shape == (it + 1,)
    assert np.all(np.diff(tf) <= 1e-12)          # Wolfe steps decrease f
    assert np.allclose(tx[-1], x) and tf[-1] == f
    assert np.allclose(tx[0], [-1.2, 1.0])


def test_iteration_and_eval_caps_and_errors():
    from paper_2407_13012_amd import QaoaError, qaoa_lbfgs_minimize
    x, f, it, ev = qaoa_lbfgs_minimize(rosen, np.array([-1.2, 1.0]), max_iter=3)
    assert it == 3
    x, f, it, ev = qaoa_lbfgs_minimize(rosen, np.array([-1.2, 1.0]), max_iter=100, max_evals=7)
    assert ev <= 7
    with pytest.raises(QaoaError):
        qaoa_lbfgs_minimize(rosen, np.array([np.nan, 1.0]))
    with pytest.raises(QaoaError):
        qaoa_lbfgs_minimize(rosen, np.array([0.0, 1.0]), history=0)

    def bad(x):
        raise RuntimeError("boom")

    with pytest.raises(RuntimeError):
        qaoa_lbfgs_minimize(bad, np.zeros(2))
