"""GPU parity: every result of the HIP library against the CPU oracle.

Tolerances: cost diagonal bit-exact (same term order, plain fp64 adds);
complex128 expectation within 1e-10 * sum|w|; gradients within 1e-8 absolute;
complex128 amplitudes within 1e-12; complex64 results within 1e-4 relative;
samples identical shot by shot (same Philox stream, same inverse-CDF rule).
Sizes span the pass structure: n <= 12 (one tile, one group per layer),
13..22 (low group + one high group), 23+ (two high groups), with ragged high
groups.
"""
import math

import numpy as np
import pytest

import oracle
import qaoa_inputs as qi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2407_13012_amd import load_library
    load_library()


def H(inst, prec="c128"):
    from paper_2407_13012_amd import QaoaHandle
    return QaoaHandle.from_instance(inst, prec)


def tol_E(inst):
    w = inst.weight_array() if hasattr(inst, "edges") else np.concatenate([inst.J, inst.h])
    return 1e-10 * max(1.0, float(np.abs(w).sum()))


def mk(kind, n, seed):
    if kind == "er":
        return qi.erdos_renyi(n, 0.5, seed, weights="uniform", wlow=-1, whigh=1)
    if kind == "unit":
        return qi.erdos_renyi(n, 0.4, seed)
    if kind == "int":
        return qi.erdos_renyi(n, 0.5, seed, weights="integer", wlow=-3, whigh=5)
    if kind == "reg":
        return qi.random_regular(n if n % 2 == 0 else n + 1, 3, seed, weights="uniform")
    if kind == "qubo":
        return qi.qubo_erdos_renyi(n, 0.3, seed, offset=0.5)
    raise ValueError(kind)


SIZES = [1, 2, 3, 5, 8, 11, 12, 13, 14, 16, 17, 19, 20, 22, 23]


# ---------------------------------------------------------------- cost diagonal

@pytest.mark.parametrize("kind", ["unit", "int", "er", "qubo"])
@pytest.mark.parametrize("n", [1, 2, 5, 12, 13, 18, 21])
def test_cost_diagonal_bit_exact(kind, n):
    if kind != "qubo" and n < 2:
        pytest.skip("MaxCut needs two vertices")
    inst = mk(kind, n, 10 + n)
    C = oracle.cost_of(inst)
    with H(inst) as q:
        assert np.array_equal(q.cost_diagonal(), C)
        lo, hi = q.cost_extrema()
        assert lo == C.min() and hi == C.max()
    with H(inst, "c64") as q:
        assert np.array_equal(q.cost_diagonal(), C.astype(np.float32).astype(np.float64))


def test_cost_diagonal_device_output():
    import torch
    inst = mk("er", 14, 3)
    C = oracle.cost_of(inst)
    with H(inst) as q:
        out = torch.empty(1 << 14, dtype=torch.float64, device="cuda")
        q.cost_diagonal(out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), C)


# ---------------------------------------------------------------- state and expectation

@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [1, 3])
def test_statevector_and_expectation(n, p):
    inst = mk("qubo" if n < 3 else "er", n, 100 + n + p)
    C = oracle.cost_of(inst)
    gamma, beta = qi.uniform_angles(p, seed=[n, p])
    psi_ref = oracle.state(n, C, gamma, beta)
    E_ref = oracle.expectation(n, C, psi_ref)
    with H(inst) as q:
        psi = q.statevector(gamma, beta)
        assert np.max(np.abs(psi - psi_ref)) < 1e-12
        assert abs(q.expectation() - E_ref) <= tol_E(inst)
        assert abs(q.evaluate(gamma, beta) - E_ref) <= tol_E(inst)
        # evaluate leaves the state current
        assert abs(q.expectation() - E_ref) <= tol_E(inst)


def test_statevector_device_output_and_p0():
    import torch
    n = 15
    inst = mk("er", n, 7)
    C = oracle.cost_of(inst)
    with H(inst) as q:
        out = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        q.statevector([0.4, 0.9], [0.3, 0.1], out=out)
        torch.cuda.synchronize()
        assert np.max(np.abs(out.cpu().numpy() - oracle.state(n, C, [0.4, 0.9], [0.3, 0.1]))) < 1e-12
        psi0 = q.statevector([], [])
        assert np.max(np.abs(psi0 - 2 ** (-n / 2))) < 1e-16
        assert abs(q.expectation() - C.mean()) <= tol_E(inst)
        assert abs(q.evaluate([], []) - C.mean()) <= tol_E(inst)


# ---------------------------------------------------------------- gradient

@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [1, 2, 4])
def test_gradient(n, p):
    inst = mk("reg" if n >= 4 else "qubo", n, 200 + n + p)
    n = inst.n
    C = oracle.cost_of(inst)
    gamma, beta = qi.uniform_angles(p, seed=[n, 7 * p])
    E_ref, dg_ref, db_ref = oracle.gradient(n, C, gamma, beta)
    with H(inst) as q:
        E, dg, db = q.gradient(gamma, beta)
    assert abs(E - E_ref) <= tol_E(inst)
    assert np.max(np.abs(dg - dg_ref)) <= 1e-8, (dg, dg_ref)
    assert np.max(np.abs(db - db_ref)) <= 1e-8, (db, db_ref)


@pytest.mark.parametrize("kind", ["unit", "int", "qubo"])
def test_gradient_instance_kinds(kind):
    n, p = 18, 3
    inst = mk(kind, n, 31)
    C = oracle.cost_of(inst)
    gamma, beta = qi.ramp_with_noise(p, seed=[5, 5])
    E_ref, dg_ref, db_ref = oracle.gradient(n, C, gamma, beta)
    with H(inst) as q:
        E, dg, db = q.gradient(gamma, beta)
    assert abs(E - E_ref) <= tol_E(inst)
    assert np.max(np.abs(dg - dg_ref)) <= 1e-8
    assert np.max(np.abs(db - db_ref)) <= 1e-8


def test_gradient_edge_cases():
    # no edges: C = 0 everywhere, E = 0, zero gradient
    g = qi.MaxCut(n=6, edges=np.zeros((0, 2), dtype=np.int32), weights=None)
    with H(g) as q:
        E, dg, db = q.gradient([0.3, 0.2], [0.1, 0.7])
        assert E == 0.0 and np.all(dg == 0) and np.all(db == 0)
    # p = 0: E = mean C
    inst = mk("er", 9, 1)
    C = oracle.cost_of(inst)
    with H(inst) as q:
        E, dg, db = q.gradient([], [])
        assert abs(E - C.mean()) <= tol_E(inst) and dg.size == 0
    # angles at zero: E = mean C, gradient zero
    with H(inst) as q:
        E, dg, db = q.gradient([0.0, 0.0], [0.0, 0.0])
        assert abs(E - C.mean()) <= tol_E(inst)
        assert np.max(np.abs(dg)) < 1e-12 and np.max(np.abs(db)) < 1e-12


def test_gradient_consumes_state_and_is_deterministic():
    from paper_2407_13012_amd import QaoaError
    inst = mk("er", 20, 77)
    gamma, beta = qi.uniform_angles(3, seed=[1, 2])
    with H(inst) as q:
        r1 = q.gradient(gamma, beta)
        with pytest.raises(QaoaError) as ei:
            q.expectation()
        assert ei.value.status == 4
        r2 = q.gradient(gamma, beta)
        assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])
        # the handle stays usable for the forward path
        q.statevector(gamma, beta, copy=False)
        assert abs(q.expectation() - r1[0]) <= tol_E(inst)


def test_gradient_finite_difference_on_gpu():
    """GPU gradient against central differences of GPU expectations."""
    inst = mk("reg", 16, 5)
    gamma, beta = qi.uniform_angles(2, seed=[3, 3])
    h = 1e-6
    with H(inst) as q:
        _, dg, db = q.gradient(gamma, beta)
        for l in range(2):
            e = np.zeros(2)
            e[l] = h
            fg = (q.evaluate(gamma + e, beta) - q.evaluate(gamma - e, beta)) / (2 * h)
            fb = (q.evaluate(gamma, beta + e) - q.evaluate(gamma, beta - e)) / (2 * h)
            assert abs(fg - dg[l]) < 1e-7 and abs(fb - db[l]) < 1e-7


# ---------------------------------------------------------------- sampling

@pytest.mark.parametrize("n", [1, 3, 8, 12, 16, 20])
def test_samples_identical_to_oracle(n):
    inst = mk("qubo" if n < 3 else "er", n, 300 + n)
    C = oracle.cost_of(inst)
    gamma, beta = qi.uniform_angles(2, seed=[n, 11])
    psi = oracle.state(n, C, gamma, beta)
    shots = 4096
    z_ref, c_ref = oracle.sample(n, psi, C, shots, seed=12345)
    with H(inst) as q:
        q.statevector(gamma, beta, copy=False)
        z, c = q.sample(shots, 12345)
        z2, _ = q.sample(shots, 12345)
    assert np.array_equal(z, z2)
    mism = np.flatnonzero(z != z_ref)
    assert mism.size == 0, (mism[:10], z[mism[:10]], z_ref[mism[:10]])
    assert np.array_equal(c, C[z.astype(np.int64)]) and np.array_equal(c, c_ref)


def test_sampling_small_workload_and_device_output():
    import torch
    w = qi.workload_small()
    g = w["instance"]
    C = oracle.cost_of(g)
    psi = oracle.state(g.n, C, w["gamma"], w["beta"])
    z_ref, c_ref = oracle.sample(g.n, psi, C, w["shots"], w["sample_seed"])
    with H(g) as q:
        q.statevector(w["gamma"], w["beta"], copy=False)
        zt = torch.empty(w["shots"], dtype=torch.int64, device="cuda")
        ct = torch.empty(w["shots"], dtype=torch.float64, device="cuda")
        q.sample(w["shots"], w["sample_seed"], z_out=zt, cost_out=ct)
        torch.cuda.synchronize()
        assert np.array_equal(zt.cpu().numpy().astype(np.uint64), z_ref)
        assert np.array_equal(ct.cpu().numpy(), c_ref)


def test_sampling_deterministic_state_and_zero_probability():
    # f = sum x_i at gamma = pi/2, beta = pi/4: the state is |1...1> up to phase
    n = 14
    inst = qi.Qubo(n=n, pairs=np.zeros((0, 2), np.int32), J=np.zeros(0), h=np.ones(n))
    with H(inst) as q:
        q.statevector([math.pi / 2], [math.pi / 4], copy=False)
        z, c = q.sample(2000, 9)
    assert np.all(z == (1 << n) - 1) and np.all(c == n)


def test_sampling_chi_square_large():
    import scipy.stats
    n = 22
    inst = mk("reg", n, 8)
    C = oracle.cost_of(inst)
    gamma, beta = qi.ramp_with_noise(2, seed=[8, 8])
    psi = oracle.state(n, C, gamma, beta)
    with H(inst) as q:
        q.statevector(gamma, beta, copy=False)
        z, _ = q.sample(200000, 2024)
    bins = (z >> np.uint64(n - 8)).astype(np.int64)      # top 8 bits
    probs = np.bincount(np.arange(1 << n) >> (n - 8), weights=np.abs(psi) ** 2, minlength=256)
    obs = np.bincount(bins, minlength=256)
    exp = probs * z.size
    keep = exp >= 5
    stat = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert scipy.stats.chi2.sf(stat, keep.sum() - 1) > 1e-3


def test_sampling_complex64_chi_square():
    # complex64 probabilities differ from the fp64 oracle's by ~1e-7 relative, so
    # shots are compared in distribution; objective values are the fp32 diagonal
    import scipy.stats
    n = 18
    inst = mk("er", n, 77)
    C = oracle.cost_of(inst)
    gamma, beta = qi.ramp_with_noise(2, seed=[77, 1])
    psi = oracle.state(n, C, gamma, beta)
    with H(inst, "c64") as q:
        q.statevector(gamma, beta, copy=False)
        z, c = q.sample(200000, 99)
    zi = z.astype(np.int64)
    assert np.array_equal(c, C[zi].astype(np.float32).astype(np.float64))
    bins = zi >> (n - 8)
    probs = np.bincount(np.arange(1 << n) >> (n - 8), weights=np.abs(psi) ** 2, minlength=256)
    obs = np.bincount(bins, minlength=256)
    exp = probs * z.size
    keep = exp >= 5
    stat = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert scipy.stats.chi2.sf(stat, keep.sum() - 1) > 1e-3


def test_sample_errors():
    from paper_2407_13012_amd import QaoaError
    inst = mk("er", 10, 1)
    with H(inst) as q:
        with pytest.raises(QaoaError) as ei:
            q.sample(10, 1)
        assert ei.value.status == 4
        q.statevector([0.1], [0.2], copy=False)
        with pytest.raises(QaoaError):
            q.sample(-1, 1)
        import torch
        t = torch.empty(1, dtype=torch.int64, device="cuda")
        with pytest.raises(QaoaError) as ei:
            q.sample(2**41, 1, z_out=t)  # rejected before anything is written
        assert ei.value.status == 1
        z, c = q.sample(0, 1)
        assert z.size == 0


def test_sample_beyond_one_grid_pass():
    """2^28 + 7 shots: more than one launch of 2^20 workgroups x 256 threads
    covers, so threads take several shots each.  The leading shots equal a
    small call's (same counters), the last ones are the smallest z whose
    cumulative probability in the exported state exceeds the oracle's uniform
    for that shot times the total, and every returned z is a valid index."""
    import torch
    n = 5
    inst = mk("er", n, 77)
    gamma, beta = [0.4, 0.9], [0.7, 0.2]
    shots = (1 << 28) + 7
    with H(inst) as q:
        psi = q.statevector(gamma, beta)
        z_small, _ = q.sample(1000, 11)
        zt = torch.empty(shots, dtype=torch.int64, device="cuda")
        q.sample(shots, 11, z_out=zt)
        torch.cuda.synchronize()
        head = zt[:1000].cpu().numpy().astype(np.uint64)
        tail = zt[-7:].cpu().numpy()
        top = int(zt.max().item())
        del zt
        torch.cuda.empty_cache()
    assert np.array_equal(head, z_small)
    assert top < (1 << n)
    prob = np.abs(psi) ** 2
    S = np.cumsum(prob)
    for k, zk in enumerate(tail):
        u = oracle.uniform53(11, shots - 7 + k)
        # smallest z whose cumulative probability exceeds u * total (the GPU's
        # prefix sums round differently, which matters only within ~1e-16 of a boundary)
        want = int(np.searchsorted(S, u * S[-1], side="right"))
        assert zk == want and prob[zk] > 0, (k, zk, want)


# ---------------------------------------------------------------- complex64

# complex64 tiles hold 2^13 amplitudes: n = 12 is a partial tile, 13 one full
# tile, 14 a 13-qubit pass plus a one-qubit pass, 24 three passes per layer
# (both layer-boundary sweeps at p = 3)
@pytest.mark.parametrize("n,p", [(6, 2), (9, 1), (12, 3), (13, 1), (13, 2), (14, 3), (15, 1), (16, 4), (17, 3),
                                 (18, 2), (19, 3), (21, 4), (22, 1), (23, 2), (24, 3)])
def test_complex64_against_fp64_oracle(n, p):
    inst = mk("er", n, 400 + n)
    C = oracle.cost_of(inst)
    gamma, beta = qi.ramp_with_noise(p, seed=[n, 1])
    E_ref, dg_ref, db_ref = oracle.gradient(n, C, gamma, beta)
    psi_ref = oracle.state(n, C, gamma, beta)
    with H(inst, "c64") as q:
        psi = q.statevector(gamma, beta)
        assert psi.dtype == np.complex64
        assert np.max(np.abs(psi - psi_ref)) < 1e-5
        E_sv = q.expectation()
        E, dg, db = q.gradient(gamma, beta)
    scale = max(abs(E_ref), 1.0)
    gscale = max(np.max(np.abs(np.concatenate([dg_ref, db_ref]))), 1.0)
    assert abs(E - E_ref) / scale <= 1e-4 and abs(E_sv - E_ref) / scale <= 1e-4
    assert np.max(np.abs(dg - dg_ref)) / gscale <= 1e-4
    assert np.max(np.abs(db - db_ref)) / gscale <= 1e-4


# Both factored rotation forms (|cos b| >= |sin b| and the reverse, and
# negative angles) on complex64 tiles whose bit 12 is rotated across lanes, in
# every pairing of forms that the layer-boundary sweeps combine (24 qubits:
# three sweeps per layer).
@pytest.mark.parametrize("n", [13, 20, 24])
def test_complex64_rotation_forms(n):
    inst = mk("qubo", n, 700 + n)
    C = oracle.cost_of(inst)
    gamma = np.array([0.35, -0.2, 0.6, 0.15])
    beta = np.array([0.3, 1.2, -2.0, 0.5])
    E_ref, dg_ref, db_ref = oracle.gradient(n, C, gamma, beta)
    psi_ref = oracle.state(n, C, gamma, beta)
    with H(inst, "c64") as q:
        psi = q.statevector(gamma, beta)
        assert np.max(np.abs(psi - psi_ref)) < 1e-5
        E, dg, db = q.gradient(gamma, beta)
    gscale = max(np.max(np.abs(np.concatenate([dg_ref, db_ref]))), 1.0)
    assert abs(E - E_ref) / max(abs(E_ref), 1.0) <= 1e-4
    assert np.max(np.abs(dg - dg_ref)) / gscale <= 1e-4
    assert np.max(np.abs(db - db_ref)) / gscale <= 1e-4


# ---------------------------------------------------------------- named workloads

def test_workload_small_full_parity():
    """Unweighted MaxCut on ER(12, 0.5) seed 0, p = 2: cost diagonal, E, the
    4-angle gradient and 1024 samples against the oracle."""
    w = qi.workload_small()
    g = w["instance"]
    C = oracle.cost_of(g)
    E_ref, dg_ref, db_ref = oracle.gradient(g.n, C, w["gamma"], w["beta"])
    psi = oracle.state(g.n, C, w["gamma"], w["beta"])
    z_ref, c_ref = oracle.sample(g.n, psi, C, w["shots"], w["sample_seed"])
    with H(g) as q:
        assert np.array_equal(q.cost_diagonal(), C)
        E, dg, db = q.gradient(w["gamma"], w["beta"])
        q.statevector(w["gamma"], w["beta"], copy=False)
        z, c = q.sample(w["shots"], w["sample_seed"])
    assert abs(E - E_ref) <= tol_E(g)
    assert np.max(np.abs(dg - dg_ref)) <= 1e-8 and np.max(np.abs(db - db_ref)) <= 1e-8
    assert np.array_equal(z, z_ref) and np.array_equal(c, c_ref)


def test_workload_regular26_full_parity():
    """Weighted 3-regular MaxCut, n = 26, p = 6, ramp + noise: E and all 12
    gradient entries against the oracle, in complex128 and complex64."""
    w = qi.workload_regular26()
    g = w["instance"]
    C = oracle.cost_of(g)
    E_ref, dg_ref, db_ref = oracle.gradient(g.n, C, w["gamma"], w["beta"])
    with H(g) as q:
        assert np.array_equal(q.cost_diagonal(), C)
        E, dg, db = q.gradient(w["gamma"], w["beta"])
    assert abs(E - E_ref) <= tol_E(g)
    assert np.max(np.abs(dg - dg_ref)) <= 1e-8 and np.max(np.abs(db - db_ref)) <= 1e-8
    with H(g, "c64") as q:
        E32, dg32, db32 = q.gradient(w["gamma"], w["beta"])
    gscale = max(np.max(np.abs(np.concatenate([dg_ref, db_ref]))), 1.0)
    assert abs(E32 - E_ref) / max(abs(E_ref), 1) <= 1e-4
    assert np.max(np.abs(np.concatenate([dg32 - dg_ref, db32 - db_ref]))) / gscale <= 1e-4


# Phase arguments |gamma C| far beyond the fast reduction's range (weights of a
# few 1e6): such passes leave the spectator-class kernels, whose phases assume
# |gamma C| < 1e6 (complex128) or |g1 C| < 4096 (complex64), for the kernels
# with the full-range fallback.  complex64 is compared with the oracle run on
# the fp32-rounded cost diagonal (the rounding of C alone moves phases of 1e7
# radians by about 1 radian).
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_phase_arguments_beyond_fast_range(prec):
    n, p = 14, 2
    inst = qi.erdos_renyi(n, 0.5, seed=[5, 14], weights="uniform", wlow=1.0e6, whigh=3.0e6)
    C = oracle.cost_of(inst)
    if prec == "c64":
        C = C.astype(np.float32).astype(np.float64)
    gamma = np.array([0.31, -0.47])
    beta = np.array([0.6, 0.25])
    assert np.abs(gamma).max() * np.abs(C).max() > 1e7
    psi_ref = oracle.state(n, C, gamma, beta)
    E_ref, dg_ref, db_ref = oracle.gradient(n, C, gamma, beta)
    with H(inst, prec) as q:
        psi = q.statevector(gamma, beta)
        E, dg, db = q.gradient(gamma, beta)
    gscale = np.abs(np.concatenate([dg_ref, db_ref])).max()
    if prec == "c128":
        assert np.max(np.abs(psi - psi_ref)) < 1e-12
        assert abs(E - E_ref) <= 1e-10 * np.abs(C).max()
        assert np.abs(np.concatenate([dg - dg_ref, db - db_ref])).max() <= 1e-9 * gscale
    else:
        assert np.max(np.abs(psi - psi_ref)) < 1e-5
        assert abs(E - E_ref) <= 1e-4 * np.abs(C).max()
        assert np.abs(np.concatenate([dg - dg_ref, db - db_ref])).max() <= 1e-4 * gscale
