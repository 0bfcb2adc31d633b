"""Parity at the full n = 32 size (64 GiB complex128 state) in the launch
configuration the benchmark times.

A full-state CPU evaluation at n = 32 is out of reach, so the checks use
facts that hold at any size:
  * a QUBO whose couplings stay inside disjoint blocks has a QAOA state that is
    a tensor product over blocks, so E and every partial derivative are sums of
    the per-block oracle values, and each block's marginal distribution is the
    block state's |psi|^2;
  * cost-diagonal entries are compared one by one with the oracle's per-entry
    evaluation;
  * results are bitwise reproducible and E lies in [C_min, C_max].
"""
import numpy as np
import pytest

import oracle
import qaoa_inputs as qi

pytestmark = pytest.mark.gpu

N = 32


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    free, _ = torch.cuda.mem_get_info()
    if free < 170 * 2**30:
        pytest.skip("needs ~160 GiB of free device memory")


def H(inst, prec="c128"):
    from paper_2407_13012_amd import QaoaHandle
    return QaoaHandle.from_instance(inst, prec)


def block_reference(inst, block, gamma, beta):
    """E, dE/dgamma, dE/dbeta and block states from the oracle, block by block."""
    E, dg, db, states = 0.0, np.zeros(len(gamma)), np.zeros(len(gamma)), []
    for b0 in range(0, inst.n, block):
        b1 = min(inst.n, b0 + block)
        sel = (inst.pairs[:, 0] >= b0) & (inst.pairs[:, 1] < b1)
        pairs = inst.pairs[sel] - b0
        C = oracle.cost_qubo(b1 - b0, pairs, inst.J[sel], inst.h[b0:b1])
        e, g, d = oracle.gradient(b1 - b0, C, gamma, beta)
        E += e
        dg += g
        db += d
        states.append(oracle.state(b1 - b0, C, gamma, beta))
    return E, dg, db, states


@pytest.fixture(scope="module")
def block_case():
    inst = qi.qubo_blocks(N, 8, 0.5, seed=21)
    gamma, beta = qi.ramp_with_noise(3, seed=[2, 1])
    return inst, gamma, beta, block_reference(inst, 8, gamma, beta)


def test_block_qubo_expectation_and_gradient_n32(block_case):
    inst, gamma, beta, (E_ref, dg_ref, db_ref, _) = block_case
    tol = 1e-10 * (np.abs(inst.J).sum() + np.abs(inst.h).sum())
    with H(inst) as q:
        E, dg, db = q.gradient(gamma, beta)
        E2, dg2, db2 = q.gradient(gamma, beta)
        E_ev = q.evaluate(gamma, beta)
        E_sv = q.expectation()
    print(f"n=32 block QUBO: E={E!r} ref={E_ref!r} |ddg|={np.abs(dg - dg_ref).max():.2e} "
          f"|ddb|={np.abs(db - db_ref).max():.2e}", flush=True)
    assert abs(E - E_ref) <= tol
    assert np.max(np.abs(dg - dg_ref)) <= 1e-8
    assert np.max(np.abs(db - db_ref)) <= 1e-8
    assert E == E2 and np.array_equal(dg, dg2) and np.array_equal(db, db2)
    assert abs(E_ev - E_ref) <= tol and abs(E_sv - E_ref) <= tol


def test_block_qubo_sampling_marginals_n32(block_case):
    import scipy.stats
    inst, gamma, beta, (_, _, _, states) = block_case
    with H(inst) as q:
        q.statevector(gamma, beta, copy=False)
        z, c = q.sample(10**6, 2)
        zr, _ = q.sample(1000, 2)
        assert np.array_equal(zr, z[:1000])          # same seed -> same leading shots
    for b, psi_b in enumerate(states):
        obs = np.bincount(((z >> np.uint64(8 * b)) & np.uint64(255)).astype(np.int64), minlength=256)
        exp = np.abs(psi_b) ** 2 * z.size
        keep = exp >= 5
        stat = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
        pval = scipy.stats.chi2.sf(stat, keep.sum() - 1)
        assert pval > 1e-4, (b, pval)
    # returned objective values are the diagonal at the returned states
    for k in range(0, 10**6, 99991):
        assert c[k] == oracle.cost_entry_of(inst, int(z[k]))


def test_block_qubo_complex64_n32(block_case):
    inst, gamma, beta, (E_ref, dg_ref, db_ref, _) = block_case
    with H(inst, "c64") as q:
        E, dg, db = q.gradient(gamma, beta)
        E2, dg2, db2 = q.gradient(gamma, beta)
    assert E == E2 and np.array_equal(dg, dg2) and np.array_equal(db, db2)  # fixed-order sums
    gscale = max(np.abs(np.concatenate([dg_ref, db_ref])).max(), 1.0)
    assert abs(E - E_ref) / max(abs(E_ref), 1.0) <= 1e-4
    assert np.abs(np.concatenate([dg - dg_ref, db - db_ref])).max() / gscale <= 1e-4


def test_headline_qubo_cost_entries_and_bounds_n32():
    """The benchmark instance itself: sampled diagonal entries bit-exact, C_min
    and C_max at their argmin/argmax, E inside [C_min, C_max], reproducible."""
    import torch
    w = qi.workload_qubo32(N)
    inst, gamma, beta = w["instance"], w["gamma"], w["beta"]
    with H(inst) as q:
        Cd = torch.empty(1 << N, dtype=torch.float64, device="cuda")
        q.cost_diagonal(Cd)
        torch.cuda.synchronize()
        rng = np.random.default_rng(0)
        zs = np.concatenate([[0, 1, (1 << N) - 1, 1 << 31], rng.integers(0, 1 << N, 2000, dtype=np.int64)])
        got = Cd[torch.from_numpy(zs).cuda()].cpu().numpy()
        want = np.array([oracle.cost_entry_of(inst, int(z)) for z in zs])
        assert np.array_equal(got, want)
        lo, hi = q.cost_extrema()
        amin, amax = int(torch.argmin(Cd)), int(torch.argmax(Cd))
        assert oracle.cost_entry_of(inst, amin) == lo and oracle.cost_entry_of(inst, amax) == hi
        del Cd
        torch.cuda.empty_cache()
        E, dg, db = q.gradient(gamma, beta)
        E2, dg2, db2 = q.gradient(gamma, beta)
        assert E == E2 and np.array_equal(dg, dg2) and np.array_equal(db, db2)
        assert lo <= E <= hi
        assert np.all(np.isfinite(dg)) and np.all(np.isfinite(db))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_block_qubo_mixed_rotation_forms_n32(prec):
    """Mixer angles on both sides of pi/4 (the rotations' tan and cot forms)
    in the n = 32 sweeps, whose plain forward sweeps take two tiles per
    workgroup; E and the gradient against the block-wise oracle."""
    inst = qi.qubo_blocks(N, 8, 0.5, seed=22)
    gamma = np.array([0.35, 0.6, 0.8])
    beta = np.array([1.1, 0.45, 1.3])
    E_ref, dg_ref, db_ref, _ = block_reference(inst, 8, gamma, beta)
    with H(inst, prec) as q:
        E, dg, db = q.gradient(gamma, beta)
        E_ev = q.evaluate(gamma, beta)
    wsum = np.abs(inst.J).sum() + np.abs(inst.h).sum()
    if prec == "c128":
        tol = 1e-10 * wsum
        assert abs(E - E_ref) <= tol and abs(E_ev - E_ref) <= tol
        assert np.max(np.abs(dg - dg_ref)) <= 1e-8 and np.max(np.abs(db - db_ref)) <= 1e-8
    else:
        gscale = max(np.abs(np.concatenate([dg_ref, db_ref])).max(), 1.0)
        assert abs(E - E_ref) / max(abs(E_ref), 1.0) <= 1e-4
        assert abs(E_ev - E_ref) / max(abs(E_ref), 1.0) <= 1e-4
        assert np.abs(np.concatenate([dg - dg_ref, db - db_ref])).max() / gscale <= 1e-4
