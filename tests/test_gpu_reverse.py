"""The reverse sweep from a stored final state (qaoa_gradient_from_state)
against qaoa_gradient and the oracle gradient, its state checks, and the
autograd wrapper built on it (forward = qaoa_evaluate, backward = reverse
sweep)."""
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


def H(inst, prec="c128"):
    from paper_2407_13012_amd import QaoaHandle
    return QaoaHandle.from_instance(inst, prec)


# n <= 12: one sweep per layer (the first reverse pass also undoes the phase);
# n = 16, 22, 26: two or three sweeps per layer with layer-boundary sweeps
CASES = [(8, 1), (12, 3), (16, 1), (16, 4), (22, 3), (26, 2)]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,p", CASES)
def test_reverse_sweep_matches_gradient_and_oracle(n, p, prec):
    inst = qi.erdos_renyi(n, 0.3 if n < 20 else 0.12, seed=400 + n, weights="uniform", wlow=-1.0, whigh=1.0)
    g, b = qi.ramp_with_noise(p, seed=[400 + n, p])
    C = oracle.cost_of(inst)
    E_ref, dg_ref, db_ref = oracle.gradient(n, C, g, b)
    ref = np.concatenate([dg_ref, db_ref])
    with H(inst, prec) as q:
        E0, dg0, db0 = q.gradient(g, b)
        E1 = q.evaluate(g, b)
        dg1, db1 = q.gradient_from_state(g, b)
    got = np.concatenate([dg1, db1])
    full = np.concatenate([dg0, db0])
    if prec == "c128":
        assert abs(E1 - E_ref) <= 1e-10 * max(1.0, float(np.abs(inst.weight_array()).sum()))
        assert np.max(np.abs(got - ref)) <= 1e-8
        assert np.max(np.abs(got - full)) <= 1e-10
    else:
        scale = max(float(np.abs(ref).max()), 1e-3)
        assert np.max(np.abs(got - ref)) <= 1e-4 * scale
        assert np.max(np.abs(got - full)) <= 1e-4 * scale
    print(f"reverse {prec} n={n} p={p}: max |dgrad| vs oracle {np.max(np.abs(got - ref)):.2e}, "
          f"vs qaoa_gradient {np.max(np.abs(got - full)):.2e}", flush=True)


def test_reverse_sweep_needs_the_state_of_the_same_angles():
    from paper_2407_13012_amd._binding import QaoaError
    inst = qi.erdos_renyi(14, 0.4, seed=410, weights="unit")
    g, b = qi.ramp_with_noise(2, seed=[410, 1])
    with H(inst) as q:
        with pytest.raises(QaoaError) as ei:
            q.gradient_from_state(g, b)             # no state yet
        assert ei.value.status == 4
        q.evaluate(g, b)
        with pytest.raises(QaoaError) as ei:
            q.gradient_from_state(g + 1e-3, b)      # state of other angles
        assert ei.value.status == 4
        dg, db = q.gradient_from_state(g, b)
        with pytest.raises(QaoaError) as ei:
            q.gradient_from_state(g, b)             # consumed
        assert ei.value.status == 4
        q.statevector(g, b, copy=False)             # qaoa_statevector also leaves a usable state
        dg2, db2 = q.gradient_from_state(g, b)
    assert np.array_equal(dg, dg2) and np.array_equal(db, db2)


def test_autograd_backward_after_the_state_was_replaced():
    import torch
    from paper_2407_13012_amd.autograd import qaoa_expectation_fn
    inst = qi.erdos_renyi(15, 0.4, seed=420, weights="uniform", wlow=0.0, whigh=1.0)
    g, b = qi.ramp_with_noise(3, seed=[420, 1])
    C = oracle.cost_of(inst)
    _, dg_ref, db_ref = oracle.gradient(inst.n, C, g, b)
    with H(inst) as q:
        gt = torch.tensor(g, requires_grad=True)
        bt = torch.tensor(b, requires_grad=True)
        E1 = qaoa_expectation_fn(gt, bt, q)
        # another evaluation on the same handle replaces the stored state
        with torch.no_grad():
            qaoa_expectation_fn(torch.tensor(g + 0.1), torch.tensor(b), q)
        E1.backward()
    assert np.max(np.abs(gt.grad.numpy() - dg_ref)) <= 1e-8
    assert np.max(np.abs(bt.grad.numpy() - db_ref)) <= 1e-8
