"""qaoa_gradient_noalloc (the expectation and adjoint gradient through the
library's fixed device scratch, no allocation) against qaoa_gradient and the
oracle: two calls in a row, the second on a smaller instance, with host and
with device outputs, plus p = 0 and the size limits."""
import ctypes

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


def _handle(inst, prec):
    from paper_2407_13012_amd import QaoaHandle
    return QaoaHandle.from_instance(inst, prec)


def _check_against(inst, prec, gamma, beta):
    """noalloc (host outputs, then device outputs) vs qaoa_gradient vs the oracle."""
    import torch
    C = oracle.cost_of(inst)
    E_ref, dg_ref, db_ref = oracle.gradient(inst.n, C, gamma, beta)
    wsum = float(np.abs(inst.weight_array()).sum()) + (float(np.abs(inst.h).sum()) if hasattr(inst, "h") and inst.h is not None else 0.0)
    p = len(gamma)
    with _handle(inst, prec) as q:
        E0, dg0, db0 = q.gradient(gamma, beta)
        E1, dg1, db1 = q.gradient_noalloc(gamma, beta)
        out = torch.full((2 * p + 1,), float("nan"), dtype=torch.float64, device="cuda")
        q.gradient_noalloc(gamma, beta, out=out)
        torch.cuda.synchronize()
        dev = out.cpu().numpy()
    # the same kernels in the same order as qaoa_gradient: identical results
    assert E1 == E0 and np.array_equal(dg1, dg0) and np.array_equal(db1, db0)
    assert dev[0] == E0 and np.array_equal(dev[1:1 + p], dg0) and np.array_equal(dev[1 + p:], db0)
    if prec == "c128":
        assert abs(E1 - E_ref) <= 1e-10 * max(wsum, 1.0)
        assert np.max(np.abs(np.concatenate([dg1 - dg_ref, db1 - db_ref]))) <= 1e-8
    else:
        gs = max(float(np.abs(np.concatenate([dg_ref, db_ref])).max()), 1.0)
        assert abs(E1 - E_ref) <= 1e-4 * max(abs(E_ref), 1.0)
        assert np.max(np.abs(np.concatenate([dg1 - dg_ref, db1 - db_ref]))) <= 1e-4 * gs
    print(f"noalloc {prec} n={inst.n} p={p}: E {E1:.12f} (oracle {E_ref:.12f})", flush=True)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_matches_gradient_two_calls(prec):
    n1 = 20 if prec == "c128" else 21
    big = qi.erdos_renyi(n1, 0.2, seed=31, weights="uniform", wlow=-1.0, whigh=1.0)
    g1, b1 = qi.ramp_with_noise(3, seed=[31, 1])
    small = qi.erdos_renyi(13, 0.5, seed=32, weights="uniform", wlow=0.0, whigh=1.0)
    g2, b2 = qi.ramp_with_noise(2, seed=[32, 1])
    _check_against(big, prec, g1, b1)     # the largest size the scratch holds
    _check_against(small, prec, g2, b2)   # then a smaller one: stale scratch contents must not matter


def test_noalloc_single_sweep_and_p0():
    inst = qi.erdos_renyi(9, 0.5, seed=33, weights="uniform", wlow=-1.0, whigh=1.0)
    g, b = qi.ramp_with_noise(4, seed=[33, 1])
    _check_against(inst, "c128", g, b)    # n <= 12: one sweep per layer
    C = oracle.cost_of(inst)
    with _handle(inst, "c128") as q:
        E, dg, db = q.gradient_noalloc([], [])
    assert dg.size == 0 and db.size == 0
    assert abs(E - float(np.mean(C))) <= 1e-12 * max(1.0, float(np.abs(C).max()))


def test_noalloc_rejects_sizes_beyond_scratch():
    from paper_2407_13012_amd._binding import QaoaError
    too_big = qi.erdos_renyi(21, 0.05, seed=34, weights="uniform", wlow=0.0, whigh=1.0)
    g, b = qi.ramp_with_noise(1, seed=[34, 1])
    with _handle(too_big, "c128") as q:
        with pytest.raises(QaoaError) as ei:
            q.gradient_noalloc(g, b)
        assert ei.value.status == 1 and "scratch" in ei.value.message
        # the handle is still usable afterwards
        E, _, _ = q.gradient(g, b)
        assert np.isfinite(E)
    small = qi.erdos_renyi(8, 0.5, seed=35, weights="uniform", wlow=0.0, whigh=1.0)
    with _handle(small, "c128") as q:
        with pytest.raises(QaoaError) as ei:
            q.gradient_noalloc(np.zeros(33), np.zeros(33))
        assert ei.value.status == 1
