"""Handles whose buffers come from torch's caching allocator (qaoa_set_allocator)."""
import numpy as np
import pytest

import qaoa_inputs as qi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def test_torch_allocator_holds_buffers_and_results_match():
    import torch
    from paper_2407_13012_amd import QaoaHandle, use_torch_allocator
    w = qi.workload_regular26()
    inst = qi.random_regular(20, 3, seed=4, weights="uniform")
    g, b = w["gamma"][:3], w["beta"][:3]
    with QaoaHandle.from_instance(inst) as ref:
        E0, dg0, db0 = ref.gradient(g, b)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    nalloc0 = torch.cuda.memory_stats()["allocation.all.allocated"]
    with use_torch_allocator():
        h = QaoaHandle.from_instance(inst)
    during = torch.cuda.memory_allocated()
    assert during - before >= (1 << 20) * 24  # state + cost diagonal of n = 20
    # state, cost diagonal, partials, results, and the term list uploaded to
    # build the diagonal: all through the allocator
    assert torch.cuda.memory_stats()["allocation.all.allocated"] - nalloc0 >= 5
    E1, dg1, db1 = h.gradient(g, b)
    assert torch.cuda.memory_allocated() - before >= (1 << 20) * 40  # plus the adjoint vector
    h.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    assert E1 == E0
    np.testing.assert_array_equal(dg1, dg0)
    np.testing.assert_array_equal(db1, db0)
    # handles created after the context use hipMalloc again
    with QaoaHandle.from_instance(inst) as h2:
        assert torch.cuda.memory_allocated() == before
        assert h2.gradient(g, b)[0] == E0
