import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.load()
    return oracle


@pytest.fixture(scope="session")
def qubo28_reference():
    """Oracle E, gradient and state of the n = 28 member of the headline QUBO
    family (p = 3, the benchmark's angles); shared by the modules that compare
    against it, since the stored-state oracle needs ~30 GiB and tens of
    seconds at this size."""
    import numpy as np

    import oracle
    import qaoa_inputs as qi
    w = qi.workload_qubo32(28)
    inst = w["instance"]
    C = oracle.cost_of(inst)
    E, dg, db = oracle.gradient(inst.n, C, w["gamma"], w["beta"])
    scale = float(np.abs(inst.J).sum() + np.abs(inst.h).sum())
    return {"inst": inst, "gamma": w["gamma"], "beta": w["beta"], "C": C, "E": E, "dg": dg, "db": db,
            "scale": scale}
