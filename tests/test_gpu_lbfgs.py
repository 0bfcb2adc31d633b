"""L-BFGS on the GPU gradient.  The optimiser's trajectory has no oracle of its
own (parity unpinned along the path); instead the oracle's E and gradient are
evaluated at the GPU's own iterates."""
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


def test_lbfgs_iterates_match_oracle_small():
    inst = qi.random_regular(16, 3, 3, weights="uniform")
    C = oracle.cost_of(inst)
    g0, b0 = qi.ramp_with_noise(3, seed=[3, 1])
    with H(inst) as q:
        g, b, E, it, ev, tx, tE = q.optimize(g0, b0, max_iter=60, gtol=1e-9, trace=True)
        assert it >= 5 and ev >= it
        assert np.all(np.diff(tE) >= -1e-12)          # maximisation: E never decreases
        for k in range(0, it + 1, 10):
            gk, bk = tx[k, :3], tx[k, 3:]
            E_ref, dg_ref, db_ref = oracle.gradient(inst.n, C, gk, bk)
            Eg, dg, db = q.gradient(gk, bk)
            assert abs(tE[k] - E_ref) < 1e-10 * inst.m and abs(Eg - E_ref) < 1e-10 * inst.m
            assert np.max(np.abs(dg - dg_ref)) < 1e-8 and np.max(np.abs(db - db_ref)) < 1e-8
        # the optimum: gradient small, E above the ramp start
        E_end, dg, db = q.gradient(g, b)
        assert E_end == pytest.approx(E, abs=1e-12)
        assert max(np.abs(dg).max(), np.abs(db).max()) < 1e-5
        assert E > tE[0]


def test_lbfgs_regular26_c128_and_c64():
    """3-regular MaxCut n=26, w ~ U[0,1], p=6, 200 L-BFGS iterations from the noisy
    ramp in complex128 and complex64; oracle E and gradient at the start and at
    each precision's final iterate."""
    w = qi.workload_regular26()
    g_inst = w["instance"]
    C = oracle.cost_of(g_inst)
    out = {}
    for prec in ["c128", "c64"]:
        with H(g_inst, prec) as q:
            g, b, E, it, ev, tx, tE = q.optimize(w["gamma"], w["beta"], max_iter=200, gtol=1e-7,
                                                 max_evals=400, trace=True)
            _, dg, db = q.gradient(g, b)
        out[prec] = (g, b, E, it, ev, tE, dg, db)
        print(f"{prec}: iterations {it}, evaluations {ev}, E {tE[0]:.9f} -> {E:.9f}", flush=True)
    E0_ref = oracle.gradient(g_inst.n, C, w["gamma"], w["beta"])[0]
    assert abs(out["c128"][5][0] - E0_ref) < 1e-10 * g_inst.m
    assert abs(out["c64"][5][0] - E0_ref) / abs(E0_ref) < 1e-4
    for prec, tol in [("c128", None), ("c64", 1e-4)]:
        g, b, E, it, ev, tE, dg, db = out[prec]
        E_ref, dg_ref, db_ref = oracle.gradient(g_inst.n, C, g, b)
        gscale = max(1.0, np.abs(np.concatenate([dg_ref, db_ref])).max())
        if tol is None:
            assert abs(E - E_ref) < 1e-10 * g_inst.m
            assert np.max(np.abs(np.concatenate([dg - dg_ref, db - db_ref]))) < 1e-8
        else:
            assert abs(E - E_ref) / abs(E_ref) < tol
            assert np.max(np.abs(np.concatenate([dg - dg_ref, db - db_ref]))) / gscale < tol
        assert E > tE[0] + 0.1
    # both precisions reach the same local optimum (approximation ratio within 1e-4)
    cmax = C.max()
    assert abs(out["c128"][2] - out["c64"][2]) / cmax < 1e-4
