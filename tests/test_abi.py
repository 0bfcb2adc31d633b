"""CPU-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qaoa.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(qaoa_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_13012_amd import load_library
    try:
        return load_library()
    except ImportError as e:
        pytest.fail(str(e))


def test_header_declares_expected_calls():
    names = declared_functions()
    for want in ["qaoa_create_maxcut", "qaoa_create_qubo", "qaoa_destroy", "qaoa_cost_diagonal",
                 "qaoa_statevector", "qaoa_expectation", "qaoa_gradient", "qaoa_sample",
                 "qaoa_status_string", "qaoa_last_error_message", "qaoa_evaluate",
                 "qaoa_cost_extrema", "qaoa_get_info"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2407_13012_amd import library_path
    out = subprocess.run(["nm", "-D", "--defined-only", library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        getattr(lib, f)


def test_library_is_gfx950_code_object():
    from paper_2407_13012_amd import library_path
    data = open(library_path(), "rb").read()
    assert b"gfx950" in data


def test_status_strings(lib):
    lib.qaoa_status_string.restype = ctypes.c_char_p
    assert lib.qaoa_status_string(0) == b"success"
    assert lib.qaoa_status_string(1) == b"invalid argument"
    assert lib.qaoa_status_string(99) == b"unknown status"


def _create_maxcut(lib, n, edges, w=None, prec=0, out=True):
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    h = ctypes.c_void_p()
    wp = None if w is None else np.ascontiguousarray(w, dtype=np.float64).ctypes.data
    return lib.qaoa_create_maxcut(n, e.shape[0], e.ctypes.data if e.size else None, wp, prec, None,
                                  ctypes.byref(h) if out else None)


@pytest.mark.parametrize("n,edges,w,prec", [
    (0, [[0, 1]], None, 0),              # n too small
    (41, [[0, 1]], None, 0),             # n too large
    (4, [[0, 4]], None, 0),              # index out of range
    (4, [[-1, 2]], None, 0),             # negative index
    (4, [[2, 2]], None, 0),              # self-loop
    (4, [[0, 1]], [float("nan")], 0),    # non-finite weight
    (4, [[0, 1]], [float("inf")], 0),
    (4, [[0, 1]], None, 7),              # unknown precision
])
def test_create_maxcut_rejects(lib, n, edges, w, prec):
    assert _create_maxcut(lib, n, edges, w, prec) == 1
    lib.qaoa_last_error_message.restype = ctypes.c_char_p
    assert lib.qaoa_last_error_message() != b""


def test_create_rejects_null_out_and_negative_m(lib):
    assert _create_maxcut(lib, 3, [[0, 1]], out=False) == 1
    h = ctypes.c_void_p()
    assert lib.qaoa_create_maxcut(3, -1, None, None, 0, None, ctypes.byref(h)) == 1
    assert lib.qaoa_create_maxcut(3, 2, None, None, 0, None, ctypes.byref(h)) == 1


def test_create_qubo_rejects(lib):
    h = ctypes.c_void_p()
    pr = np.array([[0, 1]], dtype=np.int32)
    J = np.array([1.0])
    hb = np.array([0.0, np.nan, 0.0])
    # J missing for m > 0
    assert lib.qaoa_create_qubo(3, 1, pr.ctypes.data, None, None, ctypes.c_double(0.0), 0, None,
                                ctypes.byref(h)) == 1
    # non-finite h
    assert lib.qaoa_create_qubo(3, 1, pr.ctypes.data, J.ctypes.data, hb.ctypes.data,
                                ctypes.c_double(0.0), 0, None, ctypes.byref(h)) == 1
    # non-finite offset
    assert lib.qaoa_create_qubo(3, 1, pr.ctypes.data, J.ctypes.data, None,
                                ctypes.c_double(float("nan")), 0, None, ctypes.byref(h)) == 1


def test_calls_reject_null_handle(lib):
    d = ctypes.c_double()
    g = np.zeros(1)
    assert lib.qaoa_destroy(None) == 0
    assert lib.qaoa_expectation(None, ctypes.byref(d)) == 1
    assert lib.qaoa_cost_diagonal(None, g.ctypes.data, 0) == 1
    assert lib.qaoa_cost_extrema(None, ctypes.byref(d), ctypes.byref(d)) == 1
    assert lib.qaoa_statevector(None, 1, g.ctypes.data, g.ctypes.data, None, 0) == 1
    assert lib.qaoa_evaluate(None, 1, g.ctypes.data, g.ctypes.data, ctypes.byref(d)) == 1
    assert lib.qaoa_gradient(None, 1, g.ctypes.data, g.ctypes.data, None, g.ctypes.data,
                             g.ctypes.data) == 1
    assert lib.qaoa_sample(None, 10, 0, g.ctypes.data, None, 0) == 1
    assert lib.qaoa_get_info(None, None, None) == 1


def test_valid_create_without_gpu_reports_device_error(lib):
    """In a container without a GPU a valid request passes validation and then
    fails at the first HIP call with QAOA_ERR_DEVICE (never a crash)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _create_maxcut(lib, 4, [[0, 1], [1, 2]]) == 3


def test_python_binding_has_c_names():
    import paper_2407_13012_amd as pkg
    for f in declared_functions():
        assert hasattr(pkg, f), f


# ---------------------------------------------------------------- pass planning (host logic)

@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_pass_plan_invariants(prec):
    from paper_2407_13012_amd import qaoa_pass_plan
    page = 17 if prec == "c128" else 18
    tb = 12 if prec == "c128" else 13  # 64 KiB tiles: 2^12 x 16 B or 2^13 x 8 B
    for n in range(1, 41):
        plan = qaoa_pass_plan(n, prec)
        seen = 0
        for i, (tile, tgt) in enumerate(plan):
            assert bin(tile).count("1") == min(n, tb)
            assert tgt & ~tile == 0 and tgt & seen == 0
            assert tile < (1 << n)
            seen |= tgt
            spect = tile & ~tgt
            # spectators are the lowest bits, contiguous from bit 0
            assert spect & (spect + 1) == 0
            # the first pass starts with >= 6 consecutive low target bits (>= 64 amplitudes)
            if i == 0:
                assert tgt & 63 == min(63, (1 << n) - 1)
            elif n > tb:
                # at least 2 spectator bits (>= 4 consecutive amplitudes, 64 B at complex128),
                # at least 3 at complex64 (again >= 64 B)
                assert spect >= (3 if prec == "c128" else 7)
        assert seen == (1 << n) - 1
        # at most 10 targets per later pass at either precision
        assert len(plan) == (1 if n <= tb else 1 + -(-(n - tb) // 10))
        # page-crossing qubits are spread evenly
        X = max(0, n - page)
        if X:
            per = [bin(t >> page).count("1") for _, t in plan]
            assert max(per) - min(per) <= 1, (n, per)


def test_pass_plan_n32_geometry():
    from paper_2407_13012_amd import qaoa_pass_plan
    plan = qaoa_pass_plan(32, "c128")
    assert len(plan) == 3
    assert [bin(t >> 17).count("1") for _, t in plan] == [5, 5, 5]
    assert plan[0][1] & 127 == 127          # 7 consecutive low qubits in the first pass


def test_pass_plan_n32_complex64_geometry():
    # 2^13-amplitude tiles: three sweeps per layer, as at complex128, with runs
    # of >= 8 amplitudes (64 B) in the later sweeps
    from paper_2407_13012_amd import qaoa_pass_plan
    plan = qaoa_pass_plan(32, "c64")
    assert len(plan) == 3
    assert [bin(t).count("1") for t, _ in plan] == [13, 13, 13]
    assert [bin(g).count("1") for _, g in plan] == [13, 10, 9]
    assert min(bin(tile & ~tgt).count("1") for tile, tgt in plan[1:]) == 3
    assert sorted(bin(t >> 18).count("1") for _, t in plan) == [4, 5, 5]


def test_pass_plan_rejects():
    from paper_2407_13012_amd import QaoaError, qaoa_pass_plan
    with pytest.raises(QaoaError):
        qaoa_pass_plan(0)
    with pytest.raises(QaoaError):
        qaoa_pass_plan(41)


# ---------------------------------------------------------------- batched engine (validation only)

def _batch_create(lib, n, off, edges, w=None, p=2, opt=None, out=True):
    import paper_2407_13012_amd as pkg
    nn = np.ascontiguousarray(n, dtype=np.int32)
    oo = np.ascontiguousarray(off, dtype=np.int64)
    ee = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    h = ctypes.c_void_p()
    return lib.qaoa_batch_create(len(nn), nn.ctypes.data if nn.size else None, oo.ctypes.data,
                                 ee.ctypes.data if ee.size else None,
                                 None if ww is None else ww.ctypes.data, p,
                                 ctypes.byref(opt) if opt is not None else None,
                                 ctypes.byref(h) if out else None)


@pytest.mark.parametrize("case", [
    dict(n=[], off=[0], edges=[]),                                  # empty batch
    dict(n=[4], off=[0, 1], edges=[[0, 1]], p=0),                   # p too small
    dict(n=[4], off=[0, 1], edges=[[0, 1]], p=17),                  # p too large
    dict(n=[1], off=[0, 0], edges=[]),                              # n too small
    dict(n=[25], off=[0, 1], edges=[[0, 1]]),                       # n too large
    dict(n=[4], off=[1, 1], edges=[[0, 1]]),                        # offsets must start at 0
    dict(n=[4, 4], off=[0, 2, 1], edges=[[0, 1], [1, 2]]),          # decreasing offsets
    dict(n=[4], off=[0, 1], edges=[[0, 4]]),                        # vertex out of range
    dict(n=[4], off=[0, 1], edges=[[2, 2]]),                        # self-loop
    dict(n=[4], off=[0, 1], edges=[[0, 1]], w=[float("nan")]),      # non-finite weight
    dict(n=[4], off=[0, 1], edges=[[0, 1]], out=False),             # NULL out
])
def test_batch_create_rejects(lib, case):
    assert _batch_create(lib, **case) == 1
    lib.qaoa_last_error_message.restype = ctypes.c_char_p
    assert lib.qaoa_last_error_message() != b""


@pytest.mark.parametrize("field,value", [("steps", -1), ("lr", 0.0), ("beta1", 1.0), ("beta2", -0.1),
                                         ("eps", 0.0), ("workgroups", -2), ("max_group", 0),
                                         ("max_group", 11), ("waves_per_simd", 3),
                                         ("waves_per_simd", -1), ("resident_max_n", -1),
                                         ("resident_max_n", 13)])
def test_batch_create_rejects_options(lib, field, value):
    from paper_2407_13012_amd import batch_options
    opt = batch_options()
    setattr(opt, field, value)
    assert _batch_create(lib, [4], [0, 1], [[0, 1]], opt=opt) == 1
    opt = batch_options(group_by_n={5: 11})
    assert _batch_create(lib, [4], [0, 1], [[0, 1]], opt=opt) == 1


def test_batch_run_rejects(lib):
    g = np.zeros(2)
    assert lib.qaoa_batch_run(None, g.ctypes.data, g.ctypes.data, None, None, None, None) == 1
    assert lib.qaoa_batch_timeline(None, None, None, None) == 1
    assert lib.qaoa_batch_destroy(None) == 0


def test_batch_valid_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _batch_create(lib, [4, 6], [0, 1, 3], [[0, 1], [0, 5], [2, 3]]) == 3


# ---------------------------------------------------------------- warm-start network (validation only)

def test_mpnn_rejects(lib):
    c = ctypes.c_int64()
    assert lib.qaoa_mpnn_num_params(0, ctypes.byref(c)) == 1
    assert lib.qaoa_mpnn_num_params(17, ctypes.byref(c)) == 1
    assert lib.qaoa_mpnn_num_params(8, ctypes.byref(c)) == 0 and c.value == 92688
    h = ctypes.c_void_p()
    assert lib.qaoa_mpnn_create(0, ctypes.byref(h)) == 1
    assert lib.qaoa_mpnn_create(4, None) == 1
    assert lib.qaoa_mpnn_destroy(None) == 0
    g = np.zeros(4)
    n = np.array([3], dtype=np.int32)
    off = np.array([0, 1], dtype=np.int64)
    e = np.array([[0, 1]], dtype=np.int32)
    assert lib.qaoa_mpnn_predict(None, 1, n.ctypes.data, off.ctypes.data, e.ctypes.data, None,
                                 g.ctypes.data, g.ctypes.data) == 1
    assert lib.qaoa_mpnn_set_params(None, g.ctypes.data) == 1
    assert lib.qaoa_mpnn_train_step(None, 1, n.ctypes.data, off.ctypes.data, e.ctypes.data, None,
                                    g.ctypes.data, g.ctypes.data, None, None) == 1


def test_mpnn_parameter_count_matches_oracle():
    from oracle import mpnn as om
    from paper_2407_13012_amd import qaoa_mpnn_num_params
    for p in (1, 3, 8, 16):
        assert qaoa_mpnn_num_params(p) == om.num_params(p)


def test_set_allocator_validation(lib):
    from paper_2407_13012_amd import Allocator
    from paper_2407_13012_amd._binding import ALLOC_FN
    assert lib.qaoa_set_allocator(None) == 0
    half = Allocator(ALLOC_FN(lambda n, s, u: None), ctypes.cast(None, type(Allocator().free)), None)
    assert lib.qaoa_set_allocator(ctypes.byref(half)) == 1
    assert lib.qaoa_set_allocator(None) == 0
