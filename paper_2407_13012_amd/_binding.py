"""ctypes marshalling for libqaoa.so.  Names follow the C ABI (include/qaoa.h)."""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

QAOA_C128 = 0
QAOA_C64 = 1
_PREC = {"c128": QAOA_C128, "complex128": QAOA_C128, QAOA_C128: QAOA_C128,
         "c64": QAOA_C64, "complex64": QAOA_C64, QAOA_C64: QAOA_C64}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libqaoa.so")
_lib: Optional[ctypes.CDLL] = None


class LbfgsOptions(ctypes.Structure):
    """Mirror of qaoa_lbfgs_options."""
    _fields_ = [("max_iter", ctypes.c_int32), ("history", ctypes.c_int32), ("gtol", ctypes.c_double),
                ("ftol", ctypes.c_double), ("max_evals", ctypes.c_int32)]


BATCH_MAX_QUBITS = 24


class BatchOptions(ctypes.Structure):
    """Mirror of qaoa_batch_options."""
    _fields_ = [("steps", ctypes.c_int32), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("workgroups", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("group_by_n", ctypes.c_int32 * (BATCH_MAX_QUBITS + 1)),
                ("resident_max_n", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """Mirror of qaoa_allocator."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class MpnnAdam(ctypes.Structure):
    """Mirror of qaoa_mpnn_adam."""
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


OBJECTIVE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.c_void_p)


def library_path() -> str:
    return _LIB_PATH


class QaoaError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load_library()
        self.status = status
        self.message = lib.qaoa_last_error_message().decode()
        super().__init__(f"{where}: {lib.qaoa_status_string(status).decode()} ({self.message})")


def load_library() -> ctypes.CDLL:
    """Load the built HIP library.  Raises ImportError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python paper_2407_13012_amd/build.py` (hipcc, gfx950)")
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, u64, d, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    pvp = ctypes.POINTER(ctypes.c_void_p)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pd = ctypes.POINTER(ctypes.c_double)
    sigs = {
        "qaoa_create_maxcut": [i32, i64, vp, vp, i32, vp, pvp],
        "qaoa_create_qubo": [i32, i64, vp, vp, vp, d, i32, vp, pvp],
        "qaoa_create_poly": [i32, i64, vp, vp, d, i32, vp, pvp],
        "qaoa_destroy": [vp],
        "qaoa_get_info": [vp, pi32, pi32],
        "qaoa_cost_diagonal": [vp, vp, i32],
        "qaoa_cost_extrema": [vp, pd, pd],
        "qaoa_statevector": [vp, i32, vp, vp, vp, i32],
        "qaoa_expectation": [vp, pd],
        "qaoa_evaluate": [vp, i32, vp, vp, pd],
        "qaoa_gradient": [vp, i32, vp, vp, pd, vp, vp],
        "qaoa_gradient_from_state": [vp, i32, vp, vp, vp, vp],
        "qaoa_gradient_noalloc": [vp, i32, vp, vp, vp, vp, vp, i32],
        "qaoa_sample": [vp, i64, u64, vp, vp, i32],
        "qaoa_pass_plan": [i32, i32, i32, pi32, vp, vp],
        "qaoa_lbfgs_minimize": [i32, vp, OBJECTIVE_FN, vp, ctypes.POINTER(LbfgsOptions), pd,
                                pi32, pi32, vp, vp],
        "qaoa_optimize": [vp, i32, vp, vp, ctypes.POINTER(LbfgsOptions), pd, pi32, pi32, vp, vp],
        "qaoa_profile_enable": [vp, i32],
        "qaoa_batch_create": [i32, vp, vp, vp, vp, i32, ctypes.POINTER(BatchOptions), pvp],
        "qaoa_batch_run": [vp, vp, vp, vp, vp, vp, vp],
        "qaoa_batch_destroy": [vp],
        "qaoa_batch_timeline": [vp, vp, vp, vp],
        "qaoa_set_allocator": [ctypes.POINTER(Allocator)],
        "qaoa_mpnn_num_params": [i32, ctypes.POINTER(i64)],
        "qaoa_mpnn_create": [i32, pvp],
        "qaoa_mpnn_destroy": [vp],
        "qaoa_mpnn_set_params": [vp, vp],
        "qaoa_mpnn_get_params": [vp, vp],
        "qaoa_mpnn_predict": [vp, i32, vp, vp, vp, vp, vp, vp],
        "qaoa_mpnn_loss_grad": [vp, i32, vp, vp, vp, vp, vp, vp, pd, vp],
        "qaoa_mpnn_train_step": [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(MpnnAdam), pd],
        "qaoa_profile_read": [vp, i32, ctypes.POINTER(i64), pd, pd],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.qaoa_status_string.argtypes = [ctypes.c_int]
    lib.qaoa_status_string.restype = ctypes.c_char_p
    lib.qaoa_last_error_message.argtypes = []
    lib.qaoa_last_error_message.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, where: str) -> None:
    if status != 0:
        raise QaoaError(status, where)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _stream(stream):
    """None -> torch's current HIP stream when a GPU is visible, else NULL."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _angles(gamma, beta):
    g = np.ascontiguousarray(gamma, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
    if g.shape != b.shape:
        raise ValueError("gamma and beta must have the same length")
    return g, b


def _is_device_tensor(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


# ---------------------------------------------------------------- C-named calls

def qaoa_create_maxcut(n: int, edges, weights=None, precision="c128", stream=None):
    lib = load_library()
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    if w is not None and w.shape[0] != e.shape[0]:
        raise ValueError("weights must have one entry per edge")
    h = ctypes.c_void_p()
    _check(lib.qaoa_create_maxcut(int(n), e.shape[0], _ptr(e), _ptr(w), _PREC[precision],
                                  _stream(stream), ctypes.byref(h)), "qaoa_create_maxcut")
    return h


def qaoa_create_qubo(n: int, pairs, J, h=None, offset: float = 0.0, precision="c128", stream=None):
    lib = load_library()
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    Jv = np.ascontiguousarray(J, dtype=np.float64).reshape(-1)
    if Jv.shape[0] != pr.shape[0]:
        raise ValueError("J must have one entry per pair")
    hv = None if h is None else np.ascontiguousarray(h, dtype=np.float64).reshape(-1)
    if hv is not None and hv.shape[0] != n:
        raise ValueError("h must have n entries")
    out = ctypes.c_void_p()
    _check(lib.qaoa_create_qubo(int(n), pr.shape[0], _ptr(pr), _ptr(Jv) if Jv.size else None,
                                _ptr(hv), float(offset), _PREC[precision], _stream(stream),
                                ctypes.byref(out)), "qaoa_create_qubo")
    return out


def qaoa_create_poly(n: int, masks, weights, offset: float = 0.0, precision="c128", stream=None):
    lib = load_library()
    m = np.ascontiguousarray(masks, dtype=np.uint64).reshape(-1)
    w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    if m.shape != w.shape:
        raise ValueError("masks and weights must have the same length")
    out = ctypes.c_void_p()
    _check(lib.qaoa_create_poly(int(n), m.size, _ptr(m) if m.size else None, _ptr(w) if w.size else None,
                                float(offset), _PREC[precision], _stream(stream), ctypes.byref(out)),
           "qaoa_create_poly")
    return out


def qaoa_destroy(h) -> None:
    _check(load_library().qaoa_destroy(h), "qaoa_destroy")


def qaoa_get_info(h):
    n, p = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().qaoa_get_info(h, ctypes.byref(n), ctypes.byref(p)), "qaoa_get_info")
    return n.value, p.value


def qaoa_cost_diagonal(h, out=None):
    """Return C as a numpy fp64 array, or fill `out` (numpy array or device tensor)."""
    n, _ = qaoa_get_info(h)
    lib = load_library()
    if out is None:
        out = np.empty(1 << n, dtype=np.float64)
    if _is_device_tensor(out):
        _check(lib.qaoa_cost_diagonal(h, ctypes.c_void_p(out.data_ptr()), 1), "qaoa_cost_diagonal")
    else:
        assert out.dtype == np.float64 and out.size == 1 << n and out.flags.c_contiguous
        _check(lib.qaoa_cost_diagonal(h, _ptr(out), 0), "qaoa_cost_diagonal")
    return out


def qaoa_cost_extrema(h):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(load_library().qaoa_cost_extrema(h, ctypes.byref(lo), ctypes.byref(hi)), "qaoa_cost_extrema")
    return lo.value, hi.value


def qaoa_statevector(h, gamma, beta, out=None, copy: bool = True):
    """Prepare the state; return a copy (numpy or the given device tensor) unless copy=False."""
    lib = load_library()
    g, b = _angles(gamma, beta)
    n, prec = qaoa_get_info(h)
    if not copy:
        _check(lib.qaoa_statevector(h, g.size, _ptr(g), _ptr(b), None, 0), "qaoa_statevector")
        return None
    if out is None:
        out = np.empty(1 << n, dtype=np.complex64 if prec == QAOA_C64 else np.complex128)
    if _is_device_tensor(out):
        _check(lib.qaoa_statevector(h, g.size, _ptr(g), _ptr(b), ctypes.c_void_p(out.data_ptr()), 1),
               "qaoa_statevector")
    else:
        _check(lib.qaoa_statevector(h, g.size, _ptr(g), _ptr(b), _ptr(out), 0), "qaoa_statevector")
    return out


def qaoa_expectation(h) -> float:
    E = ctypes.c_double()
    _check(load_library().qaoa_expectation(h, ctypes.byref(E)), "qaoa_expectation")
    return E.value


def qaoa_evaluate(h, gamma, beta) -> float:
    g, b = _angles(gamma, beta)
    E = ctypes.c_double()
    _check(load_library().qaoa_evaluate(h, g.size, _ptr(g), _ptr(b), ctypes.byref(E)), "qaoa_evaluate")
    return E.value


def qaoa_gradient(h, gamma, beta):
    """Return (E, dE/dgamma, dE/dbeta)."""
    g, b = _angles(gamma, beta)
    E = ctypes.c_double()
    dg = np.zeros(g.size)
    db = np.zeros(g.size)
    _check(load_library().qaoa_gradient(h, g.size, _ptr(g), _ptr(b), ctypes.byref(E), _ptr(dg), _ptr(db)),
           "qaoa_gradient")
    return E.value, dg, db


def qaoa_gradient_from_state(h, gamma, beta):
    """(dE/dgamma, dE/dbeta) by the reverse sweep alone, from the state that a
    preceding qaoa_evaluate / qaoa_statevector left at the same angles."""
    g, b = _angles(gamma, beta)
    dg = np.zeros(g.size)
    db = np.zeros(g.size)
    _check(load_library().qaoa_gradient_from_state(h, g.size, _ptr(g), _ptr(b), _ptr(dg), _ptr(db)),
           "qaoa_gradient_from_state")
    return dg, db


def qaoa_gradient_noalloc(h, gamma, beta, out=None):
    """qaoa_gradient through the library's fixed scratch (no device allocation).
    Without `out`: returns (E, dE/dgamma, dE/dbeta) on the host.  With `out`, a
    float64 device tensor of 2p + 1 entries: fills it with (E, dE/dgamma,
    dE/dbeta) in stream order and returns it."""
    g, b = _angles(gamma, beta)
    p = g.size
    lib = load_library()
    if out is None:
        E = ctypes.c_double()
        dg = np.zeros(p)
        db = np.zeros(p)
        _check(lib.qaoa_gradient_noalloc(h, p, _ptr(g), _ptr(b), ctypes.byref(E), _ptr(dg), _ptr(db), 0),
               "qaoa_gradient_noalloc")
        return E.value, dg, db
    if out.numel() != 2 * p + 1 or not out.is_cuda or out.dtype != _torch_float64() or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 device tensor of 2p + 1 entries")
    base = out.data_ptr()
    _check(lib.qaoa_gradient_noalloc(h, p, _ptr(g), _ptr(b), ctypes.c_void_p(base), ctypes.c_void_p(base + 8),
                                     ctypes.c_void_p(base + 8 * (1 + p)), 1), "qaoa_gradient_noalloc")
    return out


def _torch_float64():
    import torch
    return torch.float64


def qaoa_sample(h, shots: int, seed: int, z_out=None, cost_out=None, with_cost: bool = True):
    """Draw shots from the current state.  Host numpy outputs by default; pass
    device tensors (uint64-compatible int64 and float64) as z_out/cost_out to
    keep the results on the GPU."""
    lib = load_library()
    if z_out is not None and _is_device_tensor(z_out):
        cptr = ctypes.c_void_p(cost_out.data_ptr()) if cost_out is not None else None
        _check(lib.qaoa_sample(h, int(shots), int(seed), ctypes.c_void_p(z_out.data_ptr()), cptr, 1),
               "qaoa_sample")
        return z_out, cost_out
    m = max(int(shots), 0)  # a negative count is passed through for the library to reject
    z = np.zeros(m, dtype=np.uint64) if z_out is None else z_out
    c = (np.zeros(m, dtype=np.float64) if with_cost else None) if cost_out is None else cost_out
    _check(lib.qaoa_sample(h, int(shots), int(seed) & (2**64 - 1), _ptr(z), _ptr(c), 0), "qaoa_sample")
    return z, c


def qaoa_pass_plan(n: int, precision="c128"):
    """[(tile_bits, target_bits)] of the sweeps that make up one mixer layer."""
    cnt = ctypes.c_int32()
    tb = np.zeros(16, dtype=np.uint64)
    tg = np.zeros(16, dtype=np.uint64)
    _check(load_library().qaoa_pass_plan(int(n), _PREC[precision], 16, ctypes.byref(cnt), _ptr(tb), _ptr(tg)),
           "qaoa_pass_plan")
    return [(int(tb[i]), int(tg[i])) for i in range(cnt.value)]


def _options(max_iter, history, gtol, ftol, max_evals):
    return LbfgsOptions(int(max_iter), int(history), float(gtol), float(ftol), int(max_evals))


def qaoa_lbfgs_minimize(fun, x0, max_iter=100, history=10, gtol=1e-8, ftol=0.0, max_evals=1000,
                        trace=False):
    """Minimise fun(x) -> (f, g) from x0 with the library's L-BFGS.
    Returns (x, f, iters, evals[, trace_x, trace_f])."""
    lib = load_library()
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    dim = x.size
    err = []

    def cb(xp, fp, gp, _user):
        try:
            xv = np.ctypeslib.as_array(xp, shape=(dim,)).copy()
            f, g = fun(xv)
            fp[0] = float(f)
            gv = np.asarray(g, dtype=np.float64)
            for i in range(dim):
                gp[i] = gv[i]
            return 0
        except Exception as e:  # stop the optimiser; re-raised below
            err.append(e)
            return 1

    cfun = OBJECTIVE_FN(cb)
    fx = ctypes.c_double()
    it, ev = ctypes.c_int32(), ctypes.c_int32()
    tx = np.zeros((max_iter + 1, dim)) if trace else None
    tf = np.zeros(max_iter + 1) if trace else None
    opt = _options(max_iter, history, gtol, ftol, max_evals)
    st = lib.qaoa_lbfgs_minimize(dim, _ptr(x), cfun, None, ctypes.byref(opt), ctypes.byref(fx),
                                 ctypes.byref(it), ctypes.byref(ev), _ptr(tx), _ptr(tf))
    if err:
        raise err[0]
    _check(st, "qaoa_lbfgs_minimize")
    if trace:
        return x, fx.value, it.value, ev.value, tx[: it.value + 1], tf[: it.value + 1]
    return x, fx.value, it.value, ev.value


def qaoa_optimize(h, gamma, beta, max_iter=100, history=10, gtol=1e-8, ftol=0.0, max_evals=1000,
                  trace=False):
    """Maximise E(gamma, beta) with L-BFGS on the GPU gradient.
    Returns (gamma, beta, E, iters, evals[, trace_x, trace_E])."""
    g, b = _angles(gamma, beta)
    g, b = g.copy(), b.copy()
    p = g.size
    E = ctypes.c_double()
    it, ev = ctypes.c_int32(), ctypes.c_int32()
    tx = np.zeros((max_iter + 1, 2 * p)) if trace else None
    tf = np.zeros(max_iter + 1) if trace else None
    opt = _options(max_iter, history, gtol, ftol, max_evals)
    _check(load_library().qaoa_optimize(h, p, _ptr(g), _ptr(b), ctypes.byref(opt), ctypes.byref(E),
                                        ctypes.byref(it), ctypes.byref(ev), _ptr(tx), _ptr(tf)),
           "qaoa_optimize")
    if trace:
        return g, b, E.value, it.value, ev.value, tx[: it.value + 1], tf[: it.value + 1]
    return g, b, E.value, it.value, ev.value


def batch_options(steps=100, lr=0.05, beta1=0.9, beta2=0.999, eps=1e-8, workgroups=0, max_group=10,
                  use_graph=True, waves_per_simd=1, group_by_n=None, resident_max_n=0) -> BatchOptions:
    gb = (ctypes.c_int32 * (BATCH_MAX_QUBITS + 1))()
    for n, k in (group_by_n or {}).items():
        gb[int(n)] = int(k)
    return BatchOptions(int(steps), float(lr), float(beta1), float(beta2), float(eps), int(workgroups),
                        int(max_group), 1 if use_graph else 0, int(waves_per_simd), gb, int(resident_max_n))


def _graph_arrays(graphs):
    """(n, edge_offsets, edges, w or None) of a graph list in the batch layout."""
    count = len(graphs)
    n = np.asarray([g.n for g in graphs], dtype=np.int32)
    m = np.asarray([np.asarray(g.edges).reshape(-1, 2).shape[0] for g in graphs], dtype=np.int64)
    off = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(m, out=off[1:])
    edges = (np.concatenate([np.asarray(g.edges, dtype=np.int32).reshape(-1, 2) for g in graphs])
             if count else np.zeros((0, 2), np.int32))
    edges = np.ascontiguousarray(edges, dtype=np.int32)
    unit = all(g.weights is None for g in graphs)
    w = None if unit else np.ascontiguousarray(np.concatenate(
        [np.ones(int(mi)) if g.weights is None else np.asarray(g.weights, dtype=np.float64).reshape(-1)
         for g, mi in zip(graphs, m)]) if count else np.zeros(0), dtype=np.float64)
    return n, off, edges, w


def _graph_ptrs(arrs):
    n, off, edges, w = arrs
    return (_ptr(n) if n.size else None, _ptr(off), _ptr(edges) if edges.size else None,
            _ptr(w) if w is not None and w.size else None)


def qaoa_batch_create(graphs, p: int, options: Optional[BatchOptions] = None):
    """graphs: sequence of objects with .n, .edges (m, 2) and .weights (m,) or None."""
    lib = load_library()
    count = len(graphs)
    arrs = _graph_arrays(graphs)
    out = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(lib.qaoa_batch_create(count, *_graph_ptrs(arrs), int(p), opt, ctypes.byref(out)),
           "qaoa_batch_create")
    return out


def qaoa_batch_run(b, gamma0, beta0):
    """Run the batch from start angles [count][p]; returns (gamma, beta, e_first, e_last)."""
    g0 = np.ascontiguousarray(gamma0, dtype=np.float64)
    b0 = np.ascontiguousarray(beta0, dtype=np.float64)
    if g0.shape != b0.shape or g0.ndim != 2:
        raise ValueError("gamma0 and beta0 must both have shape (count, p)")
    g, bb = np.empty_like(g0), np.empty_like(b0)
    e0, e1 = np.empty(g0.shape[0]), np.empty(g0.shape[0])
    _check(load_library().qaoa_batch_run(b, _ptr(g0), _ptr(b0), _ptr(g), _ptr(bb), _ptr(e0), _ptr(e1)),
           "qaoa_batch_run")
    return g, bb, e0, e1


def qaoa_batch_timeline(b, count: int):
    """(start_s, end_s, which_launch) per instance of the last run."""
    t0, t1 = np.empty(count), np.empty(count)
    which = np.empty(count, dtype=np.int32)
    _check(load_library().qaoa_batch_timeline(b, _ptr(t0), _ptr(t1), _ptr(which)), "qaoa_batch_timeline")
    return t0, t1, which


def qaoa_batch_destroy(b) -> None:
    _check(load_library().qaoa_batch_destroy(b), "qaoa_batch_destroy")


def qaoa_mpnn_num_params(p: int) -> int:
    c = ctypes.c_int64()
    _check(load_library().qaoa_mpnn_num_params(int(p), ctypes.byref(c)), "qaoa_mpnn_num_params")
    return c.value


def qaoa_mpnn_create(p: int):
    out = ctypes.c_void_p()
    _check(load_library().qaoa_mpnn_create(int(p), ctypes.byref(out)), "qaoa_mpnn_create")
    return out


def qaoa_mpnn_destroy(m) -> None:
    _check(load_library().qaoa_mpnn_destroy(m), "qaoa_mpnn_destroy")


def qaoa_mpnn_set_params(m, theta) -> None:
    t = np.ascontiguousarray(theta, dtype=np.float32)
    _check(load_library().qaoa_mpnn_set_params(m, _ptr(t)), "qaoa_mpnn_set_params")


def qaoa_mpnn_get_params(m, p: int) -> np.ndarray:
    t = np.empty(qaoa_mpnn_num_params(p), dtype=np.float32)
    _check(load_library().qaoa_mpnn_get_params(m, _ptr(t)), "qaoa_mpnn_get_params")
    return t


def qaoa_mpnn_predict(m, graphs, p: int):
    arrs = _graph_arrays(graphs)
    g = np.empty((len(graphs), p))
    b = np.empty((len(graphs), p))
    _check(load_library().qaoa_mpnn_predict(m, len(graphs), *_graph_ptrs(arrs), _ptr(g), _ptr(b)),
           "qaoa_mpnn_predict")
    return g, b


def qaoa_mpnn_loss_grad(m, graphs, gamma_t, beta_t, p: int, want_grad: bool = True):
    arrs = _graph_arrays(graphs)
    gt = np.ascontiguousarray(gamma_t, dtype=np.float64)
    bt = np.ascontiguousarray(beta_t, dtype=np.float64)
    if gt.shape != (len(graphs), p) or bt.shape != (len(graphs), p):
        raise ValueError("targets must have shape (count, p)")
    loss = ctypes.c_double()
    grad = np.empty(qaoa_mpnn_num_params(p), dtype=np.float32) if want_grad else None
    _check(load_library().qaoa_mpnn_loss_grad(m, len(graphs), *_graph_ptrs(arrs), _ptr(gt), _ptr(bt),
                                              ctypes.byref(loss), _ptr(grad)), "qaoa_mpnn_loss_grad")
    return loss.value, grad


def qaoa_mpnn_train_step(m, graphs, gamma_t, beta_t, p: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    arrs = _graph_arrays(graphs)
    gt = np.ascontiguousarray(gamma_t, dtype=np.float64)
    bt = np.ascontiguousarray(beta_t, dtype=np.float64)
    if gt.shape != (len(graphs), p) or bt.shape != (len(graphs), p):
        raise ValueError("targets must have shape (count, p)")
    loss = ctypes.c_double()
    opt = MpnnAdam(float(lr), float(beta1), float(beta2), float(eps))
    _check(load_library().qaoa_mpnn_train_step(m, len(graphs), *_graph_ptrs(arrs), _ptr(gt), _ptr(bt),
                                               ctypes.byref(opt), ctypes.byref(loss)), "qaoa_mpnn_train_step")
    return loss.value


PASS_KINDS = ("forward", "turn", "backward", "boundary_forward", "boundary_backward")


def qaoa_profile_enable(h, on: bool = True) -> None:
    _check(load_library().qaoa_profile_enable(h, 1 if on else 0), "qaoa_profile_enable")


def qaoa_profile_read(h, kind: int):
    """Return (launches, total_ms, total_algorithmic_bytes) for one pass kind (index into PASS_KINDS)."""
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().qaoa_profile_read(h, int(kind), ctypes.byref(n), ctypes.byref(ms),
                                            ctypes.byref(by)), "qaoa_profile_read")
    return n.value, ms.value, by.value


def qaoa_set_allocator(allocator: Optional[Allocator]) -> None:
    """Allocator for handles created afterwards on this thread (None: hipMalloc)."""
    lib = load_library()
    _check(lib.qaoa_set_allocator(ctypes.byref(allocator) if allocator is not None else None),
           "qaoa_set_allocator")


_torch_allocator: Optional[Allocator] = None


def torch_allocator() -> Allocator:
    """An allocator backed by torch's caching allocator (the callbacks live for
    the whole process, as handles may outlive any scope)."""
    global _torch_allocator
    if _torch_allocator is None:
        import torch

        def _alloc(nbytes, stream, _user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                          int(stream or 0))
            except Exception:
                return None

        def _free(ptr, _nbytes, _stream, _user):
            torch.cuda.caching_allocator_delete(int(ptr))

        _torch_allocator = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    return _torch_allocator


class use_torch_allocator:
    """Context manager: handles created inside take their device buffers from
    torch's caching allocator."""

    def __enter__(self):
        qaoa_set_allocator(torch_allocator())
        return self

    def __exit__(self, *exc):
        qaoa_set_allocator(None)


def qaoa_status_string(status: int) -> str:
    return load_library().qaoa_status_string(status).decode()


def qaoa_last_error_message() -> str:
    return load_library().qaoa_last_error_message().decode()


# ---------------------------------------------------------------- convenience wrapper

class QaoaHandle:
    """Owning wrapper: ``with QaoaHandle.maxcut(n, edges, w) as q: q.gradient(g, b)``."""

    def __init__(self, raw):
        self._h = raw

    @classmethod
    def maxcut(cls, n, edges, weights=None, precision="c128", stream=None):
        return cls(qaoa_create_maxcut(n, edges, weights, precision, stream))

    @classmethod
    def qubo(cls, n, pairs, J, h=None, offset=0.0, precision="c128", stream=None):
        return cls(qaoa_create_qubo(n, pairs, J, h, offset, precision, stream))

    @classmethod
    def poly(cls, n, masks, weights, offset=0.0, precision="c128", stream=None):
        return cls(qaoa_create_poly(n, masks, weights, offset, precision, stream))

    @classmethod
    def from_instance(cls, inst, precision="c128", stream=None):
        if hasattr(inst, "edges"):
            return cls.maxcut(inst.n, inst.edges, inst.weights, precision, stream)
        if hasattr(inst, "masks"):
            return cls.poly(inst.n, inst.masks, inst.weights, inst.offset, precision, stream)
        return cls.qubo(inst.n, inst.pairs, inst.J, inst.h, inst.offset, precision, stream)

    @property
    def raw(self):
        return self._h

    @property
    def n(self) -> int:
        return qaoa_get_info(self._h)[0]

    def close(self):
        if self._h is not None:
            qaoa_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cost_diagonal(self, out=None):
        return qaoa_cost_diagonal(self._h, out)

    def cost_extrema(self):
        return qaoa_cost_extrema(self._h)

    def statevector(self, gamma: Sequence[float], beta: Sequence[float], out=None, copy=True):
        return qaoa_statevector(self._h, gamma, beta, out, copy)

    def expectation(self) -> float:
        return qaoa_expectation(self._h)

    def evaluate(self, gamma, beta) -> float:
        return qaoa_evaluate(self._h, gamma, beta)

    def gradient(self, gamma, beta):
        return qaoa_gradient(self._h, gamma, beta)

    def gradient_from_state(self, gamma, beta):
        return qaoa_gradient_from_state(self._h, gamma, beta)

    def gradient_noalloc(self, gamma, beta, out=None):
        return qaoa_gradient_noalloc(self._h, gamma, beta, out)

    def sample(self, shots: int, seed: int, **kw):
        return qaoa_sample(self._h, shots, seed, **kw)

    def optimize(self, gamma, beta, **kw):
        return qaoa_optimize(self._h, gamma, beta, **kw)

    def profile_enable(self, on: bool = True):
        qaoa_profile_enable(self._h, on)

    def profile_read(self):
        """{kind: (launches, ms, bytes)} for every pass kind in PASS_KINDS."""
        return {k: qaoa_profile_read(self._h, i) for i, k in enumerate(PASS_KINDS)}


class QaoaBatch:
    """Owning wrapper of a batched-engine object (qaoa_batch_*): many MaxCut
    instances optimised with on-device Adam in one persistent launch."""

    def __init__(self, graphs, p: int, **options):
        self.count = len(graphs)
        self.p = int(p)
        self.options = dict(options)
        self._b = qaoa_batch_create(graphs, p, batch_options(**options))

    def run(self, gamma0, beta0):
        """Returns (gamma, beta, e_first, e_last) as numpy arrays."""
        if self._b is None:
            raise ValueError("batch is closed")
        return qaoa_batch_run(self._b, gamma0, beta0)

    def timeline(self):
        """(start_s, end_s, which_launch) of every instance in the last run."""
        if self._b is None:
            raise ValueError("batch is closed")
        return qaoa_batch_timeline(self._b, self.count)

    def close(self):
        if self._b is not None:
            qaoa_batch_destroy(self._b)
            self._b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class QaoaMpnn:
    """Owning wrapper of the warm-start network (qaoa_mpnn_*)."""

    def __init__(self, p: int, theta=None):
        self.p = int(p)
        self._m = qaoa_mpnn_create(self.p)
        if theta is not None:
            self.set_params(theta)

    @property
    def num_params(self) -> int:
        return qaoa_mpnn_num_params(self.p)

    def set_params(self, theta):
        qaoa_mpnn_set_params(self._m, theta)

    def get_params(self) -> np.ndarray:
        return qaoa_mpnn_get_params(self._m, self.p)

    def predict(self, graphs):
        return qaoa_mpnn_predict(self._m, graphs, self.p)

    def loss_grad(self, graphs, gamma_t, beta_t, want_grad=True):
        return qaoa_mpnn_loss_grad(self._m, graphs, gamma_t, beta_t, self.p, want_grad)

    def train_step(self, graphs, gamma_t, beta_t, **adam):
        return qaoa_mpnn_train_step(self._m, graphs, gamma_t, beta_t, self.p, **adam)

    def close(self):
        if self._m is not None:
            qaoa_mpnn_destroy(self._m)
            self._m = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
