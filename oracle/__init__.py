"""CPU oracle for the QAOA hot path -- TEST INFRASTRUCTURE ONLY.

A plain FP64 implementation (``qaoa_oracle.c``) of what the GPU library
computes: cost diagonal, initial state, phase and mixer layers, expectation,
adjoint gradient and sampling, plus the Adam loop of the batched optimiser.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  The product path never
does, and this module never imports the product package.

The C source is compiled with gcc (``-O2 -ffp-contract=off -fopenmp``) into
``oracle/liboracle.so`` by :func:`build`; :func:`load` builds it on first use if
it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qaoa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib: Optional[ctypes.CDLL] = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc and return its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    d, i32, i64, u64, vp = (ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                            ctypes.c_uint64, ctypes.c_void_p)
    sig = {
        "oracle_cost_maxcut_entry": (d, [u64, i64, vp, vp]),
        "oracle_cost_maxcut": (None, [i32, i64, vp, vp, vp]),
        "oracle_cost_qubo_entry": (d, [u64, i32, i64, vp, vp, vp, d]),
        "oracle_cost_qubo": (None, [i32, i64, vp, vp, vp, d, vp]),
        "oracle_cost_poly_entry": (d, [u64, i64, vp, vp]),
        "oracle_cost_poly": (None, [i32, i64, vp, vp, vp]),
        "oracle_init_plus": (None, [i32, vp]),
        "oracle_apply_phase": (None, [i32, vp, d, vp]),
        "oracle_apply_rx": (None, [i32, i32, d, vp]),
        "oracle_apply_mixer": (None, [i32, d, vp]),
        "oracle_state": (None, [i32, vp, i32, vp, vp, vp]),
        "oracle_expectation": (d, [i32, vp, vp]),
        "oracle_gradient": (i32, [i32, vp, i32, vp, vp, vp, vp, vp]),
        "oracle_philox4x32_10": (None, [vp, vp, vp]),
        "oracle_uniform53": (d, [u64, u64]),
        "oracle_sample": (i32, [i32, vp, vp, i64, u64, vp, vp]),
        "oracle_num_threads": (i32, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(load().oracle_num_threads())


# ----------------------------------------------------------------- cost

def cost_maxcut(n: int, edges, weights=None) -> np.ndarray:
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    w = _f64(weights)
    C = np.empty(1 << n, dtype=np.float64)
    load().oracle_cost_maxcut(n, e.shape[0], _p(e), _p(w), _p(C))
    return C


def cost_maxcut_entry(z: int, edges, weights=None) -> float:
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    w = _f64(weights)
    return load().oracle_cost_maxcut_entry(int(z), e.shape[0], _p(e), _p(w))


def cost_qubo(n: int, pairs, J, h=None, offset: float = 0.0) -> np.ndarray:
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    J = _f64(J)
    h = _f64(h)
    C = np.empty(1 << n, dtype=np.float64)
    load().oracle_cost_qubo(n, pr.shape[0], _p(pr), _p(J), _p(h), float(offset), _p(C))
    return C


def cost_qubo_entry(z: int, n: int, pairs, J, h=None, offset: float = 0.0) -> float:
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    J = _f64(J)
    h = _f64(h)
    return load().oracle_cost_qubo_entry(int(z), n, pr.shape[0], _p(pr), _p(J), _p(h), float(offset))


def cost_poly(n: int, masks, weights) -> np.ndarray:
    m = np.ascontiguousarray(masks, dtype=np.uint64)
    w = _f64(weights)
    C = np.empty(1 << n, dtype=np.float64)
    load().oracle_cost_poly(n, m.shape[0], _p(m), _p(w), _p(C))
    return C


def cost_of(instance) -> np.ndarray:
    """Cost diagonal of a qaoa_inputs.MaxCut, Qubo or Poly instance."""
    if hasattr(instance, "edges"):
        return cost_maxcut(instance.n, instance.edges, instance.weights)
    if hasattr(instance, "masks"):
        # the constant is a term whose (empty) mask is always active, added first
        masks = np.concatenate([[0], np.asarray(instance.masks, np.uint64)]).astype(np.uint64)
        w = np.concatenate([[instance.offset], instance.weights])
        return cost_poly(instance.n, masks, w)
    return cost_qubo(instance.n, instance.pairs, instance.J, instance.h, instance.offset)


def cost_entry_of(instance, z: int) -> float:
    if hasattr(instance, "edges"):
        return cost_maxcut_entry(z, instance.edges, instance.weights)
    return cost_qubo_entry(z, instance.n, instance.pairs, instance.J, instance.h, instance.offset)


# ----------------------------------------------------------------- evolution

def init_plus(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    load().oracle_init_plus(n, _p(psi))
    return psi


def apply_phase(n: int, C: np.ndarray, gamma: float, psi: np.ndarray) -> None:
    load().oracle_apply_phase(n, _p(C), float(gamma), _p(psi))


def apply_rx(n: int, j: int, beta: float, psi: np.ndarray) -> None:
    load().oracle_apply_rx(n, j, float(beta), _p(psi))


def apply_mixer(n: int, beta: float, psi: np.ndarray) -> None:
    load().oracle_apply_mixer(n, float(beta), _p(psi))


def state(n: int, C: np.ndarray, gamma, beta) -> np.ndarray:
    g, b = _f64(gamma), _f64(beta)
    assert g.shape == b.shape
    C = _f64(C)
    psi = np.empty(1 << n, dtype=np.complex128)
    load().oracle_state(n, _p(C), g.shape[0], _p(g), _p(b), _p(psi))
    return psi


def expectation(n: int, C: np.ndarray, psi: np.ndarray) -> float:
    return load().oracle_expectation(n, _p(_f64(C)), _p(np.ascontiguousarray(psi, np.complex128)))


def gradient(n: int, C: np.ndarray, gamma, beta):
    """Return (E, dE/dgamma[p], dE/dbeta[p])."""
    g, b = _f64(gamma), _f64(beta)
    p = g.shape[0]
    E = ctypes.c_double()
    dg = np.zeros(p)
    db = np.zeros(p)
    rc = load().oracle_gradient(n, _p(_f64(C)), p, _p(g), _p(b), ctypes.byref(E), _p(dg), _p(db))
    if rc != 0:
        raise MemoryError("oracle_gradient: out of host memory")
    return E.value, dg, db


def philox4x32_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    load().oracle_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def uniform53(seed: int, s: int) -> float:
    return load().oracle_uniform53(int(seed), int(s))


def sample(n: int, psi: np.ndarray, C: Optional[np.ndarray], shots: int, seed: int):
    z = np.zeros(shots, dtype=np.uint64)
    cost = np.zeros(shots, dtype=np.float64) if C is not None else None
    rc = load().oracle_sample(n, _p(np.ascontiguousarray(psi, np.complex128)),
                              _p(_f64(C)), int(shots), int(seed), _p(z), _p(cost))
    if rc != 0:
        raise ValueError("oracle_sample failed (zero norm or out of memory)")
    return z, cost


def adam_ascent(fun, x0, steps: int, lr: float, beta1: float, beta2: float, eps: float):
    """Adam (Kingma & Ba 2015, Algorithm 1) on the ascent direction of fun.

    fun(x) -> (f, g) with g the gradient of f.  For t = 1..steps, with g_t the
    gradient at x_{t-1}: m_t = beta1 m_{t-1} + (1 - beta1) g_t,
    v_t = beta2 v_{t-1} + (1 - beta2) g_t^2, m^ = m_t / (1 - beta1^t),
    v^ = v_t / (1 - beta2^t), x_t = x_{t-1} + lr m^ / (sqrt(v^) + eps).
    Returns (x_steps, f(x_0), f(x_steps))."""
    x = np.array(x0, dtype=np.float64, copy=True)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    f_first = None
    for t in range(1, steps + 1):
        f, g = fun(x)
        g = np.asarray(g, dtype=np.float64)
        if f_first is None:
            f_first = f
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        x = x + lr * mh / (np.sqrt(vh) + eps)
    f_last, _ = fun(x)
    if f_first is None:
        f_first = f_last
    return x, f_first, f_last


def adam_qaoa(n: int, C: np.ndarray, gamma, beta, steps: int, lr: float = 0.05, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, scale: float = 1.0):
    """Adam ascent on scale * E(gamma, beta) with the adjoint gradient above.
    Returns (gamma, beta, E at the start angles, E at the final angles)."""
    p = len(gamma)

    def fun(x):
        E, dg, db = gradient(n, C, x[:p], x[p:])
        return E, scale * np.concatenate([dg, db])

    x, e0, e1 = adam_ascent(fun, np.concatenate([_f64(gamma), _f64(beta)]), steps, lr, beta1, beta2, eps)
    return x[:p], x[p:], e0, e1
