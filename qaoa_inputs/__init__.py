"""Seeded synthetic problem instances and angle schedules.

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark.  It holds no QAOA arithmetic: it only draws graphs, weights and
angles from numpy's PCG64 generator, so that both sides see identical inputs.

Instance families follow the evaluation section of the paper (MaxCut on
Erdos-Renyi G(n, p) and random 3-regular graphs) plus the 0-1 QUBO form of the
cost-function section (Eq. 2 restricted to terms of degree <= 2).  The paper's
own 444 graphs are not available; these generators are stand-ins with the same
structure.

Conventions
-----------
* Vertices / variables are 0-based; variable i is bit i of the basis index z.
* Edge lists are int32 arrays of shape (m, 2) with i < j, in lexicographic
  order; weights are float64 arrays of shape (m,), drawn after the structure,
  in edge order.
* Angles are float64 arrays gamma[p], beta[p]; layer l uses gamma[l], beta[l].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class MaxCut:
    """Weighted MaxCut instance: C(z) = sum of w_e over edges cut by z."""
    n: int
    edges: np.ndarray            # int32 (m, 2), i < j
    weights: Optional[np.ndarray]  # float64 (m,) or None for unit weights

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    def weight_array(self) -> np.ndarray:
        if self.weights is None:
            return np.ones(self.m, dtype=np.float64)
        return self.weights


@dataclasses.dataclass
class Qubo:
    """0-1 QUBO: C(z) = offset + sum_k J_k x_i x_j + sum_i h_i x_i, x_i = bit i of z."""
    n: int
    pairs: np.ndarray            # int32 (m, 2), i < j
    J: np.ndarray                # float64 (m,)
    h: np.ndarray                # float64 (n,)
    offset: float = 0.0

    @property
    def m(self) -> int:
        return int(self.pairs.shape[0])


def _pairs_bernoulli(rng: np.random.Generator, n: int, p_edge: float) -> np.ndarray:
    """Erdos-Renyi G(n, p): one Bernoulli(p) draw per pair i<j in lexicographic order."""
    edges = []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p_edge:
                edges.append((i, j))
    return np.asarray(edges, dtype=np.int32).reshape(-1, 2)


def erdos_renyi(n: int, p_edge: float, seed, weights: str = "unit",
                wlow: float = 0.0, whigh: float = 1.0) -> MaxCut:
    """MaxCut on G(n, p_edge).  weights: 'unit', 'uniform' (U[wlow, whigh]) or 'integer'
    (uniform integers in [wlow, whigh])."""
    rng = np.random.default_rng(seed)
    edges = _pairs_bernoulli(rng, n, p_edge)
    w = _draw_weights(rng, edges.shape[0], weights, wlow, whigh)
    return MaxCut(n=n, edges=edges, weights=w)


def random_regular(n: int, d: int, seed, weights: str = "unit",
                   wlow: float = 0.0, whigh: float = 1.0, max_tries: int = 100000) -> MaxCut:
    """Random d-regular graph by the configuration model with rejection of
    self-loops and multi-edges (uniform over simple d-regular graphs)."""
    if (n * d) % 2 or d >= n:
        raise ValueError("no simple d-regular graph on n vertices")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).size != key.size:
            continue
        order = np.argsort(key, kind="stable")
        edges = np.stack([lo[order], hi[order]], axis=1).astype(np.int32)
        w = _draw_weights(rng, edges.shape[0], weights, wlow, whigh)
        return MaxCut(n=n, edges=edges, weights=w)
    raise RuntimeError("configuration model did not produce a simple graph")


def complete_graph(n: int, seed=None, weights: str = "unit",
                   wlow: float = 0.0, whigh: float = 1.0) -> MaxCut:
    edges = np.asarray([(i, j) for i in range(n) for j in range(i + 1, n)],
                       dtype=np.int32).reshape(-1, 2)
    rng = np.random.default_rng(seed)
    return MaxCut(n=n, edges=edges, weights=_draw_weights(rng, edges.shape[0], weights, wlow, whigh))


def qubo_erdos_renyi(n: int, p_edge: float, seed, offset: float = 0.0) -> Qubo:
    """0-1 QUBO with ER(p_edge) coupling pattern, J_ij ~ N(0,1), h_i ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    pairs = _pairs_bernoulli(rng, n, p_edge)
    J = rng.standard_normal(pairs.shape[0])
    h = rng.standard_normal(n)
    return Qubo(n=n, pairs=pairs, J=J, h=h, offset=offset)


def qubo_blocks(n: int, block: int, p_edge: float, seed) -> Qubo:
    """QUBO whose couplings stay inside disjoint blocks of `block` consecutive
    variables (the last block may be shorter).  Used where an exact answer is
    needed at sizes too large for a full-state CPU evaluation: the state then
    factorises over blocks."""
    rng = np.random.default_rng(seed)
    pairs = []
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        for i in range(b0, b1):
            for j in range(i + 1, b1):
                if rng.random() < p_edge:
                    pairs.append((i, j))
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    J = rng.standard_normal(pairs.shape[0])
    h = rng.standard_normal(n)
    return Qubo(n=n, pairs=pairs, J=J, h=h)


@dataclasses.dataclass
class Poly:
    """General 0-1 polynomial (Eq. 2): C(z) = offset + sum_k w_k [z AND m_k == m_k]."""
    n: int
    masks: np.ndarray     # uint64 (L,)
    weights: np.ndarray   # float64 (L,)
    offset: float = 0.0

    @property
    def m(self) -> int:
        return int(self.masks.shape[0])


def poly_random(n: int, L: int, max_degree: int, seed, offset: float = 0.0) -> Poly:
    """L random terms of degree 1..max_degree on distinct variables, weights N(0,1)."""
    rng = np.random.default_rng(seed)
    masks = np.zeros(L, dtype=np.uint64)
    for k in range(L):
        d = int(rng.integers(1, max_degree + 1))
        vs = rng.choice(n, size=min(d, n), replace=False)
        masks[k] = np.uint64(sum(1 << int(v) for v in vs))
    return Poly(n=n, masks=masks, weights=rng.standard_normal(L), offset=offset)


def _draw_weights(rng, m, kind, wlow, whigh):
    if kind == "unit":
        return None
    if kind == "uniform":
        return rng.uniform(wlow, whigh, m)
    if kind == "integer":
        return rng.integers(int(wlow), int(whigh) + 1, m).astype(np.float64)
    raise ValueError(kind)


# ---------------------------------------------------------------- angles

def linear_ramp(p: int, dt: float = 1.0):
    """Constant-speed schedule of the QAOA background section:
    gamma_i = dt * i/p, beta_i = dt * (1 - i/p), i = 1..p."""
    i = np.arange(1, p + 1, dtype=np.float64)
    return dt * i / p, dt * (1.0 - i / p)


def ramp_with_noise(p: int, seed, sigma: float = 0.05, dt: float = 1.0):
    g, b = linear_ramp(p, dt)
    rng = np.random.default_rng(seed)
    return g + rng.normal(0.0, sigma, p), b + rng.normal(0.0, sigma, p)


def uniform_angles(p: int, seed):
    """gamma ~ U[0, pi], beta ~ U[0, pi/2]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, math.pi, p), rng.uniform(0.0, math.pi / 2, p)


# ---------------------------------------------------------------- named workloads

def workload_small():
    """Unweighted MaxCut on ER G(12, 0.5) from seed 0, depth p=2, angles
    gamma ~ U[0,pi], beta ~ U[0,pi/2] from seed (0, 1); 1024 samples, seed 0."""
    g = erdos_renyi(12, 0.5, seed=0)
    gamma, beta = uniform_angles(2, seed=[0, 1])
    return dict(instance=g, p=2, gamma=gamma, beta=beta, shots=1024, sample_seed=0)


def workload_regular26():
    """Weighted MaxCut on a random 3-regular graph, n=26, w ~ U[0,1], seed 1, p=6,
    linear ramp plus N(0, 0.05) noise (seed (1, 1))."""
    g = random_regular(26, 3, seed=1, weights="uniform", wlow=0.0, whigh=1.0)
    gamma, beta = ramp_with_noise(6, seed=[1, 1])
    return dict(instance=g, p=6, gamma=gamma, beta=beta)


def workload_qubo32(n: int = 32):
    """0-1 QUBO, ER(0.1) couplings, J,h ~ N(0,1), seed 2, p=3, ramp plus N(0,0.05)
    noise (seed (2, 1)); 10^6 samples with seed 2.  `n` below 32 gives the same
    family at a smaller size."""
    q = qubo_erdos_renyi(n, 0.1, seed=2)
    gamma, beta = ramp_with_noise(3, seed=[2, 1])
    return dict(instance=q, p=3, gamma=gamma, beta=beta, shots=10**6, sample_seed=2)


def batched_family(count: int, base_seed: int = 3_000_000, nmin: int = 10, nmax: int = 20):
    """Random weighted MaxCut graphs with n ~ U{nmin..nmax}, edge probability
    U[0.2, 0.8] and weights U[-1, 1]; graph g uses seed base_seed + g."""
    out = []
    for g in range(count):
        rng = np.random.default_rng(base_seed + g)
        n = int(rng.integers(nmin, nmax + 1))
        pe = float(rng.uniform(0.2, 0.8))
        edges = _pairs_bernoulli(rng, n, pe)
        w = rng.uniform(-1.0, 1.0, edges.shape[0])
        out.append(MaxCut(n=n, edges=edges, weights=w))
    return out


# ---------------------------------------------------------------- warm-start network inputs

def mpnn_param_shapes(p: int):
    """(name, shape) of the warm-start network's parameters in their flat order:
    three message-passing layers (W [128][2 d], b [128], d = 32 then 128) and the
    two-layer head (W [128][128], b [128], W [2p][128], b [2p])."""
    out, d = [], 32
    for l in range(3):
        out += [(f"W{l}", (128, 2 * d)), (f"b{l}", (128,))]
        d = 128
    return out + [("Wh1", (128, 128)), ("bh1", (128,)), ("Wh2", (2 * p, 128)), ("bh2", (2 * p,))]


def mpnn_init_params(p: int, seed) -> np.ndarray:
    """Initial parameters: each (W, b) pair uniform in +-1/sqrt(row length of W);
    the output layer scaled by 0.1 so that first predictions stay near the ramp."""
    rng = np.random.default_rng(seed)
    shapes = mpnn_param_shapes(p)
    parts = []
    for k in range(0, len(shapes), 2):
        (wn, ws), (_, bs) = shapes[k], shapes[k + 1]
        bound = 1.0 / math.sqrt(ws[1])
        scale = 0.1 if wn == "Wh2" else 1.0
        parts.append(scale * rng.uniform(-bound, bound, ws).reshape(-1))
        parts.append(scale * rng.uniform(-bound, bound, bs))
    return np.concatenate(parts)


def warmstart_eval_graphs(count: int = 512, n: int = 24, base_seed: int = 4_000_000):
    """Held-out Erdos-Renyi G(n, 0.5) graphs with weights U[-1, 1]; graph i uses seed base_seed + i."""
    return [erdos_renyi(n, 0.5, seed=base_seed + i, weights="uniform", wlow=-1.0, whigh=1.0)
            for i in range(count)]
