"""CPU oracle of the warm-start message-passing network -- TEST INFRASTRUCTURE ONLY.

Plain numpy (float64) forward pass, mean-squared-error loss, hand-derived
backward pass and Adam step of the network that predicts QAOA angles from a
weighted graph.  Only the test-suite may import this module; it shares no code
with the HIP path.

Network (all sizes fixed: hidden width 128, three message-passing layers):
  node input   x_v = (deg_v / 8, wdeg_v / 8, 1, sqdeg_v / 8, 0, ..., 0)  (width 32),
               with deg_v the number of incident edges, wdeg_v the sum of
               their weights and sqdeg_v the sum of their squared weights
  layer l      H' = ReLU([H | A H] W_l^T + b_l),  A the symmetric weighted
               adjacency (A[i][j] = A[j][i] = sum of w over edges {i, j})
  readout      g = mean over the graph's nodes of H after layer 3
  head         Y = ReLU(g W_1^T + b_1) W_2^T + b_2   (2p outputs)
  angles       gamma_i = i/p + Y_i,  beta_i = 1 - i/p + Y_{p+i}   (i = 1..p):
               the linear-ramp schedule plus a learned correction
  loss         mean over graphs and the 2p angles of (angle - target)^2

With ``bf16_ops=True`` every matrix-product operand is rounded to bfloat16 at the
same points as the GPU path (activations, aggregated messages, weights, and the
gradients fed to the weight-gradient products), the products themselves being
exact sums in float64; element-wise work stays unrounded.

Flat parameter layout (float32 on the GPU, float64 here):
  for l in 0, 1, 2:  W_l [128][2 d_l] row-major, b_l [128]    (d_0 = 32, d_1 = d_2 = 128)
  W_1 [128][128], b_1 [128], W_2 [2p][128], b_2 [2p]
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

HID = 128
FIN = 32
LAYERS = 3


def dims(p: int) -> List[Tuple[str, Tuple[int, ...]]]:
    out = []
    d = FIN
    for l in range(LAYERS):
        out.append((f"W{l}", (HID, 2 * d)))
        out.append((f"b{l}", (HID,)))
        d = HID
    out += [("Wh1", (HID, HID)), ("bh1", (HID,)), ("Wh2", (2 * p, HID)), ("bh2", (2 * p,))]
    return out


def num_params(p: int) -> int:
    return sum(int(np.prod(s)) for _, s in dims(p))


def unflatten(theta: np.ndarray, p: int) -> dict:
    out, o = {}, 0
    for name, shape in dims(p):
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def flatten(parts: dict, p: int) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in dims(p)])


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via float32, round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def graph_batch(graphs: Sequence):
    """Node offsets, dense block-diagonal adjacency and input features of a batch."""
    ns = [int(g.n) for g in graphs]
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum(ns, out=off[1:])
    N = int(off[-1])
    A = np.zeros((N, N))
    X = np.zeros((N, FIN))
    for gi, g in enumerate(graphs):
        o = off[gi]
        e = np.asarray(g.edges, dtype=np.int64).reshape(-1, 2)
        w = g.weight_array() if hasattr(g, "weight_array") else np.asarray(g.weights, dtype=np.float64)
        for (i, j), wk in zip(e, w):
            A[o + i, o + j] += wk
            A[o + j, o + i] += wk
            X[o + i, 0] += 1.0
            X[o + j, 0] += 1.0
            X[o + i, 1] += wk
            X[o + j, 1] += wk
            X[o + i, 3] += wk * wk
            X[o + j, 3] += wk * wk
    X[:, 0] /= 8.0
    X[:, 1] /= 8.0
    X[:, 3] /= 8.0
    X[:, 2] = 1.0
    return off, A, X


def _r(x, on):
    return bf16(x) if on else x


def forward(theta: np.ndarray, graphs: Sequence, p: int, bf16_ops: bool = False, keep: bool = False):
    """Predicted angles (gamma [G][p], beta [G][p]); with keep=True also the
    intermediates the backward pass needs."""
    P = unflatten(theta, p)
    off, A, X = graph_batch(graphs)
    G = len(graphs)
    H = X
    cache = []
    for l in range(LAYERS):
        Hr = _r(H, bf16_ops)
        M = _r(A @ Hr, bf16_ops)          # messages from bf16 activations
        XC = np.concatenate([Hr, M], axis=1)
        W = _r(P[f"W{l}"], bf16_ops)
        Z = XC @ W.T + P[f"b{l}"]
        cache.append((XC, W, Z))
        H = np.maximum(Z, 0.0)
    g = np.stack([H[off[i]:off[i + 1]].mean(axis=0) if off[i + 1] > off[i] else np.zeros(HID)
                  for i in range(G)])
    gr = _r(g, bf16_ops)
    W1 = _r(P["Wh1"], bf16_ops)
    Z1 = gr @ W1.T + P["bh1"]
    A1 = _r(np.maximum(Z1, 0.0), bf16_ops)
    W2 = _r(P["Wh2"], bf16_ops)
    Y = A1 @ W2.T + P["bh2"]
    i = np.arange(1, p + 1) / p
    gamma = i[None, :] + Y[:, :p]
    beta = (1.0 - i)[None, :] + Y[:, p:]
    if keep:
        return gamma, beta, dict(off=off, A=A, cache=cache, g=gr, W1=W1, Z1=Z1, A1=A1, W2=W2)
    return gamma, beta


def loss_and_grad(theta: np.ndarray, graphs: Sequence, gamma_t, beta_t, p: int, bf16_ops: bool = False):
    """MSE loss and its gradient with respect to the flat parameters."""
    gamma, beta, c = forward(theta, graphs, p, bf16_ops, keep=True)
    G = len(graphs)
    D = np.concatenate([gamma - np.asarray(gamma_t), beta - np.asarray(beta_t)], axis=1)  # [G][2p]
    loss = float(np.mean(D * D))
    dY = 2.0 * D / D.size
    grads = {}
    dYr = _r(dY, bf16_ops)
    grads["Wh2"] = dYr.T @ c["A1"]
    grads["bh2"] = dY.sum(axis=0)
    dA1 = dYr @ c["W2"]
    dZ1 = dA1 * (c["Z1"] > 0)
    dZ1r = _r(dZ1, bf16_ops)
    grads["Wh1"] = dZ1r.T @ c["g"]
    grads["bh1"] = dZ1.sum(axis=0)
    dg = dZ1r @ c["W1"]
    off = c["off"]
    N = int(off[-1])
    dH = np.zeros((N, HID))
    for i in range(G):
        k = off[i + 1] - off[i]
        if k:
            dH[off[i]:off[i + 1]] = dg[i] / k
    A = c["A"]
    for l in reversed(range(LAYERS)):
        XC, W, Z = c["cache"][l]
        dZ = dH * (Z > 0)
        dZr = _r(dZ, bf16_ops)
        grads[f"W{l}"] = dZr.T @ XC
        grads[f"b{l}"] = dZ.sum(axis=0)
        if l == 0:
            break
        dXC = dZr @ W
        d = XC.shape[1] // 2
        dH = dXC[:, :d] + A.T @ dXC[:, d:]
    return loss, flatten(grads, p)


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam descent step (Kingma & Ba 2015, Algorithm 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
