"""Pins of the warm-start network's CPU oracle (oracle/mpnn.py) to facts that
do not depend on it: central finite differences of its own loss (the backward
pass), torch's bfloat16 conversion (the rounding), a closed form for zero
message-passing weights (the mean readout), the one-node recursion of a
vertex-transitive graph (the weighted aggregation), and invariances of the definition (vertex relabelling,
batch composition)."""
import numpy as np
import pytest

import qaoa_inputs as qi
from oracle import mpnn


def small_graphs(seed=0):
    return [qi.erdos_renyi(n, 0.6, seed=[seed, n], weights="uniform", wlow=-1, whigh=1) for n in (4, 5, 7)]


def targets(graphs, p, seed=1):
    rng = np.random.default_rng(seed)
    g, b = qi.linear_ramp(p)
    G = len(graphs)
    return np.tile(g, (G, 1)) + rng.normal(0, 0.2, (G, p)), np.tile(b, (G, 1)) + rng.normal(0, 0.2, (G, p))


def test_param_layout_matches_input_generator():
    for p in (1, 4, 8):
        assert mpnn.num_params(p) == qi.mpnn_init_params(p, 0).size
        assert [s for _, s in mpnn.dims(p)] == [s for _, s in qi.mpnn_param_shapes(p)]


def test_backward_matches_central_differences():
    p = 3
    graphs = small_graphs()
    gt, bt = targets(graphs, p)
    rng = np.random.default_rng(5)
    theta = qi.mpnn_init_params(p, 3) + rng.normal(0, 0.05, mpnn.num_params(p))
    L, grad = mpnn.loss_and_grad(theta, graphs, gt, bt, p)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mpnn.dims(p)])
    # coordinates from every parameter block, including the first layer's live columns
    idx = []
    for k in range(len(offs) - 1):
        idx += list(rng.integers(offs[k], offs[k + 1], 6))
    W0 = mpnn.unflatten(np.arange(mpnn.num_params(p), dtype=np.float64), p)["W0"]
    idx += [int(W0[r, c]) for r, c in [(0, 0), (5, 1), (9, 2), (17, 32), (40, 33), (77, 34)]]
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mpnn.loss_and_grad(theta + e, graphs, gt, bt, p)[0]
              - mpnn.loss_and_grad(theta - e, graphs, gt, bt, p)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 5000)]).astype(np.float32)
    # exact ties between two bfloat16 neighbours, both parities
    base = np.float32(1.0) + np.arange(8, dtype=np.float32) * np.float32(2.0 ** -7)
    ties = base + np.float32(2.0 ** -8)
    x = np.concatenate([x, ties, -ties])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mpnn.bf16(x), want)


def test_zero_message_weights_closed_form():
    """With every layer weight and the first head weight zero, each layer gives
    ReLU(b_l) at every node, so Y = W_2 ReLU(b_1) + b_2 for every graph."""
    p = 4
    graphs = small_graphs(2)
    P = mpnn.unflatten(qi.mpnn_init_params(p, 7), p)
    for l in range(3):
        P[f"W{l}"][:] = 0.0
    P["Wh1"][:] = 0.0
    theta = mpnn.flatten(P, p)
    gamma, beta = mpnn.forward(theta, graphs, p)
    Y = P["Wh2"] @ np.maximum(P["bh1"], 0.0) + P["bh2"]
    i = np.arange(1, p + 1) / p
    for gi in range(len(graphs)):
        np.testing.assert_allclose(gamma[gi], i + Y[:p], rtol=0, atol=1e-15)
        np.testing.assert_allclose(beta[gi], 1 - i + Y[p:], rtol=0, atol=1e-15)


def test_readout_is_the_node_mean():
    """With every message-passing weight zero each node ends layer 3 at
    ReLU(b_2), so the readout is ReLU(b_2) itself under mean pooling (n times
    it under sum pooling) and Y = W_h2 ReLU(W_h1 ReLU(b_2) + b_h1) + b_h2 for
    graphs of every size."""
    p = 3
    graphs = small_graphs(3) + [qi.MaxCut(n=1, edges=np.zeros((0, 2), np.int32), weights=None)]
    P = mpnn.unflatten(qi.mpnn_init_params(p, 17), p)
    for l in range(3):
        P[f"W{l}"][:] = 0.0
    rng = np.random.default_rng(4)
    P["b2"] = rng.normal(0, 0.5, P["b2"].shape)   # about half the units active
    theta = mpnn.flatten(P, p)
    gamma, beta = mpnn.forward(theta, graphs, p)
    g = np.maximum(P["b2"], 0.0)
    Y = P["Wh2"] @ np.maximum(P["Wh1"] @ g + P["bh1"], 0.0) + P["bh2"]
    i = np.arange(1, p + 1) / p
    for gi in range(len(graphs)):
        np.testing.assert_allclose(gamma[gi], i + Y[:p], rtol=0, atol=1e-13)
        np.testing.assert_allclose(beta[gi], 1 - i + Y[p:], rtol=0, atol=1e-13)


def test_vertex_transitive_graph_reduces_to_one_node():
    """On a cycle C_n with one weight w on every edge all nodes are alike, so
    H stays equal across nodes and (A H)_v = 2 w h: each layer is the
    one-vector recursion h' = ReLU(W_self h + 2 w W_msg h + b), with the input
    x = (2/8, 2w/8, 1, 2w^2/8, 0, ...).  This pins the weighted, symmetric
    aggregation and the split of W_l into its self and message halves."""
    p = 2
    P = mpnn.unflatten(qi.mpnn_init_params(p, 23), p)
    theta = mpnn.flatten(P, p)
    for n, w in ((5, 0.7), (8, -0.4)):
        e = np.array([[k, (k + 1) % n] for k in range(n)], dtype=np.int32)
        cyc = qi.MaxCut(n=n, edges=e, weights=np.full(n, w))
        gamma, beta = mpnn.forward(theta, [cyc], p)
        h = np.zeros(mpnn.FIN)
        h[:4] = (2 / 8, 2 * w / 8, 1.0, 2 * w * w / 8)
        for l in range(3):
            W = P[f"W{l}"]
            d = W.shape[1] // 2
            h = np.maximum(W[:, :d] @ h + 2 * w * (W[:, d:] @ h) + P[f"b{l}"], 0.0)
        Y = P["Wh2"] @ np.maximum(P["Wh1"] @ h + P["bh1"], 0.0) + P["bh2"]
        i = np.arange(1, p + 1) / p
        np.testing.assert_allclose(gamma[0], i + Y[:p], rtol=0, atol=1e-12)
        np.testing.assert_allclose(beta[0], 1 - i + Y[p:], rtol=0, atol=1e-12)


@pytest.mark.parametrize("bf16_ops", [False, True])
def test_vertex_relabelling_and_batch_composition(bf16_ops):
    p = 2
    graphs = small_graphs(4)
    theta = qi.mpnn_init_params(p, 11)
    g_all, b_all = mpnn.forward(theta, graphs, p, bf16_ops)
    rng = np.random.default_rng(9)
    relabelled = []
    for g in graphs:
        perm = rng.permutation(g.n)
        e = perm[np.asarray(g.edges)]
        relabelled.append(qi.MaxCut(n=g.n, edges=e.astype(np.int32), weights=g.weights))
    g_rel, b_rel = mpnn.forward(theta, relabelled, p, bf16_ops)
    tol = 1e-12 if not bf16_ops else 1e-6
    np.testing.assert_allclose(g_rel, g_all, rtol=0, atol=tol)
    np.testing.assert_allclose(b_rel, b_all, rtol=0, atol=tol)
    for k, g in enumerate(graphs):
        g1, b1 = mpnn.forward(theta, [g], p, bf16_ops)
        np.testing.assert_allclose(g1[0], g_all[k], rtol=0, atol=1e-12)
        np.testing.assert_allclose(b1[0], b_all[k], rtol=0, atol=1e-12)


def test_bf16_operands_change_results_only_slightly():
    p = 8
    graphs = small_graphs(6)
    gt, bt = targets(graphs, p, 2)
    theta = qi.mpnn_init_params(p, 13)
    L0, g0 = mpnn.loss_and_grad(theta, graphs, gt, bt, p)
    L1, g1 = mpnn.loss_and_grad(theta, graphs, gt, bt, p, bf16_ops=True)
    assert abs(L1 - L0) <= 2e-2 * L0
    assert np.linalg.norm(g1 - g0) <= 3e-2 * np.linalg.norm(g0)


def test_adam_step_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    th = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    tt = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-3)
    for t in range(1, 6):
        g = rng.normal(size=50)
        th, m, v = mpnn.adam_step(th, g, m, v, t, 1e-3)
        opt.zero_grad()
        tt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(th, tt.detach().numpy(), rtol=0, atol=1e-13)
