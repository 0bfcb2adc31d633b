"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test compares the oracle with something fixed by the paper or by
mathematics: hand-derived fixtures, closed forms from the QAOA literature,
dense matrix exponentials (scipy) on tiny systems, invariants, finite
differences and exact parameter-shift rules.  Every one is chosen so that a
plausible slip in the oracle (dropped term, wrong sign, swapped operand, wrong
qubit index) fails it.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import qaoa_inputs as qi

pytestmark = pytest.mark.filterwarnings("ignore")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ helpers (tests only)

def bits(n):
    z = np.arange(1 << n, dtype=np.uint64)
    return [((z >> np.uint64(i)) & np.uint64(1)).astype(np.int64) for i in range(n)]


def dense_mixer(n, beta):
    """exp(-i beta sum_j X_j) as a dense 2^n x 2^n matrix via scipy's expm of the
    full mixer Hamiltonian (independent of any per-qubit butterfly)."""
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for j in range(n):
        # qubit j is bit j of the index: kron order puts qubit n-1 leftmost
        op = np.array([[1.0]], dtype=np.complex128)
        for q in reversed(range(n)):
            op = np.kron(op, X if q == j else np.eye(2))
        H += op
    return scipy.linalg.expm(-1j * beta * H)


def dense_state(n, C, gamma, beta):
    psi = np.full(1 << n, 1 / math.sqrt(1 << n), dtype=np.complex128)
    for g, b in zip(gamma, beta):
        psi = np.exp(-1j * g * C) * psi
        psi = dense_mixer(n, b) @ psi
    return psi


def rx2(b):
    return scipy.linalg.expm(-1j * b * np.array([[0, 1], [1, 0]], dtype=np.complex128))


def single_qubit_linear_E(hval, gamma, beta):
    """E of f = h*x on one qubit, any depth, with 2x2 library matrix exponentials."""
    v = np.array([1, 1], dtype=np.complex128) / math.sqrt(2)
    for g, b in zip(gamma, beta):
        v = np.array([1, np.exp(-1j * g * hval)]) * v
        v = rx2(b) @ v
    return hval * abs(v[1]) ** 2


def rand_graph(n, p_edge, seed, weights="unit"):
    return qi.erdos_renyi(n, p_edge, seed, weights=weights, wlow=-1.0, whigh=1.0)


# ------------------------------------------------------------------ Philox

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_uniform53_range_and_counter_dependence():
    us = np.array([oracle.uniform53(7, s) for s in range(4096)])
    assert np.all(us >= 0) and np.all(us < 1)
    assert len(np.unique(us)) == us.size
    # mean/variance of U[0,1) within 5 sigma
    assert abs(us.mean() - 0.5) < 5 * math.sqrt(1 / 12 / us.size)
    assert oracle.uniform53(7, 3) != oracle.uniform53(8, 3)


# ------------------------------------------------------------------ cost diagonal

def _gold_cost():
    out = []
    for l in open(os.path.join(GOLD, "cost_small.txt")):
        if not l.strip() or l.startswith("#"):
            continue
        kind, name, n, terms, vals = [s.strip() for s in l.split("|")]
        out.append((kind, name, int(n), terms.split(), np.array([float(v) for v in vals.split()])))
    return out


@pytest.mark.parametrize("case", _gold_cost(), ids=lambda c: c[1])
def test_cost_golden(case):
    kind, _, n, terms, want = case
    if kind == "maxcut":
        e, w = [], []
        for t in terms:
            ij, wv = t.split(":")
            e.append([int(x) for x in ij.split("-")])
            w.append(float(wv))
        got = oracle.cost_maxcut(n, np.array(e), np.array(w))
    elif kind == "qubo":
        off, pairs, J, h = 0.0, [], [], np.zeros(n)
        for t in terms:
            k, v = t.split(":")
            if k == "off":
                off = float(v)
            elif k.startswith("h"):
                h[int(k[1:])] = float(v)
            else:
                pairs.append([int(x) for x in k.split("-")])
                J.append(float(v))
        got = oracle.cost_qubo(n, np.array(pairs), np.array(J), h, off)
    else:
        masks, w = [], []
        for t in terms:
            k, v = t.split(":")
            masks.append(int(k[1:]))
            w.append(float(v))
        got = oracle.cost_poly(n, np.array(masks, dtype=np.uint64), np.array(w))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [2, 5, 9])
def test_cost_complete_graph_closed_form(n):
    # K_n, unit weights: C(z) = k (n - k) with k = popcount(z)
    g = qi.complete_graph(n)
    C = oracle.cost_maxcut(n, g.edges)
    k = np.array([bin(z).count("1") for z in range(1 << n)])
    assert np.array_equal(C, (k * (n - k)).astype(float))


def test_cost_even_cycle_bipartite():
    n = 8
    e = np.array([[i, (i + 1) % n] for i in range(n)])
    e = np.sort(e, axis=1)
    C = oracle.cost_maxcut(n, e)
    alt = sum(1 << i for i in range(0, n, 2))
    assert C[alt] == n and C.max() == n and C[0] == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cost_maxcut_invariants(seed):
    n = 10
    g = rand_graph(n, 0.4, seed, weights="uniform")
    C = oracle.cost_maxcut(n, g.edges, g.weights)
    N = 1 << n
    assert C[0] == 0.0
    # complement symmetry C(z) == C(~z)
    assert np.array_equal(C, C[::-1])
    # mean over z of each cut indicator is 1/2
    assert abs(C.mean() - g.weights.sum() / 2) < 1e-12 * max(1, abs(g.weights).sum())
    # single flipped vertex cuts exactly its incident edges
    for v in range(n):
        inc = sum(w for (a, b), w in zip(g.edges, g.weights) if v in (a, b))
        assert abs(C[1 << v] - inc) < 1e-12
    assert N == C.size


@pytest.mark.parametrize("seed", [0, 5])
def test_cost_qubo_invariants(seed):
    n = 9
    q = qi.qubo_erdos_renyi(n, 0.5, seed, offset=0.25)
    C = oracle.cost_qubo(n, q.pairs, q.J, q.h, q.offset)
    assert C[0] == q.offset
    for i in range(n):
        assert abs(C[1 << i] - (q.offset + q.h[i])) < 1e-14
    for (i, j), Jij in zip(q.pairs, q.J):
        assert abs(C[(1 << i) | (1 << j)] - (q.offset + q.h[i] + q.h[j] + Jij)) < 1e-13
    assert abs(C[-1] - (q.offset + q.J.sum() + q.h.sum())) < 1e-12
    # mean: pair terms average 1/4, linear terms 1/2
    assert abs(C.mean() - (q.offset + q.J.sum() / 4 + q.h.sum() / 2)) < 1e-12


def test_cost_entry_matches_full():
    g = rand_graph(11, 0.5, 3, weights="uniform")
    C = oracle.cost_maxcut(11, g.edges, g.weights)
    for z in [0, 1, 77, 1023, 2047]:
        assert oracle.cost_maxcut_entry(z, g.edges, g.weights) == C[z]
    q = qi.qubo_erdos_renyi(11, 0.3, 4)
    Cq = oracle.cost_qubo(11, q.pairs, q.J, q.h)
    for z in [0, 5, 999, 2047]:
        assert oracle.cost_qubo_entry(z, 11, q.pairs, q.J, q.h) == Cq[z]


def test_cost_poly_reduces_to_qubo():
    n = 6
    q = qi.qubo_erdos_renyi(n, 0.6, 9)
    masks = [(1 << int(i)) | (1 << int(j)) for i, j in q.pairs] + [1 << i for i in range(n)]
    w = np.concatenate([q.J, q.h])
    Cp = oracle.cost_poly(n, np.array(masks, dtype=np.uint64), w)
    Cq = oracle.cost_qubo(n, q.pairs, q.J, q.h)
    # same terms, same order -> identical sums
    assert np.array_equal(Cp, Cq)


# ------------------------------------------------------------------ evolution

def test_initial_state_and_p0():
    n = 7
    psi = oracle.init_plus(n)
    assert np.allclose(psi, 2 ** (-n / 2), rtol=0, atol=1e-16)
    g = rand_graph(n, 0.5, 1)
    C = oracle.cost_maxcut(n, g.edges)
    E = oracle.expectation(n, C, oracle.state(n, C, [], []))
    assert abs(E - g.m / 2) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_state_matches_dense_expm(seed):
    """Brute force: dense exp(-i beta sum X) from scipy against per-qubit butterflies."""
    n = 5
    g = rand_graph(n, 0.6, seed, weights="uniform")
    C = oracle.cost_maxcut(n, g.edges, g.weights)
    gamma, beta = qi.uniform_angles(3, seed=[seed, 9])
    got = oracle.state(n, C, gamma, beta)
    want = dense_state(n, C, gamma, beta)
    assert np.max(np.abs(got - want)) < 1e-13


def test_mixer_sign_pin():
    """f = sum_i x_i, gamma = pi/2, beta = pi/4: exp(-i beta X) sends every qubit
    to -i|1>, so psi = (-i)^n |1...1> and E = n.  With the opposite mixer sign the
    state would be |0...0> and E = 0."""
    n = 6
    C = oracle.cost_qubo(n, np.zeros((0, 2)), np.zeros(0), np.ones(n))
    psi = oracle.state(n, C, [math.pi / 2], [math.pi / 4])
    want = np.zeros(1 << n, dtype=np.complex128)
    want[-1] = (-1j) ** n
    assert np.max(np.abs(psi - want)) < 1e-15
    assert abs(oracle.expectation(n, C, psi) - n) < 1e-14


def test_single_edge_closed_form():
    # one edge of weight w: E = w (1/2 + 1/2 sin(4 beta) sin(gamma w))
    for (gm, bt, w) in [(0.3, 0.2, 1.0), (1.7, -0.4, 0.37), (2.9, 1.1, 2.5)]:
        C = oracle.cost_maxcut(2, np.array([[0, 1]]), np.array([w]))
        E = oracle.expectation(2, C, oracle.state(2, C, [gm], [bt]))
        assert abs(E - w * (0.5 + 0.5 * math.sin(4 * bt) * math.sin(gm * w))) < 1e-14


def wang_p1_unweighted(n, edges, gamma, beta):
    """<C> at p=1 for unweighted MaxCut (Wang, Hadfield, Jiang, Rieffel, PRA 97,
    022304 (2018)): per edge uv with d = deg u - 1, e = deg v - 1 and f common
    neighbours, 1/2 + 1/4 sin4b sing (cos^d g + cos^e g)
    - 1/4 sin^2 2b cos^(d+e-2f) g (1 - cos^f 2g)."""
    nb = [set() for _ in range(n)]
    for a, b in edges:
        nb[a].add(b)
        nb[b].add(a)
    tot = 0.0
    cg, sg = math.cos(gamma), math.sin(gamma)
    for a, b in edges:
        d, e, f = len(nb[a]) - 1, len(nb[b]) - 1, len(nb[a] & nb[b])
        tot += (0.5 + 0.25 * math.sin(4 * beta) * sg * (cg ** d + cg ** e)
                - 0.25 * math.sin(2 * beta) ** 2 * cg ** (d + e - 2 * f) * (1 - math.cos(2 * gamma) ** f))
    return tot


def wang_p1_weighted(n, edges, w, gamma, beta):
    """Weighted generalisation of the p=1 edge formula (products of cosines over
    the neighbourhoods, difference/sum terms over common neighbours)."""
    W = {}
    nb = [set() for _ in range(n)]
    for (a, b), x in zip(edges, w):
        W[(a, b)] = W[(b, a)] = x
        nb[a].add(b)
        nb[b].add(a)
    tot = 0.0
    for (u, v), wuv in zip(edges, w):
        pu = np.prod([math.cos(gamma * W[(u, k)]) for k in nb[u] - {v}])
        pv = np.prod([math.cos(gamma * W[(v, k)]) for k in nb[v] - {u}])
        common = nb[u] & nb[v]
        ou = np.prod([math.cos(gamma * W[(u, k)]) for k in nb[u] - nb[v] - {v}])
        ov = np.prod([math.cos(gamma * W[(v, k)]) for k in nb[v] - nb[u] - {u}])
        cm = np.prod([math.cos(gamma * (W[(u, k)] - W[(v, k)])) for k in common])
        cp = np.prod([math.cos(gamma * (W[(u, k)] + W[(v, k)])) for k in common])
        tot += wuv * (0.5 + 0.25 * math.sin(4 * beta) * math.sin(gamma * wuv) * (pu + pv)
                      - 0.25 * math.sin(2 * beta) ** 2 * ou * ov * (cm - cp))
    return tot


@pytest.mark.parametrize("seed", range(5))
def test_p1_unweighted_closed_form(seed):
    n = 10
    g = rand_graph(n, 0.45, 100 + seed)
    C = oracle.cost_maxcut(n, g.edges)
    gm, bt = qi.uniform_angles(1, seed=[seed, 3])
    E = oracle.expectation(n, C, oracle.state(n, C, gm, bt))
    assert abs(E - wang_p1_unweighted(n, g.edges.tolist(), gm[0], bt[0])) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_p1_weighted_closed_form(seed):
    n = 9
    g = rand_graph(n, 0.5, 200 + seed, weights="uniform")
    C = oracle.cost_maxcut(n, g.edges, g.weights)
    gm, bt = qi.uniform_angles(1, seed=[seed, 4])
    E = oracle.expectation(n, C, oracle.state(n, C, gm, bt))
    assert abs(E - wang_p1_weighted(n, g.edges.tolist(), g.weights, gm[0], bt[0])) < 1e-12


@pytest.mark.parametrize("p", [1, 3])
def test_linear_cost_product_state(p):
    """f = sum h_i x_i: the state is a product state, so E is the sum of
    single-qubit expectations (2x2 library exponentials)."""
    n = 8
    h = np.random.default_rng(p).normal(size=n)
    C = oracle.cost_qubo(n, np.zeros((0, 2)), np.zeros(0), h)
    gamma, beta = qi.ramp_with_noise(p, seed=[p, 2])
    E = oracle.expectation(n, C, oracle.state(n, C, gamma, beta))
    want = sum(single_qubit_linear_E(hv, gamma, beta) for hv in h)
    assert abs(E - want) < 1e-13
    if p == 1:
        closed = sum(hv * 0.5 * (1 + math.sin(2 * beta[0]) * math.sin(gamma[0] * hv)) for hv in h)
        assert abs(E - closed) < 1e-13


def test_invariants():
    n = 9
    g = rand_graph(n, 0.5, 11, weights="integer")
    g.weights = np.abs(g.weights) + 1
    C = oracle.cost_maxcut(n, g.edges, g.weights)
    gamma, beta = qi.uniform_angles(3, seed=[5, 5])

    def E(gm, bt):
        return oracle.expectation(n, C, oracle.state(n, C, gm, bt))

    e0 = E(gamma, beta)
    psi = oracle.state(n, C, gamma, beta)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13
    assert C.min() - 1e-12 <= e0 <= C.max() + 1e-12
    assert abs(E(-gamma, -beta) - e0) < 1e-12                   # time reversal + conjugation
    assert abs(E(gamma, beta + math.pi / 2) - e0) < 1e-12       # MaxCut: beta period pi/2
    assert abs(E(gamma + 2 * math.pi, beta) - e0) < 1e-11       # integer weights: gamma period 2 pi
    assert abs(E(np.zeros(3), beta) - C.mean()) < 1e-12         # no phase: |+> is a mixer eigenstate
    assert abs(E(gamma, np.zeros(3)) - C.mean()) < 1e-12        # no mixing: phases only


# ------------------------------------------------------------------ gradient

@pytest.mark.parametrize("seed,n,p", [(0, 6, 1), (1, 7, 2), (2, 8, 3)])
def test_gradient_finite_differences(seed, n, p):
    g = rand_graph(n, 0.5, 300 + seed, weights="uniform")
    C = oracle.cost_maxcut(n, g.edges, g.weights)
    gamma, beta = qi.uniform_angles(p, seed=[seed, 7])
    E, dg, db = oracle.gradient(n, C, gamma, beta)
    assert abs(E - oracle.expectation(n, C, oracle.state(n, C, gamma, beta))) < 1e-13
    h = 1e-5

    def f(gm, bt):
        return oracle.expectation(n, C, oracle.state(n, C, gm, bt))

    for l in range(p):
        e = np.zeros(p)
        e[l] = h
        fd_g = (f(gamma + e, beta) - f(gamma - e, beta)) / (2 * h)
        fd_b = (f(gamma, beta + e) - f(gamma, beta - e)) / (2 * h)
        assert abs(dg[l] - fd_g) < 1e-8
        assert abs(db[l] - fd_b) < 1e-8


def _state_general(n, edges, w, gam_edges, bet_qubits):
    """QAOA with one angle per edge (phase) and one per qubit (mixer) per layer;
    dense, for parameter-shift pins on tiny systems."""
    B = bits(n)
    psi = np.full(1 << n, 1 / math.sqrt(1 << n), dtype=np.complex128)
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    for ge, bq in zip(gam_edges, bet_qubits):
        for (a, b), we, gk in zip(edges, w, ge):
            cut = (B[a] ^ B[b]).astype(float)
            psi = np.exp(-1j * gk * we * cut) * psi
        for j in range(n):
            U = scipy.linalg.expm(-1j * bq[j] * X)
            t = psi.reshape(1 << (n - j - 1), 2, 1 << j)
            psi = np.einsum("ab,xbz->xaz", U, t).reshape(-1)
    return psi


def test_gradient_parameter_shift_exact():
    """Exact parameter-shift rules on a circuit with one angle per gate:
    dE/dbeta_l = sum_j [E(beta_lj + pi/4) - E(beta_lj - pi/4)] (generator X_j);
    dE/dgamma_l = sum_e w_e/2 [E(gamma_le + pi/(2 w_e)) - E(gamma_le - pi/(2 w_e))]
    (generator w_e cut_e with eigenvalues 0, w_e)."""
    n, p = 5, 2
    g = rand_graph(n, 0.7, 42, weights="uniform")
    edges, w = g.edges.tolist(), np.abs(g.weights) + 0.2
    C = oracle.cost_maxcut(n, g.edges, w)
    gamma, beta = qi.uniform_angles(p, seed=[42, 1])
    E, dg, db = oracle.gradient(n, C, gamma, beta)

    def Eg(ge, bq):
        psi = _state_general(n, edges, w, ge, bq)
        return float(np.real(np.vdot(psi, C * psi)))

    ge0 = [np.full(len(edges), gm) for gm in gamma]
    bq0 = [np.full(n, bt) for bt in beta]
    assert abs(Eg(ge0, bq0) - E) < 1e-13
    for l in range(p):
        sb = 0.0
        for j in range(n):
            up = [x.copy() for x in bq0]; up[l][j] += math.pi / 4
            dn = [x.copy() for x in bq0]; dn[l][j] -= math.pi / 4
            sb += Eg(ge0, up) - Eg(ge0, dn)
        sg = 0.0
        for k in range(len(edges)):
            up = [x.copy() for x in ge0]; up[l][k] += math.pi / (2 * w[k])
            dn = [x.copy() for x in ge0]; dn[l][k] -= math.pi / (2 * w[k])
            sg += w[k] / 2 * (Eg(up, bq0) - Eg(dn, bq0))
        assert abs(db[l] - sb) < 1e-12
        assert abs(dg[l] - sg) < 1e-12


def test_gradient_zero_at_origin_and_product_state():
    n = 6
    g = rand_graph(n, 0.5, 8)
    C = oracle.cost_maxcut(n, g.edges)
    E, dg, db = oracle.gradient(n, C, np.zeros(2), np.zeros(2))
    assert abs(E - C.mean()) < 1e-13 and np.max(np.abs(dg)) < 1e-14 and np.max(np.abs(db)) < 1e-14
    # product state, p = 1: E = sum h/2 (1 + sin 2b sin(g h))
    h = np.random.default_rng(3).normal(size=n)
    C = oracle.cost_qubo(n, np.zeros((0, 2)), np.zeros(0), h)
    gm, bt = 0.7, 0.3
    E, dg, db = oracle.gradient(n, C, [gm], [bt])
    assert abs(dg[0] - sum(0.5 * hv * hv * math.sin(2 * bt) * math.cos(gm * hv) for hv in h)) < 1e-13
    assert abs(db[0] - sum(hv * math.cos(2 * bt) * math.sin(gm * hv) for hv in h)) < 1e-13


# ------------------------------------------------------------------ sampling

def test_sample_deterministic_state():
    n = 7
    C = oracle.cost_qubo(n, np.zeros((0, 2)), np.zeros(0), np.ones(n))
    psi = oracle.state(n, C, [math.pi / 2], [math.pi / 4])
    z, c = oracle.sample(n, psi, C, 500, seed=3)
    assert np.all(z == (1 << n) - 1) and np.all(c == n)


def test_sample_never_returns_zero_probability():
    n = 6
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[[3, 17, 40, 63]] = [0.5, 0.5j, -0.5, 0.5]
    z, _ = oracle.sample(n, psi, None, 4000, seed=1)
    assert set(z.tolist()) <= {3, 17, 40, 63}
    counts = np.bincount(z.astype(np.int64), minlength=1 << n)[[3, 17, 40, 63]]
    assert np.all(np.abs(counts - 1000) < 5 * math.sqrt(1000 * 0.75))


def chi2_pvalue(counts, probs):
    import scipy.stats
    exp = probs * counts.sum()
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] < 5:
        obs[-2] += obs[-1]; ex[-2] += ex[-1]
        obs, ex = obs[:-1], ex[:-1]
    stat = ((obs - ex) ** 2 / ex).sum()
    return scipy.stats.chi2.sf(stat, len(ex) - 1)


def test_sample_chi_square():
    n = 8
    g = rand_graph(n, 0.5, 21, weights="uniform")
    C = oracle.cost_maxcut(n, g.edges, g.weights)
    psi = oracle.state(n, C, [0.8, 0.3], [0.5, 0.2])
    z, c = oracle.sample(n, psi, C, 200000, seed=9)
    probs = np.abs(psi) ** 2
    assert chi2_pvalue(np.bincount(z.astype(np.int64), minlength=1 << n), probs) > 1e-3
    assert np.array_equal(c, C[z.astype(np.int64)])
    # gamma = 0: uniform distribution
    psi0 = oracle.state(n, C, [0.0], [0.4])
    z0, _ = oracle.sample(n, psi0, C, 100000, seed=2)
    assert chi2_pvalue(np.bincount(z0.astype(np.int64), minlength=1 << n), np.full(1 << n, 1 / (1 << n))) > 1e-3


def test_sample_inverse_cdf_definition():
    """Shot s lands on the first z whose cumulative mass exceeds u_s * T."""
    n = 5
    rng = np.random.default_rng(0)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    z, _ = oracle.sample(n, psi, None, 64, seed=77)
    cdf = np.cumsum(np.abs(psi) ** 2)
    for s in range(64):
        t = oracle.uniform53(77, s) * cdf[-1]
        k = int(z[s])
        assert cdf[k] > t * (1 - 1e-14)
        assert k == 0 or cdf[k - 1] <= t * (1 + 1e-14)


# ---------------------------------------------------------------- Adam loop of the batched optimiser

def test_adam_constant_gradient_closed_form():
    """With a constant gradient c the bias-corrected moments are c and c^2, so
    every step moves by lr * c / (|c| + eps)."""
    c = np.array([0.3, -2.0, 1e-3])
    lr, eps = 0.05, 1e-8
    x, f0, f1 = oracle.adam_ascent(lambda x: (float(c @ x), c), np.zeros(3), 7, lr, 0.9, 0.999, eps)
    np.testing.assert_allclose(x, 7 * lr * c / (np.abs(c) + eps), rtol=1e-12, atol=0)
    assert f0 == 0.0 and f1 == pytest.approx(float(c @ x), abs=1e-15)


def test_adam_matches_torch_optimizer():
    """Ascent on f equals torch.optim.Adam's descent on -f (float64, CPU)."""
    import torch
    A = np.array([[2.0, 0.5, 0.0], [0.5, 1.0, -0.3], [0.0, -0.3, 0.7]])
    b = np.array([0.2, -1.0, 0.4])

    def f(x):
        return float(-0.5 * x @ A @ x + b @ x), -A @ x + b

    x0 = np.array([0.1, 0.2, -0.3])
    x, _, _ = oracle.adam_ascent(f, x0, 25, 0.05, 0.9, 0.999, 1e-8)
    xt = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([xt], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    At, bt = torch.tensor(A), torch.tensor(b)
    for _ in range(25):
        opt.zero_grad()
        loss = -(-0.5 * xt @ At @ xt + bt @ xt)
        loss.backward()
        opt.step()
    np.testing.assert_allclose(x, xt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_qaoa_increases_expectation_and_scales():
    """Adam on the p=1 MaxCut expectation climbs; the objective scale does not
    change the first step (Adam is invariant to a constant gradient scale up to eps)."""
    g = qi.erdos_renyi(8, 0.5, seed=11, weights="uniform", wlow=-1, whigh=1)
    C = oracle.cost_of(g)
    gm, bt, e0, e1 = oracle.adam_qaoa(8, C, [0.2], [0.3], steps=30)
    assert e1 > e0
    g1, b1, _, _ = oracle.adam_qaoa(8, C, [0.2], [0.3], steps=1, scale=1.0)
    g2, b2, _, _ = oracle.adam_qaoa(8, C, [0.2], [0.3], steps=1, scale=0.125)
    np.testing.assert_allclose(np.r_[g1, b1], np.r_[g2, b2], rtol=0, atol=1e-7)
    np.testing.assert_allclose(np.abs(np.r_[g1 - 0.2, b1 - 0.3]), 0.05, rtol=0, atol=1e-6)
