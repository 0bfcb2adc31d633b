"""Host-side logic of the warm-start pipeline and the batched-engine tuner
(no GPU): evaluation counting, ramp angles, dataset round trip, cache keys."""
import numpy as np

import qaoa_inputs as qi
from paper_2407_13012_amd import batch_tune as bt
from paper_2407_13012_amd import warmstart as ws


def test_evals_to_reach_counts_first_hit_of_running_best():
    tr = np.array([1.0, 3.0, 2.0, 5.0, 4.0])
    assert ws.evals_to_reach(tr, 3.0) == 2
    assert ws.evals_to_reach(tr, 4.5) == 4
    assert ws.evals_to_reach(tr, 0.5) == 1
    assert ws.evals_to_reach(tr, 6.0) is None


def test_ramp_angles_match_input_generator():
    g, b = bt.ramp_angles(3, 5)
    rg, rb = qi.linear_ramp(5)
    np.testing.assert_array_equal(g, np.tile(rg, (3, 1)))
    np.testing.assert_array_equal(b, np.tile(rb, (3, 1)))


def test_dataset_round_trip(tmp_path):
    graphs = qi.batched_family(5)
    p = 3
    rng = np.random.default_rng(0)
    gam, bet = rng.normal(size=(5, p)), rng.normal(size=(5, p))
    e0, e1, cm = rng.normal(size=5), rng.normal(size=5), rng.normal(size=5)
    path = str(tmp_path / "d.npz")
    bt.save_dataset(path, graphs, p, gam, bet, e0, e1, cm, meta={"steps": 7})
    d = bt.load_dataset(path)
    assert d["meta"] == {"steps": 7} and int(d["p"]) == p
    np.testing.assert_array_equal(d["gamma"], gam)
    back = ws.graphs_of(d)
    for g, h in zip(graphs, back):
        assert g.n == h.n
        np.testing.assert_array_equal(np.asarray(g.edges), h.edges)
        np.testing.assert_array_equal(g.weight_array(), h.weight_array())


def test_batch_key_is_size_histogram():
    graphs = [qi.MaxCut(n=n, edges=np.zeros((0, 2), np.int32), weights=None) for n in (12, 10, 12)]
    assert bt.batch_key(graphs, 4) == "p4;10:1,12:2"


def test_warmstart_eval_graphs_are_seeded_er24():
    gs = qi.warmstart_eval_graphs(3)
    assert [g.n for g in gs] == [24, 24, 24]
    again = qi.warmstart_eval_graphs(3)
    for a, b in zip(gs, again):
        np.testing.assert_array_equal(a.edges, b.edges)
        np.testing.assert_array_equal(a.weights, b.weights)
    assert np.all(np.abs(gs[0].weights) <= 1.0)
