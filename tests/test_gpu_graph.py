"""GPU parity of the network analysis (components, LCC, site percolation)
against the BFS oracle, exact."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tn():
    import paper_2112_06613_amd as tn
    return tn


@pytest.fixture(scope="module")
def ctx(tn):
    c = tn.Context(0)
    yield c
    c.close()


def test_components_small_graphs(tn, ctx):
    cases = [([[0, 1], [0, 2], [1, 4], [3, 4]], 5),
             ([[0, 1], [1, 2], [0, 2], [3, 4], [4, 5], [3, 5]], 7),
             (np.zeros((0, 2), np.uint32), 4),
             ([[3, 3], [2, 3], [3, 2]], 5)]
    for pairs, n in cases:
        got = tn.tcrnet_components(ctx, pairs, n)
        want = oracle.components(pairs, n)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
        assert got[2:] == want[2:]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_components_of_built_networks(tn, ctx, orc, k):
    s = synth.repertoire(30000, 3000, 70 + k)
    g = tn.tcrnet_build(ctx, s, k)
    got = tn.tcrnet_components(ctx, g.pairs, s.n)
    want = oracle.components(g.pairs, s.n)
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1], want[1])
    assert got[2:] == want[2:]


def test_paper_scale_components_and_robustness(tn, ctx):
    s = synth.paper_scale()
    g = tn.tcrnet_build(ctx, s, 1)
    got = tn.tcrnet_components(ctx, g.pairs, s.n)
    want = oracle.components(g.pairs, s.n)
    assert np.array_equal(got[0], want[0]) and got[2:] == want[2:]
    order = np.random.default_rng(20211215).permutation(s.n).astype(np.uint32)
    removed = (np.array([0.0, 0.01, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99, 1.0]) * s.n).round().astype(np.uint32)
    lcc = tn.tcrnet_robustness(ctx, g.pairs, s.n, order, removed)
    assert np.array_equal(lcc, oracle.robustness(g.pairs, s.n, order, removed))
    assert lcc[-1] == 0


def test_robustness_many_runs_in_chunks(tn, ctx):
    s = synth.repertoire(5000, 500, 3)
    g = tn.tcrnet_build(ctx, s, 2)
    order = np.random.default_rng(2).permutation(s.n).astype(np.uint32)
    removed = np.arange(0, s.n + 1, 50, dtype=np.uint32)
    lcc = tn.tcrnet_robustness(ctx, g.pairs, s.n, order, removed)
    assert np.array_equal(lcc, oracle.robustness(g.pairs, s.n, order, removed))


def test_analysis_argument_errors(tn, ctx):
    with pytest.raises(tn.TcrnetError):
        tn.tcrnet_components(ctx, [[0, 5]], 5)
    with pytest.raises(tn.TcrnetError):
        tn.tcrnet_robustness(ctx, [[0, 1]], 3, [0, 0, 1], [0])
    with pytest.raises(tn.TcrnetError):
        tn.tcrnet_robustness(ctx, [[0, 1]], 3, [0, 1, 2], [4])


def _stats_match(got, want):
    assert np.array_equal(got["degree"], want["degree"])
    assert got["max_degree"] == want["max_degree"]
    assert np.array_equal(got["count"], want["count"])
    assert np.array_equal(got["nbr_sum"], want["nbr_sum"])
    assert got["triangles"] == want["triangles"]
    # one division per node on both sides: identical doubles
    assert np.array_equal(got["clustering"], want["clustering"])
    # sums in different orders: agreement to rounding
    assert got["avg_clustering"] == pytest.approx(want["avg_clustering"], rel=1e-12, abs=1e-15)
    assert got["assortativity"] == pytest.approx(want["assortativity"], rel=1e-9, abs=1e-12)


def test_graph_stats_small(tn, ctx):
    for pairs, n in (([[0, 1], [0, 2], [1, 4], [3, 4]], 5), ([[0, 1], [0, 2], [1, 2]], 3),
                     (np.zeros((0, 2), np.uint32), 6)):
        _stats_match(tn.tcrnet_graph_stats(ctx, pairs, n), oracle.graph_stats(pairs, n))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_graph_stats_built_networks(tn, ctx, k):
    s = synth.repertoire(20000, 1000, 90 + k)
    g = tn.tcrnet_build(ctx, s, k)
    got = tn.tcrnet_graph_stats(ctx, g.pairs, s.n)
    _stats_match(got, oracle.graph_stats(g.pairs, s.n))
    assert np.array_equal(got["degree"], g.degree)


def test_graph_stats_paper_scale(tn, ctx):
    s = synth.paper_scale()
    g = tn.tcrnet_build(ctx, s, 1)
    got = tn.tcrnet_graph_stats(ctx, g.pairs, s.n)
    _stats_match(got, oracle.graph_stats(g.pairs, s.n))


def test_graph_stats_rejects_non_canonical(tn, ctx):
    with pytest.raises(tn.TcrnetError):
        tn.tcrnet_graph_stats(ctx, [[1, 0]], 3)
    with pytest.raises(tn.TcrnetError):
        tn.tcrnet_graph_stats(ctx, [[0, 2], [0, 1]], 3)
