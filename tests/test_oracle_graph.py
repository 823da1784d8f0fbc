"""Pins of the network-analysis oracle (components, LCC, site percolation)
against networkx (an independent implementation) and hand-worked graphs."""
import networkx as nx
import numpy as np
import pytest

import oracle
import synth


def _nx_graph(pairs, n):
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(map(tuple, np.asarray(pairs).reshape(-1, 2).tolist()))
    return G


def _nx_labels(G, n):
    lab = np.zeros(n, dtype=np.uint32)
    for comp in nx.connected_components(G):
        m = min(comp)
        for v in comp:
            lab[v] = m
    return lab


def test_paper_adjacency_example_is_one_component():
    # Methods, "Adjacency matrix": E = {(1,2),(1,3),(2,5),(4,5)} (1-based)
    labels, sizes, nc, lcc = oracle.components([[0, 1], [0, 2], [1, 4], [3, 4]], 5)
    assert labels.tolist() == [0] * 5 and nc == 1 and lcc == 5 and sizes[0] == 5


def test_hand_examples():
    # two triangles and an isolated node
    pairs = [[0, 1], [1, 2], [0, 2], [3, 4], [4, 5], [3, 5]]
    labels, sizes, nc, lcc = oracle.components(pairs, 7)
    assert labels.tolist() == [0, 0, 0, 3, 3, 3, 6]
    assert nc == 3 and lcc == 3 and sizes.tolist() == [3, 0, 0, 3, 0, 0, 1]
    # no edges
    labels, sizes, nc, lcc = oracle.components(np.zeros((0, 2), np.uint32), 4)
    assert labels.tolist() == [0, 1, 2, 3] and nc == 4 and lcc == 1
    assert oracle.components(np.zeros((0, 2), np.uint32), 0)[2:] == (0, 0)
    # a path 0-1-...-9 with node 5 removed splits into 5 and 4
    path = [[i, i + 1] for i in range(9)]
    assert oracle.robustness(path, 10, [5, 0, 1, 2, 3, 4, 6, 7, 8, 9], [0, 1, 2, 10]).tolist() == [10, 5, 4, 0]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_components_against_networkx(seed):
    rng = np.random.default_rng(seed)
    n = 300
    G = nx.gnp_random_graph(n, 1.2 / n, seed=seed)
    pairs = np.array(list(G.edges()), dtype=np.uint32).reshape(-1, 2)
    # duplicates and reversed copies change nothing
    pairs = np.concatenate([pairs, pairs[:, ::-1][: len(pairs) // 3]])
    labels, sizes, nc, lcc = oracle.components(pairs, n)
    assert np.array_equal(labels, _nx_labels(G, n))
    assert nc == nx.number_connected_components(G)
    assert lcc == max(len(c) for c in nx.connected_components(G))
    want = np.zeros(n, dtype=np.uint32)
    for c in nx.connected_components(G):
        want[min(c)] = len(c)
    assert np.array_equal(sizes, want)


def test_robustness_against_networkx():
    s = synth.repertoire(1500, 150, 8)
    e, _ = oracle.Oracle().build(s, 2)
    n = s.n
    G = _nx_graph(e, n)
    order = np.random.default_rng(4).permutation(n).astype(np.uint32)
    removed = [0, 15, 150, 750, 1350, 1499, 1500]
    got = oracle.robustness(e, n, order, removed)
    for r, g in zip(removed, got):
        H = G.subgraph(set(range(n)) - set(order[:r].tolist()))
        want = max((len(c) for c in nx.connected_components(H)), default=0)
        assert g == want


def test_lcc_normalisations():
    # Methods, "Computing LCC": norm1 = LCC(p) / ((1-p) N), norm2 = norm1(p) / norm1(0)
    n = 100
    lcc = [80, 60, 10]
    removed = [0, 20, 90]
    assert np.allclose(oracle.lcc_norm1(lcc, removed, n), [0.8, 0.75, 1.0])
    assert np.allclose(oracle.lcc_norm2(lcc, removed, n), [1.0, 0.75 / 0.8, 1.0 / 0.8])


@pytest.mark.parametrize("seed", [4, 5])
def test_graph_stats_against_networkx(seed):
    n = 400
    G = nx.gnp_random_graph(n, 4.0 / n, seed=seed)
    # add a few triangles and a hub
    G.add_edges_from([(0, 1), (1, 2), (0, 2), (5, 6), (6, 7), (5, 7), (5, 8), (7, 8)])
    G.add_edges_from((9, v) for v in range(10, 60))
    pairs = np.array(sorted(tuple(sorted(e)) for e in G.edges()), dtype=np.uint32)
    st = oracle.graph_stats(pairs, n)
    deg = np.array([G.degree(i) for i in range(n)])
    assert np.array_equal(st["degree"], deg)
    assert st["count"].tolist() == nx.degree_histogram(G)
    knn = nx.average_degree_connectivity(G)
    for d, v in knn.items():
        if d == 0:
            continue
        assert st["nbr_sum"][d] / (d * st["count"][d]) == pytest.approx(v, rel=1e-12)
    assert st["assortativity"] == pytest.approx(nx.degree_assortativity_coefficient(G), rel=1e-9, abs=1e-12)
    cl = nx.clustering(G)
    assert np.allclose(st["clustering"], [cl[i] for i in range(n)], rtol=0, atol=1e-15)
    assert st["avg_clustering"] == pytest.approx(nx.average_clustering(G), rel=1e-12)
    tri = nx.triangles(G)
    assert st["triangles_per_node"].tolist() == [tri[i] for i in range(n)]
    assert st["triangles"] == sum(tri.values()) // 3


def test_graph_stats_paper_example():
    st = oracle.graph_stats([[0, 1], [0, 2], [1, 4], [3, 4]], 5)
    assert st["degree"].tolist() == [2, 2, 1, 1, 2]
    assert st["count"].tolist() == [0, 2, 3]
    # <d_nn>(1) = (deg 2 + deg 2) / 2 ; <d_nn>(2) = (2+1 + 2+2 + 2+1) / (2*3)
    assert st["nbr_sum"].tolist() == [0, 4, 10]
    assert st["triangles"] == 0 and st["avg_clustering"] == 0.0
    # triangle graph: clustering 1 everywhere, assortativity undefined -> 0
    st = oracle.graph_stats([[0, 1], [0, 2], [1, 2]], 3)
    assert st["clustering"].tolist() == [1.0, 1.0, 1.0] and st["triangles"] == 1
