"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Every pin comes from the paper's text, the mathematics of the edit distance,
or a brute force that shares no arithmetic with the DP:
  * the paper's worked distance example and its 5-node adjacency example
    (tests/golden/, each with its citation);
  * textbook values (kitten/sitting = 3);
  * a breadth-first search over single edits on tiny alphabets (the definition
    of the distance as the least number of edits, no recursion);
  * metric axioms and the bounds |m-n| <= lev <= max(m, n), lev <= Hamming;
  * the DP-free closed form of threshold 1, in C and in Python.
"""
import os
import random

import numpy as np
import pytest

import synth
from oracle.checks import bfs_distances, hamming, k1_adjacent

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_worked_example_from_paper(orc):
    rows = _golden_lines("levenshtein_worked_example.txt")
    assert rows
    for a, b, d in rows:
        assert orc.lev(a, b) == int(d)
        assert orc.lev(b, a) == int(d)


def test_textbook_values(orc):
    assert orc.lev("kitten", "sitting") == 3
    assert orc.lev("flaw", "lawn") == 2
    assert orc.lev("", "") == 0
    assert orc.lev("", "ARN") == 3
    assert orc.lev("ARN", "") == 3
    assert orc.lev("CASSLGQF", "CASSLGQF") == 0


def test_equal_length_is_not_hamming(orc):
    # The Methods text calls the equal-length distance "Hamming"; that only
    # bounds it from above.  One deletion plus one insertion beats 4 mismatches.
    assert hamming("CASSF", "ASSFC") == 4
    assert orc.lev("CASSF", "ASSFC") == 2


@pytest.mark.parametrize("alphabet,max_len", [("AR", 4), ("ARN", 3)])
def test_bfs_brute_force(orc, alphabet, max_len):
    dist = bfs_distances(alphabet, max_len)
    assert len(dist) > 900
    for (a, b), d in dist.items():
        assert orc.lev(a, b) == d, (a, b)


def test_metric_axioms_random(orc):
    rng = random.Random(7)
    strs = ["".join(rng.choice(synth.ALPHABET[:4]) for _ in range(rng.randint(0, 12)))
            for _ in range(60)]
    D = {(a, b): orc.lev(a, b) for a in strs for b in strs}
    for a in strs:
        for b in strs:
            d = D[(a, b)]
            assert d == D[(b, a)]
            assert (d == 0) == (a == b)
            assert abs(len(a) - len(b)) <= d <= max(len(a), len(b))
            if len(a) == len(b):
                assert d <= hamming(a, b)
    for a in strs[:25]:
        for b in strs[:25]:
            for c in strs[:25]:
                assert D[(a, c)] <= D[(a, b)] + D[(b, c)]


def test_adjacency_example_from_paper(orc):
    rows = {r[0]: r[1:] for r in _golden_lines("adjacency_example.txt") if r[0] in ("strings", "k", "edges")}
    mat = [list(map(int, r)) for r in _golden_lines("adjacency_example.txt") if r[0] in "01"]
    strings, k = rows["strings"], int(rows["k"][0])
    edges1 = [tuple(int(x) for x in e.split("-")) for e in rows["edges"]]
    s = synth.Seqs.from_list(strings)
    e, d = orc.build(s, k)
    assert [tuple(x) for x in e.tolist()] == [(i - 1, j - 1) for i, j in edges1]
    A = np.zeros((5, 5), dtype=int)
    for i, j in e.tolist():
        A[i, j] = A[j, i] = 1
    assert A.tolist() == mat
    assert d.tolist() == A.sum(axis=1).tolist() == [2, 2, 1, 1, 2]


def test_k1_closed_form_pairwise(orc):
    s = synth.small()
    L = s.to_list()
    rng = random.Random(3)
    lens = s.lengths()
    # length-compatible pairs (the only ones where the closed form can say yes)
    # plus every pair among a block of templates' neighbours
    checked = 0
    for _ in range(20000):
        i, j = rng.randrange(len(L)), rng.randrange(len(L))
        if abs(lens[i] - lens[j]) > 1:
            continue
        d = orc.lev(L[i], L[j])
        assert k1_adjacent(L[i], L[j]) == (d <= 1)
        assert orc.k1_adjacent(L[i], L[j]) == (d <= 1)
        checked += 1
    assert checked > 5000
    for a, b in [("CASSF", "CASSF"), ("CASSF", "CASF"), ("CASF", "CASSF"), ("CASSF", "CATSF"),
                 ("CASSF", "ASSFC"), ("C", "F"), ("C", "CC"), ("CC", "C")]:
        assert orc.k1_adjacent(a, b) == (orc.lev(a, b) <= 1) == k1_adjacent(a, b)


def test_network_small_against_k1_witness(orc):
    s = synth.small()
    e, d = orc.build(s, 1)
    e1, d1 = orc.k1_build(s)
    assert np.array_equal(e, e1)
    assert np.array_equal(d, d1)
    assert int(d.sum()) == 2 * len(e)
    assert len(e) > 1000          # the generator makes template families
    assert np.all(e[:, 0] < e[:, 1])


def test_network_invariants(orc):
    s = synth.repertoire(600, 40, 99)
    e0, d0 = orc.build(s, 0)
    e1, d1 = orc.build(s, 1)
    e2, d2 = orc.build(s, 2)
    sets = [set(map(tuple, x.tolist())) for x in (e0, e1, e2)]
    assert sets[0] <= sets[1] <= sets[2]
    L = s.to_list()
    for (i, j) in sets[0]:
        assert L[i] == L[j]
    for e, d in ((e0, d0), (e1, d1), (e2, d2)):
        keys = e[:, 0].astype(np.uint64) << np.uint64(32) | e[:, 1].astype(np.uint64)
        assert np.all(np.diff(keys.astype(np.int64)) > 0)      # sorted, unique
        assert int(d.sum()) == 2 * len(e)
        # degree is the row sum of the adjacency, recomputed here
        ref = np.bincount(e.ravel(), minlength=s.n)
        assert np.array_equal(ref, d)


def test_degenerate_inputs(orc):
    e, d = orc.build(synth.Seqs.from_list([]), 1)
    assert len(e) == 0 and len(d) == 0
    e, d = orc.build(synth.Seqs.from_list(["CASSF"]), 1)
    assert len(e) == 0 and d.tolist() == [0]
    n = 40
    e, d = orc.build(synth.Seqs.from_list(["CASSLF"] * n), 0)
    assert len(e) == n * (n - 1) // 2 and np.all(d == n - 1)
    # lengths more than k apart: no edges at all
    e, d = orc.build(synth.Seqs.from_list(["A" * L for L in range(1, 30, 3)]), 2)
    assert len(e) == 0


def test_query_matches_pairwise(orc):
    rep = synth.repertoire(500, 50, 5)
    qs = synth.queries(60, 50, 5, 1234)
    R, Q = rep.to_list(), qs.to_list()
    for k in (1, 2):
        pairs, cnt = orc.query(rep, qs, k)
        ref = [(q, r) for q in range(len(Q)) for r in range(len(R)) if orc.lev(Q[q], R[r]) <= k]
        assert [tuple(p) for p in pairs.tolist()] == ref
        assert cnt.tolist() == [sum(1 for (q, _) in ref if q == i) for i in range(len(Q))]


def test_row_matches_build(orc):
    s = synth.repertoire(800, 60, 11)
    e, d = orc.build(s, 2)
    adj = [[] for _ in range(s.n)]
    for i, j in e.tolist():
        adj[i].append(j)
        adj[j].append(i)
    for i in (0, 1, 17, 400, 799):
        assert orc.row(s, 2, i).tolist() == sorted(adj[i])
    # a block of rows equals the matching slice of the full network
    eb, _ = orc.build(s, 2, row_lo=100, row_hi=300)
    sl = e[(e[:, 0] >= 100) & (e[:, 0] < 300)]
    assert np.array_equal(eb, sl)


def test_exit_step_model_against_bfs(orc):
    # The work model's exit step is the first text column j whose final-
    # diagonal cell D[j + m - n][j] exceeds k; that cell is the edit distance
    # of the two prefixes, so the breadth-first search fixes it too.
    dist = bfs_distances("AR", 4)
    strs = sorted({a for a, _ in dist if a})
    for k in (0, 1, 2):
        for a in strs:
            for b in strs:
                long_, short = (a, b) if len(a) >= len(b) else (b, a)
                m, n = len(long_), len(short)
                want = n
                for j in range(1, n + 1):
                    if dist[(long_[: j + m - n], short[:j])] > k:
                        want = j
                        break
                assert orc.exit_step(a, b, k) == want, (a, b, k)
                if dist[(a, b)] <= k:
                    assert want == n   # a true edge never exits early


def test_exit_step_hand_examples(orc):
    # CAS vs CWW already differ by 2 on the main diagonal after 3 columns
    assert orc.exit_step("CASSLF", "CWWWWF", 1) == 3
    # one deletion apart: the bound never exceeds 1
    assert orc.exit_step("CASSF", "CASF", 1) == 4
    assert orc.exit_step("CASSLGQETQYF", "CASSLGQETQYF", 0) == 12
