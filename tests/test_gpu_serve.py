"""GPU parity of the served form (resident repertoire, query and insert
requests, continuous batching) against the CPU oracle, bit-exact.

Snapshot rule checked here: a request sees the initial repertoire plus every
insert admitted before it (lower sequence number).  Each result "in the mix"
must equal the oracle's answer for that snapshot alone.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

T0 = 2000   # templates of the test repertoire


@pytest.fixture(scope="module")
def tn():
    import paper_2112_06613_amd as tn
    return tn


@pytest.fixture(scope="module")
def ctx(tn):
    c = tn.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rep():
    return synth.repertoire(20000, T0, 7)


def _query_ref(orc, rep_seqs, q, k):
    return orc.query(rep_seqs, q, k)


def _insert_ref(orc, snap, new, k):
    """Edges (i < j) of the union network with j a new id, and the new nodes'
    degrees within those edges."""
    union = snap.concat(new)
    n_old = snap.n
    e, d = orc.build(union, k, row_lo=0, row_hi=union.n)
    sel = e[e[:, 1] >= n_old]
    cnt = np.zeros(new.n, dtype=np.int32)
    for i, j in sel.tolist():
        cnt[j - n_old] += 1
        if i >= n_old:
            cnt[i - n_old] += 1
    return sel, cnt, d


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_query_matches_oracle(tn, ctx, orc, rep, k):
    q = synth.queries(400, T0, 7, 99 + k)
    with tn.tcrnet_index_create(ctx, rep, 1) as idx:
        r = tn.tcrnet_query(idx, q, k)
    e, c = _query_ref(orc, rep, q, k)
    assert np.array_equal(r.pairs, e)
    assert np.array_equal(r.counts, c)
    assert r.info["is_insert"] == 0 and r.info["snapshot_size"] == rep.n


def test_index_degrees_equal_plain_build(tn, ctx, orc, rep):
    with tn.tcrnet_index_create(ctx, rep, 1) as idx:
        assert idx.size() == rep.n
        deg = idx.degree()
    _, d = orc.k1_build(rep)
    assert np.array_equal(deg, d)


def test_insert_then_query(tn, ctx, orc):
    base = synth.repertoire(3000, 300, 21)
    new = synth.queries(250, 300, 21, 5)
    with tn.tcrnet_index_create(ctx, base, 1) as idx:
        r = tn.tcrnet_insert(idx, new)
        assert idx.size() == base.n + new.n
        deg = idx.degree()
        q = synth.queries(100, 300, 21, 6)
        rq = tn.tcrnet_query(idx, q, 2)
    sel, cnt, d = _insert_ref(orc, base, new, 1)
    assert np.array_equal(r.pairs, sel)
    assert np.array_equal(r.counts, cnt)
    assert np.array_equal(deg, d)
    union = base.concat(new)
    e, c = orc.query(union, q, 2)
    assert np.array_equal(rq.pairs, e) and np.array_equal(rq.counts, c)


def test_empty_and_single_requests(tn, ctx, orc):
    base = synth.repertoire(1500, 150, 3)
    with tn.tcrnet_index_create(ctx, base, 1) as idx:
        r = tn.tcrnet_query(idx, [], 1)
        assert r.pairs.shape == (0, 2) and r.counts.shape == (0,)
        one = base.subset([17])
        r1 = tn.tcrnet_query(idx, one, 0)
        e, c = orc.query(base, one, 0)
        assert np.array_equal(r1.pairs, e) and r1.counts.tolist() == c.tolist()
        assert (0, 17) in set(map(tuple, r1.pairs.tolist()))


def test_mixed_trace_snapshot_semantics(tn, ctx, orc):
    """Many requests submitted at once (queries and inserts of uneven sizes,
    k in {1, 2}); more than 8 inserts, so segment merges run in between."""
    base = synth.repertoire(6000, 600, 44)
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(36):
        size = int(np.exp(rng.uniform(0, np.log(600))))
        k = int(rng.integers(1, 3))
        ins = bool(rng.random() < 0.35)
        reqs.append((synth.queries(size, 600, 44, 1000 + i), k, ins))
    with tn.tcrnet_index_create(ctx, base, 1) as idx:
        tickets = [tn.tcrnet_submit(idx, q, k, ins) for q, k, ins in reqs]
        results = [tn.tcrnet_wait(idx, t) for t in tickets]
        final_deg = idx.degree()
        final_n = idx.size()
    # replay in admission order against the oracle
    order = np.argsort([r.info["seqno"] for r in results])
    assert [results[i].info["seqno"] for i in order] == sorted(r.info["seqno"] for r in results)
    snap = base
    all_new_edges = []
    for i in order:
        q, k, ins = reqs[i]
        res = results[i]
        assert res.info["snapshot_size"] == snap.n
        if ins:
            sel, cnt, _ = _insert_ref(orc, snap, q, 1)
            assert np.array_equal(res.pairs, sel), f"insert {i}"
            assert np.array_equal(res.counts, cnt)
            all_new_edges.append(sel)
            snap = snap.concat(q)
        else:
            e, c = orc.query(snap, q, k)
            assert np.array_equal(res.pairs, e), f"query {i}"
            assert np.array_equal(res.counts, c)
    assert final_n == snap.n
    # rebuild invariant: initial network + every insert's edges = network of
    # the final repertoire; degrees match
    e_full, d_full = orc.build(snap, 1)
    e0, _ = orc.build(base, 1)
    merged = np.concatenate([e0] + all_new_edges) if all_new_edges else e0
    merged = merged[np.lexsort((merged[:, 1], merged[:, 0]))]
    assert np.array_equal(merged, e_full)
    assert np.array_equal(final_deg, d_full)


def test_small_budget_serialises_admission(tn, orc):
    base = synth.repertoire(4000, 400, 12)
    qs = [synth.queries(300, 400, 12, 50 + i) for i in range(6)]
    with tn.Context(0, hbm_budget=600_000, max_inflight=4) as c:
        with tn.tcrnet_index_create(c, base, 1) as idx:
            ts = [tn.tcrnet_submit(idx, q, 1) for q in qs]
            rs = [tn.tcrnet_wait(idx, t) for t in ts]
            big = synth.queries(4000, 400, 12, 99)
            with pytest.raises(tn.TcrnetError) as ei:
                tn.tcrnet_query(idx, big, 1)
            assert ei.value.status == tn.TCRNET_ENOMEM
    for q, r in zip(qs, rs):
        e, cnt = orc.query(base, q, 1)
        assert np.array_equal(r.pairs, e) and np.array_equal(r.counts, cnt)


def test_request_errors(tn, ctx):
    base = synth.repertoire(500, 50, 2)
    with tn.tcrnet_index_create(ctx, base, 1) as idx:
        with pytest.raises(tn.TcrnetError) as ei:
            tn.tcrnet_query(idx, ["CASSXF"], 1)
        assert ei.value.status == tn.TCRNET_EINVAL
        with pytest.raises(tn.TcrnetError) as ei:
            tn.tcrnet_wait(idx, 123456)
        assert ei.value.status == tn.TCRNET_ESTATE
        with pytest.raises(tn.TcrnetError):
            tn.tcrnet_query(idx, ["CASSF"], 40)
        # still serving
        r = tn.tcrnet_query(idx, base.subset([3]), 0)
        assert (0, 3) in set(map(tuple, r.pairs.tolist()))
