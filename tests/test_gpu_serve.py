"""GPU parity of the served form (resident repertoire, query and insert
requests, continuous batching) against the CPU oracle, bit-exact.

Snapshot rule checked here: a request sees the initial repertoire plus every
insert admitted before it (lower sequence number).  Each result "in the mix"
must equal the oracle's answer for that snapshot alone.
"""
import time

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


@pytest.mark.parametrize("k", [16, 31])
def test_query_large_k_matches_oracle(tn, ctx, orc, rep, k):
    # a query's cross part plans 32 (2k + 1) entries, here more than the
    # planning block has threads: they go four to a thread; no packing (a
    # masked half's 16 set miss bits would not exceed k)
    q = synth.queries(40, T0, 7, 301 + k)
    with tn.tcrnet_index_create(ctx, rep, 1) as idx:
        r = tn.tcrnet_query(idx, q, k)
    e, c = _query_ref(orc, rep, q, k)
    assert np.array_equal(r.pairs, e)
    assert np.array_equal(r.counts, c)


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
    q_last = synth.queries(20, 80000, synth.SEED_PAPER, 5999)
    with tn.tcrnet_index_create(ctx, base, 1) as idx:
        tickets = [tn.tcrnet_submit(idx, q, k, ins) for q, k, ins in reqs]
        results = [tn.tcrnet_wait(idx, t) for t in tickets]
        final_deg = idx.degree()
        final_n = idx.size()
        # merges of the base and the insert segments are published once
        # their device work is done: a later query reads a merged base and
        # at most the 5 insert segments a merge waits for, not 1 + 10
        # segments
        time.sleep(0.2)
        last = tn.tcrnet_query(idx, q_last, 2)
        assert last.info["parts"] <= 6, last.info
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


def _insert_ref_cross(orc, snap, new, k):
    """Insert reference without the O(N^2) rebuild: the new sequences against
    the snapshot (oracle query) plus the new sequences among themselves."""
    n_old = snap.n
    e1, c1 = orc.query(snap, new, k)          # (q, r) pairs
    e2, d2 = orc.build(new, k)                # (a, b), a < b
    parts = []
    if len(e1):
        parts.append(np.stack([e1[:, 1], e1[:, 0] + n_old], axis=1).astype(np.uint32))
    if len(e2):
        parts.append((e2 + n_old).astype(np.uint32))
    sel = np.concatenate(parts) if parts else np.zeros((0, 2), dtype=np.uint32)
    sel = sel[np.lexsort((sel[:, 1], sel[:, 0]))]
    return sel, (c1 + d2).astype(np.int32)


def test_paper_scale_resident_mixed_trace(tn, ctx, orc):
    """The served form at its real resident size: 800,000 sequences indexed at
    k = 1, then 26 requests submitted at once -- queries of 1-64 sequences at
    k in {1, 2} and 10 inserts (so a segment merge of the 800,000-sequence
    base runs in between).  Every result equals the oracle's answer for its
    snapshot; the final degrees equal those of the final repertoire."""
    base = synth.paper_scale()
    rng = np.random.default_rng(31)
    reqs = []
    n_ins = 0
    for i in range(26):
        ins = (i % 5 in (1, 3)) or (i > 20 and n_ins < 10)
        n_ins += ins
        size = int(np.exp(rng.uniform(0, np.log(64)))) if not ins else int(rng.integers(1, 33))
        k = 1 if ins else int(rng.integers(1, 3))
        reqs.append((synth.queries(size, 80000, synth.SEED_PAPER, 5000 + i), k, ins))
    assert sum(r[2] for r in reqs) >= 9     # more than 8 insert segments: a merge runs
    q_last = synth.queries(20, 80000, synth.SEED_PAPER, 5999)
    with tn.tcrnet_index_create(ctx, base, 1) as idx:
        tickets = [tn.tcrnet_submit(idx, q, k, ins) for q, k, ins in reqs]
        results = [tn.tcrnet_wait(idx, t) for t in tickets]
        final_deg = idx.degree()
        final_n = idx.size()
        # merges of the base and the insert segments are published once
        # their device work is done: a later query reads a merged base and
        # at most the 5 insert segments a merge waits for, not 1 + 10
        # segments
        time.sleep(0.2)
        last = tn.tcrnet_query(idx, q_last, 2)
        assert last.info["parts"] <= 6, last.info
    order = np.argsort([r.info["seqno"] for r in results])
    snap = base
    new_edges = []
    for i in order:
        q, k, ins = reqs[i]
        res = results[i]
        assert res.info["snapshot_size"] == snap.n
        if ins:
            sel, cnt = _insert_ref_cross(orc, snap, q, 1)
            assert np.array_equal(res.pairs, sel), f"insert {i}"
            assert np.array_equal(res.counts, cnt), f"insert {i}"
            new_edges.append(sel)
            snap = snap.concat(q)
        else:
            e, c = orc.query(snap, q, k)
            assert np.array_equal(res.pairs, e), f"query {i}"
            assert np.array_equal(res.counts, c), f"query {i}"
    assert final_n == snap.n
    e, c = orc.query(snap, q_last, 2)
    assert np.array_equal(last.pairs, e) and np.array_equal(last.counts, c)
    # final degrees: the base network (k = 1 witness) plus every insert's edges
    _, d0 = orc.k1_build(base)
    deg = np.zeros(snap.n, dtype=np.int64)
    deg[:base.n] = d0
    for sel in new_edges:
        np.add.at(deg, sel[:, 0].astype(np.int64), 1)
        np.add.at(deg, sel[:, 1].astype(np.int64), 1)
    assert np.array_equal(final_deg, deg.astype(np.int32))


def test_insert_failing_after_admission_never_leaves_a_torn_index(tn, orc):
    """Every allocation of an insert failing in turn: the insert reports
    TCRNET_ENOMEM and the index is either unchanged (the failure came before
    the insert's sequences joined the repertoire; later requests are exact)
    or failed (every later call reports TCRNET_ESTATE) -- never a repertoire
    with sequences whose edges and degrees are missing.  The insert is larger
    than the 4,096 sequences a serving slot holds buffers for, so that it
    still allocates after its sequences joined the repertoire."""
    base = synth.repertoire(2000, 200, 61)
    new = synth.queries(5000, 200, 61, 62)
    _, d_base = orc.build(base, 1)
    sel, cnt, d_union = _insert_ref(orc, base, new, 1)
    lib = tn.load_library()
    seen_failed = seen_unchanged = 0
    try:
        with tn.Context(0) as c:
            for after in range(30):
                with tn.tcrnet_index_create(c, base, 1) as idx:
                    lib.tcrnet_debug_fail_alloc(after)
                    try:
                        r = tn.tcrnet_insert(idx, new)
                        lib.tcrnet_debug_fail_alloc(-1)
                        assert np.array_equal(r.pairs, sel) and np.array_equal(r.counts, cnt)
                        assert np.array_equal(idx.degree(), d_union)
                        continue
                    except tn.TcrnetError as err:
                        lib.tcrnet_debug_fail_alloc(-1)
                        assert err.status == tn.TCRNET_ENOMEM, err
                    try:
                        n_now = idx.size()
                    except tn.TcrnetError as err:
                        assert err.status == tn.TCRNET_ESTATE
                        with pytest.raises(tn.TcrnetError) as ei:
                            tn.tcrnet_query(idx, new, 1)
                        assert ei.value.status == tn.TCRNET_ESTATE
                        seen_failed += 1
                        continue
                    assert n_now == base.n
                    assert np.array_equal(idx.degree(), d_base)
                    r = tn.tcrnet_insert(idx, new)
                    assert np.array_equal(r.pairs, sel) and np.array_equal(r.counts, cnt)
                    assert np.array_equal(idx.degree(), d_union)
                    seen_unchanged += 1
    finally:
        lib.tcrnet_debug_fail_alloc(-1)
    assert seen_unchanged >= 1 and seen_failed >= 1
