"""GPU parity of the batched form (many repertoires in one captured launch
sequence) against the CPU oracle, bit-exact per repertoire."""
import numpy as np
import pytest

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


def test_uneven_batch_matches_oracle(tn, ctx, orc):
    sizes = [0, 1, 2, 63, 64, 65, 700, 3000, 1500, 90, 4100, 10]
    reps = [synth.repertoire(n, max(1, n // 10), 500 + i) for i, n in enumerate(sizes)]
    for k in (1, 2):
        gs = tn.tcrnet_build_batch(ctx, reps, k)
        assert len(gs) == len(reps)
        for r, g in zip(reps, gs):
            e, d = orc.build(r, k)
            assert np.array_equal(g.pairs, e)
            assert np.array_equal(g.degree, d)


def test_many_small_repertoires_partial_plan_rounds(tn, ctx, orc):
    # 70 repertoires plan 32 (k + 1) entries each, 4,480 at k = 1 and 6,720 at
    # k = 2: more than the planning block has threads, so the planner hands
    # them out four to a thread, in rounds of 4,096 entries whose last one is
    # partial
    sizes = [37 + (i * 53) % 400 for i in range(70)]
    reps = [synth.repertoire(n, max(1, n // 8), 700 + i) for i, n in enumerate(sizes)]
    for k in (1, 2):
        gs = tn.tcrnet_build_batch(ctx, reps, k)
        assert len(gs) == len(reps)
        for r, g in zip(reps, gs):
            e, d = orc.build(r, k)
            assert np.array_equal(g.pairs, e)
            assert np.array_equal(g.degree, d)


def test_replayed_graph_gives_same_results(tn, ctx):
    reps = [synth.repertoire(n, n // 10, 900 + n) for n in (1200, 2500, 800)]
    a = tn.tcrnet_build_batch(ctx, reps, 1)
    b = tn.tcrnet_build_batch(ctx, reps, 1)   # same shape: captured graph replayed
    for x, y in zip(a, b):
        assert np.array_equal(x.pairs, y.pairs) and np.array_equal(x.degree, y.degree)
    # interleaved with a plain build on the same context
    tn.tcrnet_build(ctx, reps[0], 2)
    c = tn.tcrnet_build_batch(ctx, reps, 1)
    for x, y in zip(a, c):
        assert np.array_equal(x.pairs, y.pairs) and np.array_equal(x.degree, y.degree)


def test_paper_batch_256_repertoires(tn, ctx, orc):
    reps = synth.batch()
    gs = tn.tcrnet_build_batch(ctx, reps, 1)
    for r, g in zip(reps, gs):
        e, d = orc.k1_build(r)
        assert np.array_equal(g.pairs, e)
        assert np.array_equal(g.degree, d)


def test_invalid_repertoire_is_named(tn, ctx):
    reps = [["CASSF", "CASSY"], ["CASSF", "CASBF"]]
    with pytest.raises(tn.TcrnetError) as ei:
        tn.tcrnet_build_batch(ctx, reps, 1)
    assert ei.value.status == tn.TCRNET_EINVAL
    assert "repertoire 1" in ei.value.message and "sequence 1" in ei.value.message


def _check_batch(gs, reps, orc, k):
    for r, g in zip(reps, gs):
        e, d = orc.build(r, k)
        assert np.array_equal(g.pairs, e)
        assert np.array_equal(g.degree, d)


def test_graph_recaptured_after_plan_buffers_grow(tn, orc):
    """A plain build with a large k grows the work-plan buffers the captured
    batch graph uses; the next batch must capture again, not replay stale
    descriptor addresses."""
    reps = [synth.repertoire(n, n // 10, 1300 + n) for n in (900, 1700, 400)]
    with tn.Context(0) as c:
        a = tn.tcrnet_build_batch(c, reps, 1)
        assert c.last_info()["graph_captured"] == 1
        tn.tcrnet_build_batch(c, reps, 1)
        assert c.last_info()["graph_captured"] == 0     # replayed
        tn.tcrnet_build(c, synth.repertoire(600, 60, 5), 31)   # k = 31: many more descriptors
        b = tn.tcrnet_build_batch(c, reps, 1)
        assert c.last_info()["graph_captured"] == 1
    _check_batch(a, reps, orc, 1)
    _check_batch(b, reps, orc, 1)


def test_graph_recaptured_after_io_buffers_grow(tn, orc):
    """A larger plain build grows the degree, offset and pair buffers between
    two batches; an index on the same context grows them first."""
    reps = [synth.repertoire(n, n // 10, 1400 + n) for n in (1000, 2200)]
    with tn.Context(0) as c:
        idx = tn.tcrnet_index_create(c, synth.repertoire(5000, 500, 8), 1)
        a = tn.tcrnet_build_batch(c, reps, 1)
        tn.tcrnet_build(c, synth.repertoire(20000, 2000, 9), 1)
        b = tn.tcrnet_build_batch(c, reps, 1)
        assert c.last_info()["graph_captured"] == 1
        idx.close()
    _check_batch(a, reps, orc, 1)
    _check_batch(b, reps, orc, 1)


def test_autotuned_batch_is_exact_and_cached(tn, orc, tmp_path):
    reps = [synth.repertoire(n, max(1, n // 10), 1500 + i)
            for i, n in enumerate([1000, 2600, 1400, 5200, 1100, 3300, 1900, 700])]
    total = sum(r.n for r in reps)
    path = str(tmp_path / "tune.json")
    with tn.Context(0) as c:
        assert tn.tcrnet_autotune_get(c, True, total, 1) is None
        tn.tcrnet_autotune_batch(c, reps, 1)
        best = tn.tcrnet_autotune_get(c, True, total, 1)
        assert best is not None and best["ms"] > 0
        gs = tn.tcrnet_build_batch(c, reps, 1)
        info = c.last_info()
        assert info["tuned"] == 1
        for f in ("texts_per_item", "waves_per_simd", "peq_lds", "pack"):
            assert info[f] == best[f], f
        tn.tcrnet_autotune_save(c, path)
    for r, g in zip(reps, gs):
        e, d = orc.k1_build(r)
        assert np.array_equal(g.pairs, e) and np.array_equal(g.degree, d)
    # the table round-trips through its file into a fresh context
    with tn.Context(0) as c2:
        assert tn.tcrnet_autotune_load(c2, path) == 1
        assert tn.tcrnet_autotune_get(c2, True, total, 1) == best
        gs2 = tn.tcrnet_build_batch(c2, reps, 1)
        assert c2.last_info()["tuned"] == 1
    for a, b in zip(gs, gs2):
        assert np.array_equal(a.pairs, b.pairs) and np.array_equal(a.degree, b.degree)
    # a malformed file is rejected and leaves the table unchanged
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "tcrnet-autotune", "entries": [{"arch": "gfx950", "cus": 1}]}')
    with tn.Context(0) as c3:
        with pytest.raises(tn.TcrnetError) as ei:
            tn.tcrnet_autotune_load(c3, str(bad))
        assert ei.value.status == tn.TCRNET_EINVAL
        assert tn.tcrnet_autotune_get(c3, True, total, 1) is None
