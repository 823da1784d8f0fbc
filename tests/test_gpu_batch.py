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
