"""The pair kernel's counting variant (TCRNET_F_COUNT_WORK) counts exactly the
work the benchmark's work model prices: visited texts, wave text steps and
the packed steps among them, at the small workload (N = 2,000, the figures
stored in bench_model.json) and at a 20,000-sequence build; its edges and
degrees equal the oracle's."""
import json
import os

import numpy as np
import pytest

import synth
import workmodel as wm

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tn():
    import paper_2112_06613_amd as tn
    return tn


def _counted(tn, s, k, **opts):
    with tn.Context(0, flags=tn.TCRNET_F_COUNT_WORK, **opts) as ctx:
        g = tn.tcrnet_build(ctx, s, k)
    assert g.info["work_counted"] == 1
    return g


@pytest.mark.parametrize("which,k", [("small", 1), ("n20000", 1), ("n20000", 2)])
def test_counts_equal_the_work_model(tn, orc, which, k):
    s = synth.small() if which == "small" else synth.repertoire(20000, 2000, 20211304)
    g = _counted(tn, s, k)
    e, d = orc.build(s, k)
    assert np.array_equal(g.pairs, e) and np.array_equal(g.degree, d)
    info = g.info
    model = wm.traversal(s, k, info["texts_per_item"], 1 << 22, pack=bool(info["pack"]))
    assert model["exact"]
    assert info["wave_steps"] == model["wave_steps"]
    assert info["wave_steps_packed"] == model["wave_steps_packed"]
    assert info["visited_texts"] == model["visited_texts"]
    if which == "small":
        with open(os.path.join(ROOT, "bench_model.json")) as f:
            stored = json.load(f)["workloads"]["small_n2000_k1"]["traversal"]
        assert stored["texts_per_item"] == info["texts_per_item"]
        assert info["wave_steps"] == stored["wave_steps"]
        assert info["visited_texts"] == stored["visited_texts"]


def test_counts_without_packing_and_other_item_sizes(tn):
    s = synth.repertoire(6000, 600, 20211305)
    for T, flags in ((64, 0), (1024, tn.TCRNET_F_NO_PACK)):
        with tn.Context(0, texts_per_item=T, flags=tn.TCRNET_F_COUNT_WORK | flags) as ctx:
            g = tn.tcrnet_build(ctx, s, 1)
        model = wm.traversal(s, 1, T, 1 << 22, pack=not flags)
        assert model["exact"]
        assert (g.info["wave_steps"], g.info["wave_steps_packed"], g.info["visited_texts"]) == \
            (model["wave_steps"], model["wave_steps_packed"], model["visited_texts"])
