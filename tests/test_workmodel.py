"""The benchmark's work model (workmodel/walk.c via workmodel/__init__.py):
its own DP exit steps and distances equal the oracle's, the prefix-group
walk it replays is exact (every text a jump skips has no lane within k,
checked against the oracle's full DP distances), and the C replay matches a
plain Python walk over the same items."""
import numpy as np
import pytest

import synth
import workmodel as wm


def _setup(n, T, k, seed, pack=True):
    s = synth.repertoire(n, max(1, n // 10), seed)
    M, L = wm.code_matrix(s)
    order = wm.sorted_order(M, L)
    gend = wm.group_ends(M, L, order)
    items = wm.plan_items(L[order], k, T, pack)
    return s, L, order, gend, items


def test_sorted_order_and_group_ends():
    s, L, order, gend, _ = _setup(600, 64, 1, 5)
    strs = s.to_list()
    srt = [strs[i] for i in order]
    assert [len(x) for x in srt] == sorted(len(x) for x in srt)
    for p in range(len(srt)):
        for d in range(1, wm.DEPTHS + 1):
            e = gend[p, d - 1]
            assert e > p
            key = (len(srt[p]), srt[p][:d])
            assert all((len(srt[q]), srt[q][:d]) == key for q in range(p, e))
            assert e == len(srt) or (len(srt[e]), srt[e][:d]) != key


@pytest.mark.parametrize("k,pack", [(1, True), (2, True), (1, False)])
def test_walk_is_exact_and_matches_python(orc, k, pack):
    s, L, order, gend, items = _setup(500, 128, k, 9 + k, pack)
    assert (items[:, 5] > wm.WAVE).any() == pack
    strs = s.to_list()
    steps_c, texts_c = wm.work_items(s, order, gend, items, k, wm.RESUME)
    skipped = 0
    for q, (gbase, npat, tb, te, tri, width) in enumerate(items.tolist()):
        steps = visited = 0
        t = tb
        prev = None
        while t < te:
            b = strs[order[t]]
            lanes = [p for p in range(gbase, gbase + npat) if not (tri and p >= t)]
            ex = [orc.exit_step(strs[order[p]], b, k) for p in lanes]
            full = any(orc.lev(strs[order[p]], b) <= k for p in lanes)
            e = max(ex)
            r = 0
            if prev is not None:
                a = strs[order[prev]]
                while r < min(len(b), wm.RESUME) and a[r] == b[r]:
                    r += 1
            steps += (len(b) if full else e) - r
            visited += 1
            prev = t if (not tri or t - gbase >= width) else None
            tn = t + 1
            if not full and e <= wm.DEPTHS and (not tri or t - gbase >= width):
                tn = max(int(gend[t, e - 1]), t + 1)
                skipped += min(tn, te) - t - 1
                # every skipped text: no lane within k (full DP distances)
                for u in range(t + 1, min(tn, te)):
                    bu = strs[order[u]]
                    assert all(orc.lev(strs[order[p]], bu) > k for p in range(gbase, gbase + npat)
                               if not (tri and p >= u))
            t = tn
        assert (steps, visited) == (int(steps_c[q]), int(texts_c[q]))
    assert skipped > 0


@pytest.mark.parametrize("k", [0, 1, 2, 5])
def test_model_exit_steps_equal_the_oracles(orc, k):
    s = synth.repertoire(400, 40, 31 + k)
    rng = np.random.default_rng(k)
    pi = rng.integers(0, s.n, 3000)
    pj = rng.integers(0, s.n, 3000)
    got = wm.exit_steps(s, pi, pj, k)
    want = orc.exit_steps(s, pi, pj, k)
    assert np.array_equal(got, want)
    strs = s.to_list()
    for i, j in list(zip(pi, pj))[:300]:
        e, lev = wm.exit_step(strs[i], strs[j], k)
        assert e == orc.exit_step(strs[i], strs[j], k) and lev == orc.lev(strs[i], strs[j])


def test_traversal_totals_small():
    out = wm.traversal(synth.small(), 1, 16384, 1 << 20)
    assert out["exact"] and out["items"] == out["items_modelled"]
    assert 0 < out["visited_texts"] <= out["wave_steps"]


def test_group_widths_follow_pattern_length():
    """Two patterns share a lane for pattern lengths up to 16 (k < 16): the
    items of a bucket pair cover its patterns in groups of 128, otherwise 64,
    and every pattern lands in exactly one group per text chunk."""
    s, L, order, gend, items = _setup(3000, 256, 1, 4)
    Ls = L[order]
    for gbase, npat, tb, te, tri, width in items.tolist():
        m = int(Ls[gbase])
        assert width == (128 if m <= wm.PACK_MAX_LEN else 64)
        assert 1 <= npat <= width and (Ls[gbase:gbase + npat] == m).all()
    assert wm.group_width(16, 15, True) == 128 and wm.group_width(16, 16, True) == 64
    assert wm.group_width(17, 1, True) == 64 and wm.group_width(10, 1, False) == 64


@pytest.mark.parametrize("T,pack", [(128, True), (256, False), (64, True)])
def test_items_cover_every_kept_pair_once(T, pack):
    """The modelled work items tile the length-filtered pair space: summed
    over items, the (pattern, text) pairs they hold (pattern before text in
    a triangle) equal the kept pairs of the length histogram, and no item
    holds a pair twice (its patterns and texts are disjoint ranges)."""
    s, L, order, gend, items = _setup(3000, T, 1, 7, pack)
    Ls = L[order]
    total = 0
    for gbase, npat, tb, te, tri, width in items.tolist():
        if te <= tb:
            continue
        if tri:
            # pairs (p, t): gbase <= p < gbase + npat, tb <= t < te, p < t
            for p in range(gbase, gbase + npat):
                total += max(0, te - max(tb, p + 1))
        else:
            total += npat * (te - tb)
        assert (Ls[tb:te] == Ls[tb]).all()
    cnt = np.bincount(Ls, minlength=34).astype(np.int64)
    want = sum(int(cnt[m] * (cnt[m] - 1) // 2 + cnt[m] * cnt[m - 1]) for m in range(2, 33)) + int(cnt[1] * (cnt[1] - 1) // 2)
    assert total == want
