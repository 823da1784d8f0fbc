"""The seeded generator: C and pure-Python twins agree; recipe statistics."""
import math

import numpy as np
import pytest

import synth


@pytest.mark.parametrize("tseed,T,sseed,N", [(1, 1, 2, 50), (20211213, 200, 20211214, 700),
                                             (2**64 - 1, 37, 0, 300)])
def test_c_and_python_agree(tseed, T, sseed, N):
    a = synth.generate(tseed, T, sseed, N)
    b = synth.generate_py(tseed, T, sseed, N)
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.chars, b.chars)


def test_deterministic_and_seed_sensitive():
    a, b, c = synth.small(), synth.small(), synth.small(seed=1)
    assert np.array_equal(a.chars, b.chars) and np.array_equal(a.offsets, b.offsets)
    assert not np.array_equal(a.chars[:1000], c.chars[:1000])


def test_alphabet_and_lengths():
    s = synth.medium()
    assert s.n == 50000
    assert set(np.unique(s.chars).tobytes().decode()) <= set(synth.ALPHABET)
    L = s.lengths()
    assert L.min() >= 1 and L.max() <= 32
    assert 13.5 < L.mean() < 14.5


def test_template_statistics():
    # templates: 'C' ... 'F', length round(N(14,2)) clipped to [6, 25]
    tm = synth.generate(77, 4000, 78, 0)
    assert tm.n == 0
    r = synth.SplitMix64(77)
    lens = []
    for _ in range(4000):
        L = synth._template_len(r)
        lens.append(L)
        for _ in range(L - 2):
            r.next()
    lens = np.array(lens)
    assert lens.min() >= 6 and lens.max() <= 25
    assert abs(lens.mean() - 14.0) < 0.15
    assert abs(lens.std() - 2.0) < 0.15


def test_edit_count_statistics():
    # P(no edit) = exp(-1.5): fraction of exact template copies
    T = 50
    s = synth.generate(5, T, 6, 20000)
    # reconstruct templates from the Python twin with zero sequences drawn
    r = synth.SplitMix64(5)
    tm = set()
    for _ in range(T):
        L = synth._template_len(r)
        t = "C" + "".join(synth.ALPHABET[r.below(20)] for _ in range(L - 2)) + "F"
        tm.add(t)
    frac = sum(x in tm for x in s.to_list()) / s.n
    assert abs(frac - math.exp(-1.5)) < 0.02


def test_batch_and_trace_shapes():
    sizes = synth.batch_sizes()
    assert len(sizes) == 256 and min(sizes) >= 1000 and max(sizes) <= 40000
    assert 6000 < np.mean(sizes) < 16000
    tr = synth.request_trace(2000, 100.0)
    assert all(1 <= q.size <= 4096 for q in tr)
    assert 0.15 < np.mean([q.insert for q in tr]) < 0.25
    assert set(q.k for q in tr) == {1, 2}
    t = np.array([q.t_arrival for q in tr])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.01) < 0.002
