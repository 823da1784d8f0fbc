"""GPU parity of the plain build against the CPU oracle (bit-exact).

Every comparison is element by element: the sorted (i < j) edge list and the
int32 degree array of the HIP path must equal the oracle's.  Inputs are seeded
synthetic repertoires (generator in ``synth``) or hand-made edge cases.
"""
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


def _eq(g, e, d):
    assert g.pairs.dtype == np.uint32 and g.degree.dtype == np.int32
    assert g.pairs.shape == e.shape, (g.pairs.shape, e.shape)
    assert np.array_equal(g.pairs, e)
    assert np.array_equal(g.degree, d)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 5, 8, 15, 16, 31])
def test_small_repertoire_matches_oracle(tn, ctx, orc, k):
    s = synth.small()
    g = tn.tcrnet_build(ctx, s, k)
    e, d = orc.build(s, k)
    _eq(g, e, d)
    assert g.info["evaluated_pairs"] > 0


def test_full_oracle_ragged_20000_k2(tn, ctx, orc):
    # several tiles per bucket, ragged tails everywhere (N not a multiple of 64)
    s = synth.repertoire(20011, 2001, 4242)
    g = tn.tcrnet_build(ctx, s, 2)
    e, d = orc.build(s, 2)
    _eq(g, e, d)


def test_medium_k1_against_closed_form(tn, ctx, orc):
    s = synth.medium()
    g = tn.tcrnet_build(ctx, s, 1)
    info = ctx.last_info()  # the defaults at 50,000 sequences: masks in VGPRs, 256 texts per item
    assert info["peq_lds"] == 0 and info["texts_per_item"] == 256
    e, d = orc.k1_build(s)
    _eq(g, e, d)


def test_medium_k2_full_oracle(tn, ctx, orc):
    # N = 50,000 at k = 2: the whole edge list and degree array against the
    # full-table DP over all 1.25e9 pairs (about 30 s on 16 host threads)
    s = synth.medium()
    g = tn.tcrnet_build(ctx, s, 2)
    e, d = orc.build(s, 2)
    _eq(g, e, d)


def test_medium_k2_sampled_rows_and_soundness(tn, ctx, orc):
    s = synth.medium()
    g = tn.tcrnet_build(ctx, s, 2)
    L = s.to_list()
    # every reported edge is a true edge (oracle DP on each pair)
    for i, j in g.pairs[:: max(1, len(g.pairs) // 4000)].tolist():
        assert orc.lev(L[i], L[j]) <= 2
    # sampled rows are complete and exact
    rng = np.random.default_rng(5)
    adj_from = {}
    for i, j in g.pairs.tolist():
        adj_from.setdefault(i, []).append(j)
        adj_from.setdefault(j, []).append(i)
    for i in rng.choice(s.n, 48, replace=False).tolist():
        ref = orc.row(s, 2, i)
        assert sorted(adj_from.get(i, [])) == ref.tolist()
        assert g.degree[i] == len(ref)
    assert int(g.degree.sum()) == 2 * len(g.pairs)


def test_paper_scale_k1_bit_exact(tn, ctx, orc):
    s = synth.paper_scale()
    g = tn.tcrnet_build(ctx, s, 1)
    info = ctx.last_info()  # the defaults at this size and k: masks in VGPRs, 8,192 texts per item
    assert info["peq_lds"] == 0 and info["texts_per_item"] == 8192
    e, d = orc.k1_build(s)
    _eq(g, e, d)
    # the same launch with the pattern masks in LDS
    with tn.Context(0, flags=tn.TCRNET_F_PEQ_LDS) as c:
        gv = tn.tcrnet_build(c, s, 1)
        assert c.last_info()["peq_lds"] == 1
    _eq(gv, e, d)
    # DP oracle on sampled rows (full rows of 800,000 comparisons each)
    rng = np.random.default_rng(11)
    rows = rng.choice(s.n, 12, replace=False).tolist()
    for i in rows:
        ref = orc.row(s, 1, i)
        got = np.sort(np.concatenate([g.pairs[g.pairs[:, 0] == i, 1], g.pairs[g.pairs[:, 1] == i, 0]]))
        assert np.array_equal(got, ref)


def test_degenerate_sizes(tn, ctx):
    for strs in ([], ["CASSF"]):
        g = tn.tcrnet_build(ctx, strs, 1)
        assert g.pairs.shape == (0, 2) and len(g.degree) == len(strs)
        assert np.all(g.degree == 0)


def test_all_duplicates_complete_graph_overflow(tn, ctx):
    # 500 equal strings: 124,750 edges, more than the default first capacity
    # of 65,536, so the overflow re-run runs
    n = 500
    g = tn.tcrnet_build(ctx, ["CASSLGQETQYF"] * n, 0)
    iu = np.triu_indices(n, 1)
    assert np.array_equal(g.pairs, np.stack(iu, 1).astype(np.uint32))
    assert np.all(g.degree == n - 1)
    assert g.info["pair_launches"] == 2


def test_lengths_spaced_apart_have_no_edges(tn, ctx):
    strs = ["A" * L for L in range(1, 33, 3)] * 3
    g = tn.tcrnet_build(ctx, strs, 2)
    # only equal strings (distance 0) are joined
    e = {(i, j) for i in range(len(strs)) for j in range(i + 1, len(strs)) if strs[i] == strs[j]}
    assert set(map(tuple, g.pairs.tolist())) == e


def test_extreme_lengths(tn, ctx, orc):
    rng = np.random.default_rng(3)
    alpha = np.array(list(synth.ALPHABET))
    base = "".join(rng.choice(alpha, 32))
    strs = [base, base[:31], base[1:], base[:16] + "W" + base[17:], "A", "C", "AC", base[::-1]]
    strs += ["".join(rng.choice(alpha[:3], rng.integers(1, 33))) for _ in range(300)]
    s = synth.Seqs.from_list(strs)
    for k in (0, 1, 2, 5, 31):
        g = tn.tcrnet_build(ctx, s, k)
        e, d = orc.build(s, k)
        _eq(g, e, d)


def test_bucket_edges_ragged_counts(tn, ctx, orc):
    # buckets of 1, 63, 64, 65, 129 sequences over a tiny alphabet (many edges)
    rng = np.random.default_rng(8)
    strs = []
    for L, cnt in ((7, 1), (8, 63), (9, 64), (10, 65), (11, 129)):
        strs += ["".join(rng.choice(list("ARN"), L)) for _ in range(cnt)]
    rng.shuffle(strs)
    s = synth.Seqs.from_list(strs)
    for k in (1, 2):
        g = tn.tcrnet_build(ctx, s, k)
        e, d = orc.build(s, k)
        _eq(g, e, d)


def test_permutation_invariance_and_determinism(tn, ctx):
    s = synth.small(seed=77)
    g1 = tn.tcrnet_build(ctx, s, 1)
    g2 = tn.tcrnet_build(ctx, s, 1)
    assert np.array_equal(g1.pairs, g2.pairs) and np.array_equal(g1.degree, g2.degree)
    perm = np.random.default_rng(1).permutation(s.n)
    sp = s.subset(perm.tolist())
    gp = tn.tcrnet_build(ctx, sp, 1)
    back = np.sort(perm[gp.pairs.astype(np.int64)], axis=1)
    order = np.lexsort((back[:, 1], back[:, 0]))
    assert np.array_equal(back[order].astype(np.uint32), g1.pairs)
    assert np.array_equal(gp.degree, g1.degree[perm])


def test_threshold_monotone(tn, ctx):
    s = synth.small(seed=5)
    prev = set()
    for k in range(0, 5):
        cur = set(map(tuple, tn.tcrnet_build(ctx, s, k).pairs.tolist()))
        assert prev <= cur
        prev = cur


@pytest.mark.parametrize("opts", [dict(texts_per_item=64), dict(texts_per_item=2048, waves_per_simd=2),
                                  dict(flags=2), dict(flags=2, texts_per_item=192), dict(edge_capacity=16),
                                  dict(flags=4), dict(flags=4 | 2, texts_per_item=320),
                                  dict(texts_per_item=576, waves_per_simd=3), dict(flags=8),
                                  dict(flags=8 | 2), dict(flags=8 | 4, texts_per_item=128)])
def test_schedules_give_identical_results(tn, orc, opts):
    s = synth.repertoire(5000, 500, 31)
    e, d = orc.build(s, 2)
    with tn.Context(0, **opts) as c:
        g = tn.tcrnet_build(c, s, 2)
    _eq(g, e, d)


@pytest.mark.parametrize("bad,msg", [(["CASSF", "CAXSF"], "sequence 1"), (["CASSF", ""], "sequence 1"),
                                     (["C" * 33], "sequence 0"), (["cassf"], "sequence 0"),
                                     (["CASSF", "CASBF"], "sequence 1"), (["CASSF", "CASSZ"], "sequence 1"),
                                     (["C@SSF"], "sequence 0"), (["CASS["], "sequence 0"),
                                     (["CASSF", "CASSF", "CASJF", "CAOSF"], "sequence 2")])
def test_invalid_input_rejected(tn, ctx, bad, msg):
    with pytest.raises(tn.TcrnetError) as ei:
        tn.tcrnet_build(ctx, bad, 1)
    assert ei.value.status == tn.TCRNET_EINVAL
    assert msg in ei.value.message
    # the context stays usable after an error
    g = tn.tcrnet_build(ctx, ["CASSF", "CASSY"], 1)
    assert g.pairs.tolist() == [[0, 1]]


@pytest.mark.parametrize("k", [-1, 32])
def test_bad_threshold_rejected(tn, ctx, k):
    with pytest.raises(tn.TcrnetError) as ei:
        tn.tcrnet_build(ctx, ["CASSF"], k)
    assert ei.value.status == tn.TCRNET_EINVAL


def test_device_entry_point_matches_host(tn, ctx):
    import torch
    s = synth.repertoire(30000, 3000, 17)
    ref = tn.tcrnet_build(ctx, s, 1)
    dev = torch.device("cuda", 0)
    chars = torch.from_numpy(s.chars).to(dev)
    offs = torch.from_numpy(s.offsets.astype(np.int64)).to(dev)
    deg = torch.empty(s.n, dtype=torch.int32, device=dev)
    pairs = torch.empty((len(ref.pairs) + 10, 2), dtype=torch.int32, device=dev)
    E = tn.tcrnet_build_device(ctx, chars, offs, 1, pairs, deg, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert E == len(ref.pairs)
    assert np.array_equal(pairs[:E].cpu().numpy().view(np.uint32), ref.pairs)
    assert np.array_equal(deg.cpu().numpy(), ref.degree)
    # too small an output buffer: ETRUNC with the required count; a repeat
    # with that capacity gives the full result
    small = torch.empty((10, 2), dtype=torch.int32, device=dev)
    with pytest.raises(tn.TcrnetError) as ei:
        tn.tcrnet_build_device(ctx, chars, offs, 1, small, deg)
    assert ei.value.status == tn.TCRNET_ETRUNC and ei.value.n_edges == E
    exact = torch.empty((E, 2), dtype=torch.int32, device=dev)
    assert tn.tcrnet_build_device(ctx, chars, offs, 1, exact, deg) == E
    torch.cuda.synchronize()
    assert np.array_equal(exact.cpu().numpy().view(np.uint32), ref.pairs)
    assert np.array_equal(deg.cpu().numpy(), ref.degree)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_device_entry_point_unaligned_chars(tn, ctx, shift):
    # the strings start 1-3 bytes past an aligned address and the last one
    # ends at the end of the buffer the caller passes
    import torch
    s = synth.repertoire(5000, 500, 41)
    ref = tn.tcrnet_build(ctx, s, 1)
    dev = torch.device("cuda", 0)
    buf = torch.zeros(len(s.chars) + shift, dtype=torch.uint8, device=dev)
    buf[shift:] = torch.from_numpy(s.chars).to(dev)
    chars = buf[shift:]
    assert chars.data_ptr() % 4 == shift
    offs = torch.from_numpy(s.offsets.astype(np.int64)).to(dev)
    deg = torch.empty(s.n, dtype=torch.int32, device=dev)
    pairs = torch.empty((len(ref.pairs) + 1, 2), dtype=torch.int32, device=dev)
    E = tn.tcrnet_build_device(ctx, chars, offs, 1, pairs, deg, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert E == len(ref.pairs)
    assert np.array_equal(pairs[:E].cpu().numpy().view(np.uint32), ref.pairs)
    assert np.array_equal(deg.cpu().numpy(), ref.degree)


@pytest.mark.parametrize("k_max", [2, 4])
def test_weighted_build_every_threshold(tn, ctx, orc, k_max):
    s = synth.repertoire(3000, 300, 123)
    g = tn.tcrnet_build_weighted(ctx, s, k_max)
    assert g.dist is not None and len(g.dist) == len(g.pairs)
    L = s.to_list()
    for (i, j), d in zip(g.pairs.tolist()[::7], g.dist.tolist()[::7]):
        assert orc.lev(L[i], L[j]) == d
    for k in range(0, k_max + 1):
        e, d = orc.build(s, k)
        assert np.array_equal(g.at(k), e)
        if k == k_max:
            assert np.array_equal(g.degree, d)
    plain = tn.tcrnet_build(ctx, s, k_max)
    assert plain.dist is None and np.array_equal(plain.pairs, g.pairs)


def test_valu_peak_probe(tn, ctx):
    # measured 32-bit VALU issue rate of xor/add chains: above one wave64
    # instruction per SIMD per 4 clocks at half the clock, and not above the
    # dual-issue peak 256 CUs x 128 lanes x 2.4 GHz (margin for the timer)
    rate, sec = tn.tcrnet_valu_peak(ctx)
    assert sec > 0
    assert 0.5 * 256 * 64 * 2.4e9 < rate < 1.05 * 256 * 128 * 2.4e9


def test_valu_rate_probe(tn, ctx):
    """Every instruction form gets a positive rate; the plain xor form runs at
    the rate the peak probe measures (same chains, same grid)."""
    rates = tn.tcrnet_valu_rates(ctx)
    assert len(rates) == 12 and "v_pk_add_u16" in rates and "v_cmp_eq_u32" in rates
    assert all(v > 1e12 for v in rates.values())
    peak, _ = tn.tcrnet_valu_peak(ctx)
    assert 0.7 < rates["v_xor_b32"] / peak < 1.3


def test_injected_allocation_failures_are_clean(tn, orc):
    """Every device or pinned allocation of a build failing in turn: the call
    returns TCRNET_ENOMEM with no result, and the next call on the same
    context is correct."""
    s = synth.repertoire(3000, 300, 77)
    e, d = orc.build(s, 1)
    lib = tn.load_library()
    failures = 0
    try:
        for after in range(40):
            with tn.Context(0) as c:
                lib.tcrnet_debug_fail_alloc(after)
                try:
                    g = tn.tcrnet_build(c, s, 1)
                except tn.TcrnetError as err:
                    assert err.status == tn.TCRNET_ENOMEM, err
                    failures += 1
                    lib.tcrnet_debug_fail_alloc(-1)
                    g = tn.tcrnet_build(c, s, 1)
                lib.tcrnet_debug_fail_alloc(-1)
                _eq(g, e, d)
    finally:
        lib.tcrnet_debug_fail_alloc(-1)
    assert failures >= 10   # the sweep reached the build's allocations
