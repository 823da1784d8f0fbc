"""The allocation-free device build (tcrnet_build_device_noalloc) against the
allocating one (tcrnet_build_device) through the C-ABI: bit-exact edge lists
and degrees on two calls in a row, the second over a smaller input (the
shared static scratch keeps the first call's contents), and no library
allocation during the calls."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tn():
    import paper_2112_06613_amd as tn
    return tn


def _to_dev(s):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(s.chars).to(dev), torch.from_numpy(s.offsets.astype(np.int64)).to(dev))


def _out(n, cap):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.full((cap, 2), -1, dtype=torch.int32, device=dev),
            torch.full((n,), -7, dtype=torch.int32, device=dev))


def test_noalloc_matches_device_build_on_two_calls(tn, orc):
    import torch
    lib = tn.load_library()
    cases = [(40000, 4000, 20211301, 1), (9000, 900, 20211302, 2)]  # the second smaller
    with tn.Context(0) as ctx:
        for n, templates, seed, k in cases:
            s = synth.repertoire(n, templates, seed)
            chars, offs = _to_dev(s)
            cap = 4 * n
            ref_pairs, ref_deg = _out(n, cap)
            E_ref = tn.tcrnet_build_device(ctx, chars, offs, k, ref_pairs, ref_deg)
            pairs, deg = _out(n, cap)
            torch.cuda.synchronize()
            # any allocation through the library's allocators fails from here
            lib.tcrnet_debug_fail_alloc(0)
            try:
                E = tn.tcrnet_build_device_noalloc(ctx, chars, offs, k, pairs, deg,
                                                   torch.cuda.current_stream())
                # still armed: the call made no allocation (a new context
                # allocates pinned memory and must hit the armed failure)
                with pytest.raises(tn.TcrnetError) as ei:
                    tn.Context(0)
                assert ei.value.status == tn.TCRNET_ENOMEM
            finally:
                lib.tcrnet_debug_fail_alloc(-1)
            torch.cuda.synchronize()
            assert E == E_ref and E > 0
            assert np.array_equal(pairs[:E].cpu().numpy(), ref_pairs[:E].cpu().numpy())
            assert np.array_equal(deg.cpu().numpy(), ref_deg.cpu().numpy())
            assert (pairs[E:].cpu().numpy() == -1).all()  # nothing written past E
            if n <= 10000:  # the oracle finishes in seconds here
                e, d = orc.build(s, k)
                assert np.array_equal(pairs[:E].cpu().numpy().view(np.uint32), e)
                assert np.array_equal(deg.cpu().numpy(), d)


def test_noalloc_limits_and_truncation(tn):
    import torch
    s = synth.repertoire(3000, 300, 20211303)
    chars, offs = _to_dev(s)
    with tn.Context(0) as ctx:
        ref_pairs, ref_deg = _out(s.n, 4 * s.n)
        E = tn.tcrnet_build_device(ctx, chars, offs, 1, ref_pairs, ref_deg)
        # an output capacity whose edge staging exceeds the static scratch:
        # rejected before any device work
        big = tn.NOALLOC_SCRATCH_BYTES // 24
        pairs, deg = _out(s.n, big)
        with pytest.raises(tn.TcrnetError) as ei:
            tn.tcrnet_build_device_noalloc(ctx, chars, offs, 1, pairs, deg)
        assert ei.value.status == tn.TCRNET_EINVAL and "scratch" in str(ei.value)
        assert (deg.cpu().numpy() == -7).all()
        del pairs
        # too small an output: TCRNET_ETRUNC with the required count
        small, deg = _out(s.n, 5)
        with pytest.raises(tn.TcrnetError) as ei:
            tn.tcrnet_build_device_noalloc(ctx, chars, offs, 1, small, deg)
        assert ei.value.status == tn.TCRNET_ETRUNC and ei.value.n_edges == E
        # empty input and a single sequence
        for m in (0, 1):
            c2, o2 = _to_dev(synth.Seqs.from_list(["CASSF"] * m))
            p2, d2 = _out(max(m, 1), 4)
            assert tn.tcrnet_build_device_noalloc(ctx, c2, o2, 1, p2, d2) == 0
        # the allocating entry point still works after the static one
        pairs, deg = _out(s.n, 4 * s.n)
        assert tn.tcrnet_build_device(ctx, chars, offs, 1, pairs, deg) == E
        torch.cuda.synchronize()
        assert np.array_equal(pairs[:E].cpu().numpy(), ref_pairs[:E].cpu().numpy())
        assert np.array_equal(deg.cpu().numpy(), ref_deg.cpu().numpy())
