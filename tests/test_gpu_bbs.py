"""GPU parity of the BBS-based variant (V3, Algorithm 5) against the CPU oracle.

Outputs are compared bit for bit, per call: each call picks the two
arrangement arrays from slots 1 and 2 at its start and rotates the slots at
its end, so split calls are checked against the oracle split the same way.
Sizes span several tiles of every kernel, partial waves and ragged tails.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

V3 = 3


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def G(torch):
    from paper_1112_5239_amd import generator
    return generator


def _check(orc, G, ns, ns_calls, sigma, tuning=None, group=0, interleaved=False):
    """Generate len(ns_calls) calls of the given lengths and compare each."""
    g = G.Generator(ns, "v3", seed=sigma, group=group, interleaved=interleaved)
    try:
        if tuning:
            g.set_tuning(**tuning)
        st = orc.seed(V3, sigma, 0, ns)
        assert np.array_equal(g.get_state(), st), "seeding differs"
        combs = orc.bbs_comb_tables(group or 32)
        for n in ns_calls:
            got = G.as_u32(g.generate(n))
            want, _ = orc.generate(V3, st, n, comb=combs)
            if interleaved:
                got = got.T
            assert got.shape == want.shape
            bad = np.argwhere(got != want)
            assert bad.size == 0, f"n={n}: first mismatch (stream, step) at {bad[:3].tolist()}"
            assert np.array_equal(g.get_state(), st), f"n={n}: state after the call differs"
    finally:
        g.close()


@pytest.mark.parametrize("store", [1, 2, 3, 4])
@pytest.mark.parametrize("unroll", [8, 16, 32, 64])
def test_stream_major_store_modes(orc, G, store, unroll):
    # 2,048 streams: several workgroups; n = 1,003 leaves a tail after whole
    # K-step rounds; the second call continues with rotated slots.
    _check(orc, G, 2048, (1003, 64), sigma=31, tuning=dict(store=store, unroll=unroll))


@pytest.mark.parametrize("exchange", [1, 2, 3])
@pytest.mark.parametrize("unroll,block,slots", [(32, 128, 1), (64, 64, 2), (16, 256, 4)])
def test_exchange_modes(orc, G, exchange, unroll, block, slots):
    # exchange 3 (two steps per read round) falls back to 1 for this variant.
    _check(orc, G, 4096, (512, 77), sigma=32,
           tuning=dict(store=2, exchange=exchange, unroll=unroll, block=block, streams_per_lane=slots))


@pytest.mark.parametrize("store", [7, 8])
@pytest.mark.parametrize("unroll", [16, 32, 128])
def test_pipelined_persistent(orc, G, store, unroll):
    # unroll 128 is lowered to 32 for this variant.
    _check(orc, G, 4096, (1024, 1000), sigma=33, tuning=dict(store=store, unroll=unroll))


@pytest.mark.parametrize("group", [4, 8, 16, 64])
def test_group_sizes(orc, G, group):
    _check(orc, G, 1024, (300, 4), sigma=34, group=group, tuning=dict(exchange=2))
    _check(orc, G, 1024, (300,), sigma=35, group=group, tuning=dict(exchange=1, store=4))


@pytest.mark.parametrize("ns,group", [(96, 32), (40, 8), (8, 4)])
def test_partial_waves(orc, G, ns, group):
    # fewer streams than a wave, and a wave cut in the middle of its groups
    _check(orc, G, ns, (129, 3), sigma=36, group=group)


@pytest.mark.parametrize("n", [1, 3, 4, 37, 100, 1029])
def test_ragged_tail_lengths(orc, G, n):
    _check(orc, G, 512, (n, n), sigma=37)


def test_many_short_calls_rotate_the_slots(orc, G):
    # eight calls of one output bring every slot through both selector seats
    _check(orc, G, 256, (1,) * 9 + (2, 5), sigma=38)


def test_zero_length_call_is_a_no_op(orc, G):
    g = G.Generator(256, "v3", seed=39)
    try:
        before = g.get_state()
        g.generate(0)
        assert np.array_equal(g.get_state(), before)
        st = orc.seed(V3, 39, 0, 256)
        orc.generate(V3, st, 0)
        assert np.array_equal(st, before)
        want, _ = orc.generate(V3, st, 16)
        assert np.array_equal(G.as_u32(g.generate(16)), want)
    finally:
        g.close()


@pytest.mark.parametrize("store", [2, 4, 1])
@pytest.mark.parametrize("block,unroll", [(256, 64), (512, 32), (1024, 16), (256, 8)])
def test_interleaved_tiles(orc, G, store, block, unroll):
    # 3,008 streams: a partial last tile; n = 1,003 rounds plus a tail.
    _check(orc, G, 3008, (1003, 40), sigma=40, interleaved=True,
           tuning=dict(store=store, block=block, unroll=unroll))


@pytest.mark.parametrize("exchange", [1, 2])
@pytest.mark.parametrize("block,unroll", [(1024, 8), (512, 16), (256, 32)])
def test_interleaved_double_buffered_tiles(orc, G, block, unroll, exchange):
    _check(orc, G, 5024, (1003, 17), sigma=41, interleaved=True,
           tuning=dict(exchange=exchange, block=block, unroll=unroll, streams_per_lane=2, store=4))


def test_interleaved_fallback_per_lane(orc, G):
    # n_streams % 4 != 0 selects the per-lane interleaved kernel
    _check(orc, G, 1000, (100, 3), sigma=42, group=8, interleaved=True)


def test_consume_counts(orc, G):
    ns, n = 512, 4096
    g = G.Generator(ns, "v3", seed=43)
    try:
        st = orc.seed(V3, 43, 0, ns)
        combs = orc.bbs_comb_tables(32)
        for _ in range(2):
            got = g.consume_qc(n).cpu().numpy().astype(np.uint64)
            want = orc.consume_qc(V3, st, n, comb=combs)
            assert np.array_equal(got, want)
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


def test_set_state_round_trip_and_validation(orc, G):
    g = G.Generator(128, "v3", seed=44)
    try:
        st = orc.seed(V3, 45, 0, 128)
        g.set_state(st)
        assert np.array_equal(g.get_state(), st)
        want, _ = orc.generate(V3, st.copy(), 64)
        assert np.array_equal(G.as_u32(g.generate(64)), want)
        bad = st.copy()
        bad[5, 2] = 1 << 16          # a BBS slot outside [0, 2^16)
        from paper_1112_5239_amd import _lib as L
        with pytest.raises(L.CprngError):
            g.set_state(bad)
    finally:
        g.close()


def test_paper_shape_sampled(orc, G, torch):
    # 2^20 streams x 1,024 outputs, interleaved, in the default configuration;
    # the first 64 streams and a seeded sample of whole groups are checked.
    ns, n = 1 << 20, 1024
    g = G.Generator(ns, "v3", seed=46, interleaved=True)
    try:
        out = g.generate(n)
        torch.cuda.synchronize()
        combs = orc.bbs_comb_tables(32)
        rng = np.random.default_rng(20111223)
        groups = np.unique(np.concatenate([[0, 1, ns // 32 - 1], rng.integers(0, ns // 32, 200)]))
        for gr in groups:
            cols = out[:, gr * 32:(gr + 1) * 32].cpu()
            got = G.as_u32(cols).T
            st = orc.seed(V3, 46, int(gr) * 32, 32)
            want, _ = orc.generate(V3, st, n, comb=combs)
            assert np.array_equal(got, want), f"group {gr}"
    finally:
        g.close()


def test_every_slot_state_below_2_16(orc, G):
    # Across 65,536 streams each slot takes every value in [0, 2^16) (a
    # different permutation per slot), so the kernel's modular squaring is
    # checked on its whole input range against the oracle's plain remainder.
    ns = 1 << 16
    g = G.Generator(ns, "v3", seed=47)
    try:
        st = orc.seed(V3, 47, 0, ns)
        s = np.arange(ns, dtype=np.uint64)
        for k in range(8):
            st[:, k] = (s * (2 * k + 1) + k) & 0xFFFF
        g.set_state(st)
        for n in (2, 5):
            want, _ = orc.generate(V3, st, n)
            assert np.array_equal(G.as_u32(g.generate(n)), want)
            assert np.array_equal(g.get_state(), st)
    finally:
        g.close()
