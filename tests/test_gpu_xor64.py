"""GPU parity of the xor64 pieces against the CPU oracle: the V4 variant
(Algorithm 4 with xor64 as each stream's generator) and V1 with xor64 as
Listing 1's first generator.  Outputs and written-back states are compared bit
for bit, across store modes, layouts, exchange modes, group sizes, tails and
split calls.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

V4 = 4


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


def _check(orc, G, variant_name, ov, ns, calls, sigma, tuning=None, group=0, comb=None,
           interleaved=False, v1_xor64=False):
    g = G.Generator(ns, variant_name, seed=sigma, group=group, comb=comb, interleaved=interleaved,
                    v1_xor64=v1_xor64)
    try:
        if tuning:
            g.set_tuning(**tuning)
        st = orc.seed(ov, sigma, 0, ns)
        assert np.array_equal(g.get_state(), st), "seeding differs"
        combs = None
        if ov == V4:
            combs = comb if comb is not None else orc.comb_tables(group or 32)
        for n in calls:
            got = G.as_u32(g.generate(n))
            want, _ = orc.generate(ov, st, n, comb=combs)
            if interleaved:
                got = got.T
            assert got.shape == want.shape
            bad = np.argwhere(got != want)
            assert bad.size == 0, f"n={n}: first mismatch (stream, step) at {bad[:3].tolist()}"
            assert np.array_equal(g.get_state(), st), f"n={n}: state after the call differs"
    finally:
        g.close()


@pytest.mark.parametrize("store", [1, 2, 3, 4])
@pytest.mark.parametrize("unroll", [8, 32, 128])
def test_v4_stream_major_store_modes(orc, G, store, unroll):
    _check(orc, G, "v4", V4, 2048, (1003, 64), sigma=51, tuning=dict(store=store, unroll=unroll))


@pytest.mark.parametrize("exchange", [1, 2, 3])
@pytest.mark.parametrize("unroll,block,slots", [(32, 128, 1), (64, 64, 2), (16, 256, 4)])
def test_v4_exchange_modes(orc, G, exchange, unroll, block, slots):
    # exchange 3 (two steps per read round) falls back to 1 for this variant
    _check(orc, G, "v4", V4, 4096, (512, 77), sigma=52,
           tuning=dict(store=2, exchange=exchange, unroll=unroll, block=block, streams_per_lane=slots))


@pytest.mark.parametrize("store", [7, 8])
def test_v4_pipelined(orc, G, store):
    _check(orc, G, "v4", V4, 4096, (1024, 1000), sigma=53, tuning=dict(store=store, unroll=64))


@pytest.mark.parametrize("group", [4, 8, 16, 64])
def test_v4_group_sizes(orc, G, group):
    _check(orc, G, "v4", V4, 1024, (300, 4), sigma=54, group=group, tuning=dict(exchange=2))


def test_v4_custom_combs_partial_wave(orc, G):
    c1 = np.array([3, 4, 0, 1, 7, 6, 2, 5], dtype=np.uint32)
    c2 = np.array([1, 3, 4, 2, 0, 7, 5, 6], dtype=np.uint32)
    _check(orc, G, "v4", V4, 40, (129, 3), sigma=55, group=8, comb=(c1, c2))


@pytest.mark.parametrize("n", [1, 3, 37, 1029])
def test_v4_ragged_tails(orc, G, n):
    _check(orc, G, "v4", V4, 512, (n, n), sigma=56)


@pytest.mark.parametrize("store", [2, 4, 1])
@pytest.mark.parametrize("block,unroll", [(256, 64), (512, 32), (1024, 16)])
def test_v4_interleaved_tiles(orc, G, store, block, unroll):
    _check(orc, G, "v4", V4, 3008, (1003, 40), sigma=57, interleaved=True,
           tuning=dict(store=store, block=block, unroll=unroll))


@pytest.mark.parametrize("exchange", [1, 2])
def test_v4_interleaved_double_buffered(orc, G, exchange):
    _check(orc, G, "v4", V4, 5024, (1003, 17), sigma=58, interleaved=True,
           tuning=dict(exchange=exchange, block=1024, unroll=16, streams_per_lane=2, store=4))


def test_v4_consume_counts(orc, G):
    ns, n = 512, 4096
    g = G.Generator(ns, "v4", seed=59)
    try:
        st = orc.seed(V4, 59, 0, ns)
        combs = orc.comb_tables(32)
        for _ in range(2):
            got = g.consume_qc(n).cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, orc.consume_qc(V4, st, n, comb=combs))
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


def test_v4_paper_shape_sampled(orc, G, torch):
    ns, n = 1 << 20, 1024
    g = G.Generator(ns, "v4", seed=60, interleaved=True)
    try:
        out = g.generate(n)
        torch.cuda.synchronize()
        combs = orc.comb_tables(32)
        rng = np.random.default_rng(20111223)
        for gr in np.unique(np.concatenate([[0, ns // 32 - 1], rng.integers(0, ns // 32, 200)])):
            got = G.as_u32(out[:, gr * 32:(gr + 1) * 32].cpu()).T
            st = orc.seed(V4, 60, int(gr) * 32, 32)
            want, _ = orc.generate(V4, st, n, comb=combs)
            assert np.array_equal(got, want), f"group {gr}"
    finally:
        g.close()


@pytest.mark.parametrize("interleaved,tuning", [(False, None), (False, dict(store=1, unroll=16)),
                                                (True, None), (True, dict(store=1))])
def test_v1_xor64_alternative(orc, G, interleaved, tuning):
    _check(orc, G, "v1", 1 | orc.F_XOR64, 1024, (1003, 21), sigma=61, tuning=tuning,
           interleaved=interleaved, v1_xor64=True)


def test_v1_xor64_consume(orc, G):
    ns, n = 256, 2048
    g = G.Generator(ns, "v1", seed=62, v1_xor64=True)
    try:
        st = orc.seed(1 | orc.F_XOR64, 62, 0, ns)
        got = g.consume_qc(n).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, orc.consume_qc(1 | orc.F_XOR64, st, n))
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()
