"""GPU parity of the DPP exchange (two row rotations per step) for V2 and V4.

The DPP exchange implements one fixed pair of combination arrays: groups of
16 streams, stream j mixing the previous words of streams (j + 1) mod 16 and
(j + 4) mod 16.  Handles created with those arrays are compared with the
oracle given the same arrays; handles with other arrays that ask for the DPP
exchange fall back to the cross-lane reads and must still match.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

C16 = 16
COMB1 = np.array([(j + 1) % C16 for j in range(C16)], dtype=np.uint32)
COMB2 = np.array([(j + 4) % C16 for j in range(C16)], dtype=np.uint32)


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


def _check(orc, G, name, ov, ns, calls, sigma, tuning, comb=(COMB1, COMB2), interleaved=False):
    g = G.Generator(ns, name, seed=sigma, group=len(comb[0]), comb=comb, interleaved=interleaved)
    try:
        g.set_tuning(**tuning)
        st = orc.seed(ov, sigma, 0, ns)
        for n in calls:
            got = G.as_u32(g.generate(n))
            want, _ = orc.generate(ov, st, n, comb=comb)
            if interleaved:
                got = got.T
            bad = np.argwhere(got != want)
            assert bad.size == 0, f"n={n}: first mismatch (stream, step) at {bad[:3].tolist()}"
            assert np.array_equal(g.get_state(), st), f"n={n}: state after the call differs"
    finally:
        g.close()


VARIANTS = [("v2", 2), ("v4", 4)]


@pytest.mark.parametrize("name,ov", VARIANTS)
@pytest.mark.parametrize("store,unroll,slots", [(2, 16, 1), (4, 32, 2), (4, 128, 1), (2, 64, 4)])
def test_dpp_stream_major_tiles(orc, G, name, ov, store, unroll, slots):
    _check(orc, G, name, ov, 2048, (1003, 64), sigma=71,
           tuning=dict(store=store, unroll=unroll, streams_per_lane=slots, exchange=4))


@pytest.mark.parametrize("name,ov", VARIANTS)
@pytest.mark.parametrize("store", [7, 8])
def test_dpp_pipelined(orc, G, name, ov, store):
    _check(orc, G, name, ov, 4096, (1024, 1000), sigma=72, tuning=dict(store=store, unroll=64, exchange=4))


@pytest.mark.parametrize("name,ov", VARIANTS)
@pytest.mark.parametrize("block,unroll,slots", [(1024, 16, 2), (512, 32, 1), (256, 8, 2)])
def test_dpp_interleaved_tiles(orc, G, name, ov, block, unroll, slots):
    _check(orc, G, name, ov, 5024, (1003, 17), sigma=73, interleaved=True,
           tuning=dict(store=4, block=block, unroll=unroll, streams_per_lane=slots, exchange=4))


@pytest.mark.parametrize("name,ov", VARIANTS)
def test_dpp_partial_wave(orc, G, name, ov):
    _check(orc, G, name, ov, 48, (129, 3), sigma=74, tuning=dict(store=2, unroll=16, exchange=4))


@pytest.mark.parametrize("name,ov", VARIANTS)
def test_dpp_consume(orc, G, name, ov):
    ns, n = 512, 4096
    g = G.Generator(ns, name, seed=75, group=C16, comb=(COMB1, COMB2))
    try:
        g.set_tuning(exchange=4)
        st = orc.seed(ov, 75, 0, ns)
        for _ in range(2):
            got = g.consume_qc(n).cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, orc.consume_qc(ov, st, n, comb=(COMB1, COMB2)))
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


def test_dpp_request_on_other_arrays_falls_back(orc, G):
    # group 16 with other arrays, and the default group of 32
    c1 = np.roll(COMB1, 3)
    c2 = np.roll(COMB2, 5)
    assert not np.any(c1 == np.arange(C16)) and not np.any(c2 == np.arange(C16)) and not np.any(c1 == c2)
    _check(orc, G, "v2", 2, 1024, (300,), sigma=76, comb=(c1, c2), tuning=dict(store=4, unroll=32, exchange=4))
    _check(orc, G, "v4", 4, 1024, (300,), sigma=77, comb=orc.comb_tables(32),
           tuning=dict(store=4, unroll=32, exchange=4), interleaved=True)
