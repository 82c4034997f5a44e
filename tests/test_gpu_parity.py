"""GPU parity: the HIP kernels (through the C ABI) against the CPU oracle.

Integer outputs are compared bit for bit.  Sizes span several tiles of every
kernel plus ragged tails; the full-size paper-shaped case is checked on the
first 64 streams plus a seeded 1% sample of streams expanded to whole
exchange groups.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _oracle_states(orc, variant, sigma, ns, W=64):
    return orc.seed(variant, sigma, 0, ns, W=W)


def _gen_check(orc, G, variant_name, variant, ns, n, sigma=0, w32=False, calls=1, tuning=None,
               comb=None, group=0):
    W = 32 if w32 else 64
    g = G.Generator(ns, variant_name, seed=sigma, w32=w32, comb=comb, group=group)
    try:
        if tuning:
            g.set_tuning(**tuning)
        st = _oracle_states(orc, variant, sigma, ns, W)
        assert np.array_equal(g.get_state(), st), "seeding differs"
        combs = None
        if variant == 2:
            combs = comb if comb is not None else orc.comb_tables(group or 32)
        for _ in range(calls):
            got = G.as_u32(g.generate(n))
            want, _ = orc.generate(variant, st, n, W=W, comb=combs)
            assert got.shape == want.shape
            bad = np.argwhere(got != want)
            assert bad.size == 0, f"first mismatch at {bad[:3].tolist()}"
        assert np.array_equal(g.get_state(), st), "end state differs"
    finally:
        g.close()


# ---------------------------------------------------------------------------
# Plain generator, 1,024 streams x 1,024 outputs, seed 0 (V0 and V1).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("store", [1, 2, 3, 4])
@pytest.mark.parametrize("unroll", [8, 16, 32, 64, 128, 256])
def test_v0_plain_1024x1024_all_store_modes(orc, G, store, unroll):
    _gen_check(orc, G, "v0", 0, 1024, 1024, sigma=0, tuning=dict(store=store, unroll=unroll, block=256))


# The stream-major defaults depend on the stream count: one-wave blocks with
# direct stores up to one wave per CU (16,384 streams on 256 CUs; V1 up to six,
# 98,304), one-wave LDS tiles above that (V0 up to six waves per CU, V2 up to
# four, 65,536), the large-shape defaults beyond.
def _cu_count(torch):
    return torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v1", 1), ("v2", 2)])
@pytest.mark.parametrize("ns", [16384, 16448, 65536, 65600, 81920, 81952, 98304, 98336])
def test_few_streams_default_bands(orc, G, torch, variant_name, variant, ns):
    # Both sides of each band edge with the default configuration; n with a
    # tail after the 32-step rounds.
    _gen_check(orc, G, variant_name, variant, ns, 44, sigma=5, calls=2)


def test_few_streams_defaults_resolved(G, torch):
    if _cu_count(torch) != 256:
        pytest.skip("the band edges are stated for 256 compute units")
    cases = [(1024, "v0", (64, 32, 1)), (16384, "v2", (64, 32, 1)), (16384, "v1", (64, 32, 1)),
             (16448, "v0", (64, 32, 2)), (65536, "v2", (64, 32, 2)), (65600, "v2", (256, 32, 2)),
             (98304, "v0", (64, 32, 2)), (98336, "v0", (128, 128, 4)),
             (98304, "v1", (64, 32, 1)), (98336, "v1", (256, 32, 4))]
    for ns, name, want in cases:
        g = G.Generator(ns, name, seed=0)
        try:
            cfg = g.resolved_tuning(1024)
            assert cfg["source"] == "default", (ns, name, cfg)
            assert (cfg["block"], cfg["unroll"], cfg["store"]) == want, (ns, name, cfg)
        finally:
            g.close()


@pytest.mark.parametrize("unroll,block,waves,slots", [(64, 64, 2, 1), (128, 128, 4, 1), (256, 64, 0, 1),
                                                      (32, 192, 6, 1), (64, 128, 0, 2), (32, 64, 4, 4),
                                                      (128, 64, 0, 4), (16, 256, 0, 2)])
def test_lds_tiles_and_occupancy_caps(orc, G, unroll, block, waves, slots):
    # n = 1000: rounds of K plus a tail; 1000 streams: a partial last wave
    # (and partial slots when several streams share a lane).
    for name, variant in (("v0", 0), ("v2", 2), ("v1", 1)):
        ns = 992 if variant == 2 else 1000
        _gen_check(orc, G, name, variant, ns, 1000, sigma=12,
                   tuning=dict(store=2, unroll=unroll, block=block, waves_per_cu=waves,
                               streams_per_lane=slots))


@pytest.mark.parametrize("store", [7, 8])
@pytest.mark.parametrize("unroll", [16, 32, 64, 128])
def test_pipelined_persistent_modes(orc, G, store, unroll):
    # One persistent wave per CU over ~40k streams: each workgroup takes
    # several 64-stream blocks in turn, the last block is partial, and
    # n = 1056 (rows on 128-byte lines) leaves a tail after the pipelined
    # rounds of 64 and 128.
    for name, variant in (("v0", 0), ("v2", 2), ("v1", 1)):
        ns = 40032 if variant == 2 else 40037
        _gen_check(orc, G, name, variant, ns, 1056, sigma=21,
                   tuning=dict(store=store, unroll=unroll, waves_per_cu=1))


@pytest.mark.parametrize("exchange", [1, 2, 3])
@pytest.mark.parametrize("n", [32, 1024, 1056, 1000])
def test_pipelined_v2_exchange_modes(orc, G, exchange, n):
    # n = 32: shorter than a round of 64, or one round of 32; 1024: rounds only;
    # 1056: rounds and a tail; 1000: rows off the lines (LDS tiles instead).
    _gen_check(orc, G, "v2", 2, 20480, n, sigma=22, calls=2,
               tuning=dict(store=7, unroll=64 if exchange != 2 else 32, waves_per_cu=2, exchange=exchange))


@pytest.mark.parametrize("w32", [False, True])
def test_v1_naive3_1024x1024(orc, G, w32):
    _gen_check(orc, G, "v1", 1, 1024, 1024, sigma=0, w32=w32)


@pytest.mark.parametrize("store", [1, 2])
def test_v1_naive3_store_modes_and_blocks(orc, G, store):
    for block in (64, 128):
        _gen_check(orc, G, "v1", 1, 640, 96, sigma=5, tuning=dict(store=store, unroll=16, block=block))


# ---------------------------------------------------------------------------
# Neighbour-exchange variant (Algorithm 4).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("store,unroll", [(1, 32), (2, 32), (3, 32), (4, 32), (2, 128), (4, 256)])
def test_v2_shmem_4096x1024(orc, G, store, unroll):
    _gen_check(orc, G, "v2", 2, 4096, 1024, sigma=1, tuning=dict(store=store, unroll=unroll, block=64))


@pytest.mark.parametrize("exchange", [1, 2, 3])
@pytest.mark.parametrize("unroll,block,slots", [(32, 128, 1), (64, 64, 2), (128, 64, 1), (16, 256, 4)])
def test_v2_exchange_modes(orc, G, exchange, unroll, block, slots):
    # Cross-lane reads, LDS word buffer, and two steps per read round; a
    # partial last wave (2080 streams) and a tail (n = 1000).
    _gen_check(orc, G, "v2", 2, 2080, 1000, sigma=14,
               tuning=dict(store=2, unroll=unroll, block=block, streams_per_lane=slots, exchange=exchange))


@pytest.mark.parametrize("exchange", [2, 3])
@pytest.mark.parametrize("group", [4, 16, 64])
def test_v2_exchange_modes_group_sizes(orc, G, exchange, group):
    _gen_check(orc, G, "v2", 2, 512, 200, sigma=15, group=group,
               tuning=dict(store=4, unroll=32, block=128, exchange=exchange))


@pytest.mark.parametrize("group", [4, 8, 16, 64])
def test_v2_other_group_sizes_default_combs(orc, G, group):
    _gen_check(orc, G, "v2", 2, 512, 200, sigma=3, group=group)


def test_v2_custom_combs_and_partial_wave(orc, G):
    # 96 streams = one full wave plus half a wave; explicit combination arrays.
    rng = np.random.default_rng(17)
    c1 = rng.permutation(32).astype(np.uint32)
    c2 = rng.permutation(32).astype(np.uint32)
    for store in (1, 2):
        _gen_check(orc, G, "v2", 2, 96, 64, sigma=9, comb=(c1, c2), group=32,
                   tuning=dict(store=store, unroll=16, block=128))


# ---------------------------------------------------------------------------
# Tails, alignment, continuation, interleaved layout.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v1", 1), ("v2", 2)])
@pytest.mark.parametrize("n", [1, 3, 4, 37, 100, 1029])
def test_ragged_tail_lengths(orc, G, variant_name, variant, n):
    ns = 160 if variant == 2 else 131           # partial last wave
    _gen_check(orc, G, variant_name, variant, ns, n, sigma=2)


@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v1", 1), ("v2", 2)])
@pytest.mark.parametrize("unroll,store,exchange", [(32, 2, 2), (64, 4, 1), (128, 4, 2), (32, 4, 3),
                                                   (64, 2, 3), (128, 2, 1), (32, 1, 1), (64, 7, 2)])
def test_rows_off_lines(orc, G, torch, variant_name, variant, unroll, store, exchange):
    # Stream-major rows that start off 128-byte lines (n not a multiple of 32
    # or of 4, a base at any 4-byte phase of a line) take line-aligned pieces
    # whatever the store mode asked (LDS tiles, per-lane quads, pipelined);
    # rows shorter than a round, a partial last wave, several calls.  Words
    # around the output must stay untouched.
    ns, sigma, fill = (1056 if variant == 2 else 1000), 31, 0x5A5A5A5A
    g = G.Generator(ns, variant_name, seed=sigma)
    try:
        kw = dict(store=store, unroll=unroll, block=256)
        if variant == 2:
            kw["exchange"] = exchange
        g.set_tuning(**kw)
        st = _oracle_states(orc, variant, sigma, ns)
        combs = orc.comb_tables(32) if variant == 2 else None
        buf = torch.full((ns * 1060 + 96,), fill, dtype=torch.int32, device="cuda")
        assert buf.data_ptr() % 16 == 0
        phase0 = (buf.data_ptr() // 4) % 32
        for n, phase in ((1000, 0), (1024, 4), (1024, 28), (4, 0), (28, 12), (100, 8), (1060, 20), (132, 0),
                         (1001, 1), (1003, 30), (7, 5), (1, 3), (1026, 2), (1024, 17), (33, 0), (64, 31)):
            off = (phase - phase0) % 32
            g.generate(n, out=buf[off:off + ns * n])
            torch.cuda.synchronize()
            want, _ = orc.generate(variant, st, n, comb=combs)
            host = G.as_u32(buf)
            got = host[off:off + ns * n].reshape(ns, n)
            bad = np.argwhere(got != want)
            assert bad.size == 0, f"n={n}, line phase {phase}: first mismatch at {bad[:3].tolist()}"
            assert (host[:off] == fill).all() and (host[off + ns * n:] == fill).all(), f"n={n}: wrote outside"
            buf.fill_(fill)
        assert np.array_equal(g.get_state(), st), "end state differs"
    finally:
        g.close()


@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v1", 1), ("v2", 2)])
def test_continuation_across_calls(orc, G, variant_name, variant):
    _gen_check(orc, G, variant_name, variant, 256, 64, sigma=4, calls=3)


def test_misaligned_output_pointer(orc, G, torch):
    g = G.Generator(100, "v0", seed=6)
    try:
        buf = torch.zeros(100 * 64 + 1, dtype=torch.int32, device="cuda")
        g.generate(64, out=buf[1:])               # 4-byte but not 16-byte aligned
        want, _ = orc.generate(0, _oracle_states(orc, 0, 6, 100), 64)
        assert np.array_equal(G.as_u32(buf[1:]).reshape(100, 64), want)
        assert G.as_u32(buf[:1])[0] == 0
    finally:
        g.close()


@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v2", 2), ("v1", 1)])
def test_interleaved_layout(orc, G, variant_name, variant):
    ns, n = 192, 50
    g = G.Generator(ns, variant_name, seed=8, interleaved=True)
    try:
        got = G.as_u32(g.generate(n))
        assert got.shape == (n, ns)
        want, _ = orc.generate(variant, _oracle_states(orc, variant, 8, ns), n)
        assert np.array_equal(got.T, want)
    finally:
        g.close()


def _ilv_check(orc, G, variant_name, variant, ns, n, sigma, tuning=None, calls=2):
    g = G.Generator(ns, variant_name, seed=sigma, interleaved=True)
    try:
        if tuning:
            g.set_tuning(**tuning)
        st = _oracle_states(orc, variant, sigma, ns)
        for _ in range(calls):
            got = G.as_u32(g.generate(n))
            assert got.shape == (n, ns)
            want, _ = orc.generate(variant, st, n)
            bad = np.argwhere(got.T != want)
            assert bad.size == 0, f"first mismatch (stream, step) at {bad[:3].tolist()}"
        assert np.array_equal(g.get_state(), st), "end state differs"
    finally:
        g.close()


@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v1", 1), ("v2", 2)])
@pytest.mark.parametrize("ns", [81920, 81952, 131072, 131104])
def test_interleaved_few_streams_default_band(orc, G, torch, variant_name, variant, ns):
    # With few streams the interleaved default is the per-lane dword kernel
    # (V0 up to 81,920 streams on 256 CUs, V1 and V2 up to 131,072), above it
    # the tiles: both sides of each edge.
    _ilv_check(orc, G, variant_name, variant, ns, 44, sigma=6)


def test_interleaved_few_streams_resolved(G, torch):
    if torch.cuda.get_device_properties(0).multi_processor_count != 256:
        pytest.skip("the band edge is stated for 256 compute units")
    cases = [(1024, "v0", (64, 32, 5)), (81920, "v0", (64, 32, 5)), (81952, "v0", (1024, 16, 10)),
             (131072, "v2", (64, 32, 5)), (131072, "v1", (64, 32, 5)), (131072, "v4", (64, 32, 5)),
             (131104, "v2", (1024, 16, 10)), (131104, "v1", (256, 32, 10)), (65536, "v3", (256, 16, 10)),
             (65568, "v3", (512, 16, 10))]
    for ns, name, want in cases:
        g = G.Generator(ns, name, seed=0, interleaved=True)
        try:
            cfg = g.resolved_tuning(1024)
            assert cfg["source"] == "default", (ns, name, cfg)
            assert (cfg["block"], cfg["unroll"], cfg["store"]) == want, (ns, name, cfg)
        finally:
            g.close()


@pytest.mark.parametrize("store", [2, 4, 1])
@pytest.mark.parametrize("block,unroll", [(256, 64), (512, 32), (1024, 16), (1024, 8), (256, 8)])
def test_interleaved_tiles(orc, G, store, block, unroll):
    # 3008 streams: a partial last tile (whole V2 groups); n = 1003: rounds
    # plus a tail of single steps; two calls continue the streams.
    for name, variant in (("v0", 0), ("v2", 2), ("v1", 1)):
        _ilv_check(orc, G, name, variant, 3008, 1003, sigma=23,
                   tuning=dict(store=store, block=block, unroll=unroll))


@pytest.mark.parametrize("exchange", [1, 2, 3])
def test_interleaved_tiles_v2_exchange(orc, G, exchange):
    _ilv_check(orc, G, "v2", 2, 4096, 512, sigma=24, tuning=dict(exchange=exchange, block=512, unroll=16))


@pytest.mark.parametrize("block,unroll", [(1024, 8), (512, 16), (256, 32), (256, 8)])
@pytest.mark.parametrize("exchange", [1, 2, 3])
def test_interleaved_double_buffered_tiles(orc, G, block, unroll, exchange):
    # Two tile buffers: each round's stores overlap the next round's steps;
    # 5,024 streams leave a partial last tile, n = 1003 a tail, and a tile
    # count that is not a multiple of 8 exercises the XCD band map.
    _ilv_check(orc, G, "v2", 2, 5024, 1003, sigma=27,
               tuning=dict(exchange=exchange, block=block, unroll=unroll, streams_per_lane=2, store=4))
    if exchange == 1:
        for name, variant in (("v0", 0), ("v1", 1)):
            _ilv_check(orc, G, name, variant, 5024, 1003, sigma=27,
                       tuning=dict(block=block, unroll=unroll, streams_per_lane=2, store=2))


def test_interleaved_fallbacks(orc, G, torch):
    # n_streams % 4 != 0 and a misaligned output select the per-lane kernel.
    _ilv_check(orc, G, "v0", 0, 1001, 100, sigma=25)
    g = G.Generator(1024, "v0", seed=26, interleaved=True)
    try:
        buf = torch.empty(1024 * 64 + 1, dtype=torch.int32, device="cuda")
        view = buf[1:]
        g.generate(64, out=view)
        want, _ = orc.generate(0, _oracle_states(orc, 0, 26, 1024), 64)
        got = G.as_u32(view).reshape(64, 1024)
        assert np.array_equal(got.T, want)
    finally:
        g.close()


def test_checkpoint_resume(orc, G):
    g = G.Generator(256, "v2", seed=10)
    try:
        g.generate(100)
        snap = g.get_state()
        a = G.as_u32(g.generate(77))
        g.close()
        g = G.Generator(256, "v2", seed=999)
        g.set_state(snap)
        b = G.as_u32(g.generate(77))
        assert np.array_equal(a, b)
        bad = snap.copy()
        bad[3, :4] = 0
        with pytest.raises(Exception):
            g.set_state(bad)
    finally:
        g.close()


# ---------------------------------------------------------------------------
# Paper-shaped run: 2^20 streams x 1,024 outputs (4 GiB), exchange variant,
# seed 1.  First 64 streams in full plus a seeded 1% sample of streams
# expanded to their whole groups of 32.
# ---------------------------------------------------------------------------
def _sample_groups(ns, frac=0.01, group=32, seed=20111223):
    rng = np.random.default_rng(seed)
    picks = rng.choice(ns, size=int(ns * frac), replace=False)
    groups = np.unique(picks // group)
    return np.unique(np.concatenate([np.arange(64) // group, groups]))


@pytest.mark.parametrize("n", [1024, 1000])
def test_v2_paper_shape_sampled(orc, G, torch, n):
    # n = 1000: rows off the 128-byte lines (line-aligned pieces through a ring).
    ns = 1 << 20
    g = G.Generator(ns, "v2", seed=1)
    try:
        out = g.generate(n)
        torch.cuda.synchronize()
        groups = _sample_groups(ns)
        combs = orc.comb_tables(32)
        idx = torch.from_numpy(np.concatenate([np.arange(gr * 32, gr * 32 + 32) for gr in groups])).cuda()
        got = G.as_u32(out.index_select(0, idx))
        for k, gr in enumerate(groups):
            st = orc.seed(2, 1, gr * 32, 32)
            want, _ = orc.generate(2, st, n, comb=combs)
            assert np.array_equal(got[k * 32:(k + 1) * 32], want), f"group {gr}"
        assert len(groups) > 300
        del out
    finally:
        g.close()


@pytest.mark.parametrize("n", [1024, 1000])
@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v1", 1)])
def test_plain_paper_shape_sampled(orc, G, torch, variant_name, variant, n):
    ns = 1 << 20
    g = G.Generator(ns, variant_name, seed=1)
    try:
        out = g.generate(n)
        rng = np.random.default_rng(7)
        streams = np.unique(np.concatenate([np.arange(64), rng.choice(ns, 2000, replace=False),
                                            [ns - 1]]))
        got = G.as_u32(out.index_select(0, torch.from_numpy(streams).cuda()))
        for k, s in enumerate(streams):
            st = orc.seed(variant, 1, int(s), 1)
            want, _ = orc.generate(variant, st, n)
            assert np.array_equal(got[k], want[0]), f"stream {s}"
        del out
    finally:
        g.close()


# ---------------------------------------------------------------------------
# In-kernel consumption: per-stream counts bit-exact.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant_name,variant", [("v0", 0), ("v2", 2), ("v1", 1)])
def test_consume_counts_small(orc, G, variant_name, variant):
    ns, n = 256, 4096
    g = G.Generator(ns, variant_name, seed=3)
    try:
        st = _oracle_states(orc, variant, 3, ns)
        for _ in range(2):
            got = g.consume_qc(n).cpu().numpy().astype(np.uint64)
            want = orc.consume_qc(variant, st, n)
            assert np.array_equal(got, want)
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


@pytest.mark.parametrize("exchange", [1, 2])
@pytest.mark.parametrize("unroll", [8, 16, 32])
def test_consume_exchange_modes(orc, G, exchange, unroll):
    # Cross-lane reads or the per-wave LDS word buffer; a partial last wave
    # (160 streams) and pairs after the last full round (n = 4098).
    ns, n = 160, 4098
    g = G.Generator(ns, "v2", seed=5)
    try:
        g.set_tuning(exchange=exchange, unroll=unroll)
        st = _oracle_states(orc, 2, 5, ns)
        for _ in range(2):
            got = g.consume_qc(n).cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, orc.consume_qc(2, st, n))
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


def test_consume_paper_scale_sampled(orc, G, torch):
    # 2^36 numbers: 2^20 streams x 2^16, exchange variant, seed 3.
    ns, n = 1 << 20, 1 << 16
    g = G.Generator(ns, "v2", seed=3)
    try:
        counts = g.consume_qc(n).cpu().numpy().astype(np.uint64)
        groups = _sample_groups(ns, frac=0.0001)
        combs = orc.comb_tables(32)
        for gr in groups:
            st = orc.seed(2, 3, gr * 32, 32)
            want = orc.consume_qc(2, st, n, comb=combs)
            assert np.array_equal(counts[gr * 32:(gr + 1) * 32], want), f"group {gr}"
        total = int(counts.sum())
        pairs = ns * n // 2
        pi_est = 4 * total / pairs
        sigma = 4 * np.sqrt((np.pi / 4) * (1 - np.pi / 4) / pairs)
        assert abs(pi_est - np.pi) < 6 * sigma
    finally:
        g.close()


@pytest.mark.parametrize("name,variant", [("v2", 2), ("v0", 0), ("v4", 4)])
def test_interleaved_persistent_workgroups(orc, G, name, variant):
    # 2^17 streams in 512 tiles of 256 on one persistent workgroup per CU:
    # each workgroup takes two tiles (its XCD band), rounds plus a tail.
    ns, n = 1 << 17, 200
    _ilv_check(orc, G, name, variant, ns, n, sigma=28,
               tuning=dict(block=256, unroll=16, store=4, streams_per_lane=2, waves_per_cu=1), calls=2)


# ---------------------------------------------------------------------------
# Interleaved layout, four consecutive streams per lane (tuning store 5 / 6):
# no LDS tile; the exchange through a per-wave LDS word buffer.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("store", [5, 6])
@pytest.mark.parametrize("block", [64, 128, 256])
def test_interleaved_quad_lanes(orc, G, store, block):
    # 5,024 streams: a partial last tile and a partial last wave (whole
    # groups); n = 1003: four-step iterations plus a tail; two calls.
    for name, variant in (("v0", 0), ("v2", 2), ("v4", 4)):
        _ilv_check(orc, G, name, variant, 5024, 1003, sigma=29, tuning=dict(store=store, block=block))


@pytest.mark.parametrize("group", [4, 16, 64])
def test_interleaved_quad_lanes_group_sizes(orc, G, group):
    # groups of 4 (one lane), 16 (four lanes) and 64 (sixteen lanes)
    ns, n = 3072, 133
    g = G.Generator(ns, "v2", seed=30, group=group, interleaved=True)
    try:
        g.set_tuning(store=6)
        st = _oracle_states(orc, 2, 30, ns)
        combs = orc.comb_tables(group)
        for _ in range(2):
            got = G.as_u32(g.generate(n))
            want, _ = orc.generate(2, st, n, comb=combs)
            assert np.array_equal(got.T, want)
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


def test_interleaved_quad_lanes_persistent_and_fallbacks(orc, G, torch):
    # persistent workgroups (two per CU) over 2^17 streams
    _ilv_check(orc, G, "v2", 2, 1 << 17, 64, sigma=31, tuning=dict(store=6, waves_per_cu=2))
    # V1 and V3 take the LDS tiles when the quad lanes are asked
    _ilv_check(orc, G, "v1", 1, 1024, 77, sigma=32, tuning=dict(store=6))
    # n_streams % 4 != 0 and a misaligned output select the per-lane kernel
    _ilv_check(orc, G, "v0", 0, 1001, 50, sigma=33, tuning=dict(store=5))
    g = G.Generator(1024, "v0", seed=34, interleaved=True)
    try:
        g.set_tuning(store=5)
        buf = torch.empty(1024 * 64 + 1, dtype=torch.int32, device="cuda")
        g.generate(64, out=buf[1:])
        want, _ = orc.generate(0, _oracle_states(orc, 0, 34, 1024), 64)
        assert np.array_equal(G.as_u32(buf[1:]).reshape(64, 1024).T, want)
    finally:
        g.close()


def test_quad_store_modes_rejected_for_stream_major(G):
    from paper_1112_5239_amd import _lib as L
    g = G.Generator(64, "v0", seed=0)
    try:
        with pytest.raises(L.CprngError) as e:
            g.set_tuning(store=5)
        assert e.value.status == L.E_INVAL
    finally:
        g.close()
