"""GPU parity of the chunked plain-variant paths: batched uneven streams
(persistent kernel in a hipGraph) and request batches.

Each stream's numbers must equal that stream generated alone by the oracle,
whatever the chunking, alignment and grouping of requests.
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


def _oracle_runs(orc, sigma, streams, lengths):
    """Oracle: each listed stream generated alone, lengths[i] outputs."""
    res = []
    for s, L in zip(streams, lengths):
        st = orc.seed(0, sigma, int(s), 1)
        o, _ = orc.generate(0, st, int(L))
        res.append(o[0])
    return res


def _check_ragged(orc, G, torch, lengths, offsets=None, sigma=2, tuning=None, calls=1, pad=0):
    ns = len(lengths)
    lengths = np.asarray(lengths, dtype=np.uint64)
    g = G.Generator(ns, "v0", seed=sigma)
    try:
        if tuning:
            g.set_tuning(**tuning)
        if offsets is None:
            offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
        else:
            offs = np.asarray(offsets, dtype=np.uint64)
        total = int((offs + lengths).max()) + pad
        out = torch.zeros(total + 1, dtype=torch.int32, device="cuda")
        st = orc.seed(0, sigma, 0, ns)
        for _ in range(calls):
            out.zero_()
            g.generate_ragged(lengths, offsets, out=out)
            host = G.as_u32(out)
            covered = np.zeros(total + 1, dtype=bool)
            for s in range(ns):
                want, _ = orc.generate(0, st[s:s + 1], int(lengths[s]))
                o, L = int(offs[s]), int(lengths[s])
                assert np.array_equal(host[o:o + L], want[0]), f"stream {s} (len {L}, off {o})"
                covered[o:o + L] = True
            assert not host[~covered].any(), "wrote outside the runs"
        assert np.array_equal(g.get_state(), st), "end states differ"
    finally:
        g.close()


def test_ragged_small_default_offsets(orc, G, torch):
    rng = np.random.default_rng(1)
    _check_ragged(orc, G, torch, rng.integers(0, 5000, 100))


@pytest.mark.parametrize("chunk", [64, 256, 1024])
@pytest.mark.parametrize("store,unroll", [(1, 16), (2, 32), (4, 64), (2, 128), (2, 256), (7, 64), (8, 128),
                                          (7, 256)])
def test_ragged_many_chunks_jump_ahead(orc, G, torch, chunk, store, unroll):
    # Small chunks force many jumped segment starts per stream; per-lane and
    # LDS-tiled stores, tiles longer and shorter than the chunks.
    rng = np.random.default_rng(chunk)
    lengths = rng.integers(1, 20000, 70)
    _check_ragged(orc, G, torch, lengths,
                  tuning=dict(chunk=chunk, unroll=unroll, waves_per_cu=2, store=store))


@pytest.mark.parametrize("store", [1, 4, 7])
def test_ragged_explicit_misaligned_offsets_with_gaps(orc, G, torch, store):
    rng = np.random.default_rng(3)
    lengths = rng.integers(0, 3000, 50)
    lengths[[3, 17]] = 0
    order = rng.permutation(50)
    offs = np.zeros(50, dtype=np.uint64)
    pos = 1
    for s in order:
        offs[s] = pos
        pos += int(lengths[s]) + int(rng.integers(0, 7))
    _check_ragged(orc, G, torch, lengths, offsets=offs, tuning=dict(chunk=512, store=store), pad=5)


def test_ragged_graph_replay_continues_streams(orc, G, torch):
    rng = np.random.default_rng(4)
    _check_ragged(orc, G, torch, rng.integers(1, 40000, 64), calls=3, tuning=dict(chunk=2048))


def test_ragged_rejects_bbs_and_interleaved(G):
    # The BBS variant has no jump-ahead; the interleaved layout no ragged form.
    from paper_1112_5239_amd import CprngError
    for v, kw in (("v3", {}), ("v0", {"interleaved": True})):
        g = G.Generator(64, v, seed=0, **kw)
        try:
            with pytest.raises(CprngError) as e:
                g.generate_ragged(np.full(64, 10, dtype=np.uint64))
            assert e.value.status == -4
        finally:
            g.close()


def test_ragged_paper_shape_sampled(orc, G, torch):
    # 4,096 streams, lengths log-uniform in [1e3, 1e7] (about 4.5e9 numbers,
    # 18 GB), one graph launch; sampled streams checked in full.
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_lengths()
    ns = lengths.size
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    total = int(lengths.sum())
    g = G.Generator(ns, "v0", seed=2)
    try:
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        g.generate_ragged(lengths, out=out)
        torch.cuda.synchronize()
        pick = np.unique(np.concatenate([workloads.parity_sample(ns, 0.01, 99),
                                         [int(np.argmax(lengths)), int(np.argmin(lengths)), 0, ns - 1]]))
        st = orc.seed(0, 2, 0, ns)
        for s in pick:
            o, L = int(offs[s]), int(lengths[s])
            got = G.as_u32(out[o:o + L])
            want, _ = orc.generate(0, st[s:s + 1].copy(), L)
            assert np.array_equal(got, want[0]), f"stream {s}"
        del out
    finally:
        g.close()


def test_requests_multiple_per_stream_and_misaligned(orc, G, torch):
    ns = 40
    g = G.Generator(ns, "v0", seed=11)
    try:
        rng = np.random.default_rng(5)
        st = orc.seed(0, 11, 0, ns)
        for call in range(3):
            reqs, bufs, plan = [], [], []
            for r in range(60):
                s = int(rng.integers(0, ns // 2))        # streams >= ns/2 stay untouched
                L = int(rng.integers(0, 9000))
                b = torch.zeros(L + 8, dtype=torch.int32, device="cuda")
                shift = int(rng.integers(0, 4))
                reqs.append((s, L, b.data_ptr() + 4 * shift))
                bufs.append((b, shift))
                plan.append((s, L))
            g.generate_requests(reqs)
            torch.cuda.synchronize()
            # expected: per stream, requests in order, consecutive outputs
            per_stream = {}
            for s, L in plan:
                per_stream.setdefault(s, []).append(L)
            want_by_stream = {}
            for s, Ls in per_stream.items():
                o, _ = orc.generate(0, st[s:s + 1], sum(Ls))
                want_by_stream[s] = o[0]
                # st[s] advanced in place
            cursor = {s: 0 for s in per_stream}
            for (s, L), (b, shift) in zip(plan, bufs):
                got = G.as_u32(b)
                c = cursor[s]
                assert np.array_equal(got[shift:shift + L], want_by_stream[s][c:c + L]), f"call {call} stream {s}"
                assert not got[:shift].any() and not got[shift + L:].any()
                cursor[s] = c + L
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()


def test_requests_large_single_request(orc, G, torch):
    # One 64M-number request (256 MiB) split over many lanes.
    g = G.Generator(10, "v0", seed=4)
    try:
        n = 64 << 20
        b = torch.empty(n, dtype=torch.int32, device="cuda")
        g.generate_requests([(7, n, b)])
        st = orc.seed(0, 4, 7, 1)
        want, _ = orc.generate(0, st, n)
        assert np.array_equal(G.as_u32(b), want[0])
    finally:
        g.close()


@pytest.mark.parametrize("n_req", [1, 64, 65, 100])
def test_requests_inline_and_staged_batches(orc, G, torch, n_req):
    # Up to 64 runs per launch the batch travels in the kernel arguments,
    # above that through the staged upload; three calls in a row (the queue
    # counters carry over between launches), lengths across several chunks.
    ns = 128
    g = G.Generator(ns, "v0", seed=17)
    try:
        rng = np.random.default_rng(n_req)
        st = orc.seed(0, 17, 0, ns)
        for call in range(3):
            streams = rng.permutation(ns)[:n_req]
            lengths = rng.integers(1, 20000, n_req)
            bufs = [torch.zeros(int(L) + 4, dtype=torch.int32, device="cuda") for L in lengths]
            g.generate_requests([(int(s), int(L), b.data_ptr() + 4) for s, L, b in zip(streams, lengths, bufs)])
            torch.cuda.synchronize()
            for s, L, b in zip(streams, lengths, bufs):
                want, _ = orc.generate(0, st[s:s + 1], int(L))
                got = G.as_u32(b)
                assert np.array_equal(got[1:1 + L], want[0]), f"call {call} stream {s} (length {L})"
                assert got[0] == 0 and not got[1 + L:].any()
        assert np.array_equal(g.get_state(), st)
    finally:
        g.close()
