"""GPU parity of batched uneven runs for V1 (Listing 1).

Long runs are split into chunks; each chunk jumps the three generators ahead
(GF(2) jump polynomials, the Weyl counter arithmetically) and starts its x
from an aggregate pass over the earlier chunks of its stream.  Every run and
end state is compared bit for bit with the oracle generating each stream
alone, with chunk lengths small enough to cross many chunk boundaries.
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


def _lengths(ns, seed, cap):
    rng = np.random.default_rng(seed)
    base = np.array([0, 1, 3, 31, 32, 33, 63, 64, 65, 1000, cap], dtype=np.uint64)
    extra = rng.integers(0, cap + 1, size=ns - base.size).astype(np.uint64)
    return rng.permutation(np.concatenate([base, extra]))


def _run(orc, G, kw, ov, W, ns, lengths, sigma, chunk, offsets=None, calls=2, rnd=0, blk=0, parts=0):
    g = G.Generator(ns, "v1", seed=sigma, **kw)
    try:
        if chunk or rnd or blk or parts:
            g.set_tuning(chunk=chunk, unroll=rnd, block=blk, streams_per_lane=parts)
        st = orc.seed(ov, sigma, 0, ns, W=W)
        offs = offsets if offsets is not None else np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
        for _ in range(calls):
            out = G.as_u32(g.generate_ragged(lengths, offsets=offsets))
            for s in range(ns):
                one = st[s:s + 1].copy()
                want, _ = orc.generate(ov, one, int(lengths[s]), W=W)
                st[s] = one[0]
                got = out[int(offs[s]):int(offs[s]) + int(lengths[s])]
                assert np.array_equal(got, want[0]), f"stream {s} (length {int(lengths[s])})"
            assert np.array_equal(g.get_state(), st), "end states differ"
    finally:
        g.close()


CASES = [({}, 1, 64), ({"v1_xor64": True}, None, 64), ({"w32": True}, 1, 32)]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("chunk", [64, 1024, 0])
def test_v1_ragged_matches_the_oracle(orc, G, case, chunk):
    kw, ov, W = CASES[case]
    if ov is None:
        ov = 1 | orc.F_XOR64
    lengths = _lengths(128, 91, 5000)
    _run(orc, G, kw, ov, W, 128, lengths, sigma=91, chunk=chunk)


@pytest.mark.parametrize("rnd", [32, 64, 128])
@pytest.mark.parametrize("blk", [64, 256])
def test_v1_ragged_store_rounds(orc, G, rnd, blk):
    # each store-round length and workgroup size, runs misaligned by 3-word gaps
    lengths = _lengths(96, 93, 4000)
    offs = np.zeros(96, dtype=np.uint64)
    pos = 0
    for s in reversed(range(96)):
        offs[s] = pos
        pos += int(lengths[s]) + 3
    _run(orc, G, {}, 1, 64, 96, lengths, sigma=93, chunk=448, offsets=offs, rnd=rnd, blk=blk)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("parts", [1, 2, 4])
@pytest.mark.parametrize("chunk", [64, 320, 0])
def test_v1_ragged_aggregate_lanes(orc, G, case, parts, chunk):
    # lanes per chunk of the aggregate pass (each steps xorwow through its own
    # share of the chunk from its own jump), including shares of 16 and 80 steps
    kw, ov, W = CASES[case]
    if ov is None:
        ov = 1 | orc.F_XOR64
    lengths = _lengths(72, 94, 30000 if chunk == 0 else 3000)
    _run(orc, G, kw, ov, W, 72, lengths, sigma=94, chunk=chunk, parts=parts)


def test_v1_ragged_offsets_and_a_long_run(orc, G):
    lengths = _lengths(64, 92, 3000)
    lengths[7] = 150000                           # 147 chunks of 1,024
    offs = np.zeros(64, dtype=np.uint64)
    pos = 0
    for s in reversed(range(64)):
        offs[s] = pos
        pos += int(lengths[s]) + 3
    _run(orc, G, {}, 1, 64, 64, lengths, sigma=92, chunk=1024, offsets=offs, calls=1)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_v1_requests_multiple_per_stream_and_misaligned(orc, G, torch, case):
    kw, ov, W = CASES[case]
    if ov is None:
        ov = 1 | orc.F_XOR64
    ns = 24
    g = G.Generator(ns, "v1", seed=12, **kw)
    try:
        g.set_tuning(chunk=256)
        rng = np.random.default_rng(6)
        st = orc.seed(ov, 12, 0, ns, W=W)
        for call in range(2):
            reqs, bufs, plan = [], [], []
            for r in range(40):
                s = int(rng.integers(0, ns // 2))        # streams >= ns/2 stay untouched
                L = int(rng.integers(0, 3000))
                b = torch.zeros(L + 8, dtype=torch.int32, device="cuda")
                shift = int(rng.integers(0, 4))
                reqs.append((s, L, b.data_ptr() + 4 * shift))
                bufs.append((b, shift))
                plan.append((s, L))
            g.generate_requests(reqs)
            torch.cuda.synchronize()
            per_stream = {}
            for s, L in plan:
                per_stream.setdefault(s, []).append(L)
            want_by_stream = {}
            for s, Ls in per_stream.items():
                o, _ = orc.generate(ov, st[s:s + 1], sum(Ls), W=W)
                want_by_stream[s] = o[0]
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
