"""GPU parity of batched uneven runs for the exchange variants (V2, V4).

Every group of C streams runs its own length (equal within the group); long
runs are split into chunks that start from a state reached by the group
jump-ahead (X^J modulo the minimal polynomial of the group's one-step map).
Each stream's run and every end state are compared bit for bit with the
oracle generating that group alone, with chunk lengths small enough that
runs cross many chunk boundaries.
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


def _group_lengths(n_groups, seed, cap):
    rng = np.random.default_rng(seed)
    base = np.array([0, 1, 3, 63, 64, 65, 1000, cap], dtype=np.uint64)
    extra = rng.integers(0, cap + 1, size=max(0, n_groups - base.size)).astype(np.uint64)
    return rng.permutation(np.concatenate([base, extra]))[:n_groups]


def _run(orc, G, name, ov, ns, Cg, gl, sigma, chunk, comb=None, offsets_mode=None, calls=2, rnd=0, blk=0):
    g = G.Generator(ns, name, seed=sigma, group=Cg, comb=comb)
    try:
        if chunk or rnd or blk:
            g.set_tuning(chunk=chunk, unroll=rnd, block=blk)
        combs = comb if comb is not None else orc.comb_tables(Cg)
        st = orc.seed(ov, sigma, 0, ns)
        lengths = np.repeat(gl, Cg).astype(np.uint64)
        offsets = None
        if offsets_mode == "reversed":
            # streams laid out last-first with a gap of 5 words between runs
            offsets = np.zeros(ns, dtype=np.uint64)
            pos = 0
            for s in reversed(range(ns)):
                offsets[s] = pos
                pos += int(lengths[s]) + 5
        for _ in range(calls):
            out = G.as_u32(g.generate_ragged(lengths, offsets=offsets))
            offs = offsets if offsets is not None else np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
            for gi in range(ns // Cg):
                rows = slice(gi * Cg, (gi + 1) * Cg)
                sub = st[rows].copy()
                want, _ = orc.generate(ov, sub, int(gl[gi]), comb=combs)
                st[rows] = sub
                for j in range(Cg):
                    s = gi * Cg + j
                    got = out[int(offs[s]):int(offs[s]) + int(lengths[s])]
                    assert np.array_equal(got, want[j]), f"group {gi} stream {j} (length {int(gl[gi])})"
            assert np.array_equal(g.get_state(), st), "end states differ"
    finally:
        g.close()


@pytest.mark.parametrize("name,ov", [("v2", 2), ("v4", 4)])
@pytest.mark.parametrize("chunk", [64, 512, 0])
def test_group_ragged_matches_the_oracle(orc, G, name, ov, chunk):
    gl = _group_lengths(16, 81, 3000)
    _run(orc, G, name, ov, 16 * 32, 32, gl, sigma=81, chunk=chunk)


@pytest.mark.parametrize("name,ov", [("v2", 2), ("v4", 4)])
@pytest.mark.parametrize("Cg", [4, 8, 16, 64])
def test_group_ragged_group_sizes(orc, G, name, ov, Cg):
    gl = _group_lengths(8, 82 + Cg, 2000)
    _run(orc, G, name, ov, 8 * Cg, Cg, gl, sigma=82, chunk=128)


def test_group_ragged_custom_arrays_and_offsets(orc, G):
    c1 = np.array([3, 4, 0, 1, 7, 6, 2, 5], dtype=np.uint32)
    c2 = np.array([1, 3, 4, 2, 0, 7, 5, 6], dtype=np.uint32)
    gl = _group_lengths(12, 83, 1500)
    _run(orc, G, "v2", 2, 96, 8, gl, sigma=83, chunk=192, comb=(c1, c2), offsets_mode="reversed")


@pytest.mark.parametrize("name,ov", [("v2", 2), ("v4", 4)])
@pytest.mark.parametrize("rnd", [32, 64, 128])
@pytest.mark.parametrize("blk", [64, 256])
def test_group_ragged_store_rounds(orc, G, name, ov, rnd, blk):
    # each store-round length and workgroup size, runs misaligned by the 5-word gaps
    gl = _group_lengths(10, 86, 2500)
    _run(orc, G, name, ov, 10 * 16, 16, gl, sigma=86, chunk=320, offsets_mode="reversed", rnd=rnd, blk=blk)


def test_group_ragged_long_run(orc, G):
    # one group far longer than the others: 200 chunks of 1024 steps
    gl = np.array([204800, 10, 0, 4096], dtype=np.uint64)
    _run(orc, G, "v2", 2, 128, 32, gl, sigma=84, chunk=1024, calls=1)


def test_group_ragged_rejects_unequal_lengths_within_a_group(G):
    from paper_1112_5239_amd import _lib as L
    g = G.Generator(64, "v2", seed=85)
    try:
        lengths = np.full(64, 10, dtype=np.uint64)
        lengths[5] = 11
        with pytest.raises(L.CprngError) as e:
            g.generate_ragged(lengths)
        assert e.value.status == L.E_INVAL
    finally:
        g.close()


@pytest.mark.parametrize("shift", [1, 2, 3, 17])
@pytest.mark.parametrize("rnd", [32, 64, 128])
def test_group_ragged_misaligned_output_base(orc, G, rnd, shift):
    # the output pointer itself off its lines by `shift` words: each stream's
    # first line starts at its own column of the store ring
    import torch
    Cg = 16
    gl = _group_lengths(6, 87 + shift, 1800)
    ns = gl.size * Cg
    lengths = np.repeat(gl, Cg).astype(np.uint64)
    total = int(lengths.sum())
    g = G.Generator(ns, "v2", seed=87, group=Cg)
    try:
        g.set_tuning(chunk=256, unroll=rnd, block=256)
        buf = torch.zeros(total + 64, dtype=torch.int32, device="cuda")
        view = buf[shift:shift + total]
        g.generate_ragged(lengths, out=view)
        got = G.as_u32(buf)
        st = orc.seed(2, 87, 0, ns)
        combs = orc.comb_tables(Cg)
        pos = shift
        for gi in range(gl.size):
            sub = st[gi * Cg:(gi + 1) * Cg].copy()
            want, _ = orc.generate(2, sub, int(gl[gi]), comb=combs)
            for j in range(Cg):
                L = int(gl[gi])
                assert np.array_equal(got[pos:pos + L], want[j]), f"group {gi} stream {j}"
                pos += L
        assert not got[:shift].any() and not got[shift + total:].any(), "words outside the runs were written"
    finally:
        g.close()
