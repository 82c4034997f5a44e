"""The allocation-free variant of batched uneven streams (V0), through the C ABI.

cprng_generate_ragged_noalloc keeps every work buffer of the chunk kernels in
one file-scope device array.  Its outputs and end states must equal those of
cprng_generate_ragged (the entry point it is a variant of) on the same inputs,
bit for bit, and the oracle's, over two calls in a row whose second input is
smaller (the array keeps the first call's contents); sizes beyond the array
are rejected before any device work.
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


def _offsets(lengths, gap=0, reverse=False):
    offs = np.zeros(lengths.size, dtype=np.uint64)
    pos = 0
    for s in (reversed(range(lengths.size)) if reverse else range(lengths.size)):
        offs[s] = pos
        pos += int(lengths[s]) + gap
    return offs, pos


def _check_calls(orc, G, torch, ns, seed, inputs):
    from paper_1112_5239_amd import _lib as L
    a = G.Generator(ns, "v0", seed=seed)
    b = G.Generator(ns, "v0", seed=seed)
    try:
        st = orc.seed(0, seed, 0, ns)
        for lengths, gap, reverse in inputs:
            offs, size = _offsets(lengths, gap, reverse)
            oa = torch.full((size + 1,), -1, dtype=torch.int32, device="cuda")
            ob = torch.full((size + 1,), -1, dtype=torch.int32, device="cuda")
            a.generate_ragged(lengths, offsets=offs, out=oa)
            L.cprng_generate_ragged_noalloc(b.h, ob, lengths, offs, torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            ga, gb = G.as_u32(oa), G.as_u32(ob)
            assert np.array_equal(ga, gb), "differs from cprng_generate_ragged"
            for s in range(ns):
                o, n = int(offs[s]), int(lengths[s])
                want, _ = orc.generate(0, st[s:s + 1], n)      # advances st[s]
                assert np.array_equal(gb[o:o + n], want[0]), f"stream {s} (length {n})"
            covered = np.zeros(size + 1, dtype=bool)
            for s in range(ns):
                covered[int(offs[s]):int(offs[s]) + int(lengths[s])] = True
            assert np.all(gb[~covered] == 0xFFFFFFFF), "wrote outside the runs"
        assert np.array_equal(b.get_state(), a.get_state())
        assert np.array_equal(b.get_state(), st)
    finally:
        a.close()
        b.close()


def test_noalloc_matches_ragged_two_calls_second_smaller(orc, G, torch):
    rng = np.random.default_rng(7)
    ns = 512
    first = rng.integers(0, 60000, ns).astype(np.uint64)
    first[:4] = [0, 1, 63, 400000]                      # a run of ~200 chunks
    second = (first // 7).astype(np.uint64)
    second[::5] = 0
    _check_calls(orc, G, torch, ns, 31, [(first, 0, False), (second, 0, False)])


def test_noalloc_misaligned_runs_with_gaps(orc, G, torch):
    rng = np.random.default_rng(8)
    ns = 200
    first = rng.integers(0, 9000, ns).astype(np.uint64)
    second = rng.integers(0, 900, ns).astype(np.uint64)
    _check_calls(orc, G, torch, ns, 32, [(first, 3, True), (second, 5, False)])


def test_noalloc_rejects_sizes_beyond_the_array_and_other_variants(G, torch):
    from paper_1112_5239_amd import _lib as L
    ns = 900_000                                       # end-state staging alone: 18 MB > 16 MiB
    g = G.Generator(ns, "v0", seed=33)
    try:
        lengths = np.ones(ns, dtype=np.uint64)
        out = torch.empty(ns, dtype=torch.int32, device="cuda")
        with pytest.raises(L.CprngError) as e:
            L.cprng_generate_ragged_noalloc(g.h, out, lengths, None, torch.cuda.current_stream().cuda_stream)
        assert e.value.status == L.E_INVAL and "scratch" in str(e.value)
    finally:
        g.close()
    g = G.Generator(64, "v1", seed=33)
    try:
        out = torch.empty(640, dtype=torch.int32, device="cuda")
        with pytest.raises(L.CprngError) as e:
            L.cprng_generate_ragged_noalloc(g.h, out, np.full(64, 10, dtype=np.uint64), None,
                                            torch.cuda.current_stream().cuda_stream)
        assert e.value.status == L.E_UNSUPPORTED
    finally:
        g.close()
