"""Bit-exact checks of the configurations the benchmark times, at their full sizes
and in the launch configuration it uses (default tuning, automatic chunk length).

- Paper-shaped exchange variant (Algorithm 4, Section 6.2): 2^20 streams x
  1,024 outputs, seed 1, interleaved layout out[i * 2^20 + s] (the collision-free
  reading of the store index NumThreads*threadId+i with NumThreads the thread
  count): 1,024 banded tiles of 1,024 streams, a 4 GiB output.  The first 64
  streams and a seeded 1% sample of streams, expanded to their whole groups of
  32, are read back as columns and compared element by element with the oracle
  generating each group alone; end states too; then a second call (the
  benchmark repeats the call, so streams continue).
- The plain variants at the same shape and layout (V0 and Listing 1's V1) and
  the xor64 and BBS exchange variants (V4, V3): sampled streams / groups.
- Batched uneven streams of Listing 1 (V1): 4,096 streams with log-uniform
  lengths in [1e3, 1e7] (4.5e9 outputs, word offsets above 2^32), seed 2,
  automatic chunk: a 1% sample plus the longest and shortest streams, over two
  calls, and their end states.
- Batched uneven runs of the exchange variant (V2) in 128 groups of 32 with
  log-uniform group lengths: a 1% sample of groups plus the longest and shortest,
  over two calls, and their end states.
- The plain variant's batched workload (4,096 streams, the same lengths) as a
  device-described subset: a 1% sample plus the longest and shortest streams,
  over two calls, and their end states.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NS, N = 1 << 20, 1024


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


def _sample_groups(ns, group, frac, seed):
    """Groups holding the first 64 streams, the last stream and a seeded sample
    of `frac` of the streams."""
    rng = np.random.default_rng(seed)
    picks = rng.choice(ns, size=max(1, int(ns * frac)), replace=False)
    return np.unique(np.concatenate([np.arange(64) // group, picks // group, [(ns - 1) // group]]))


def _check_interleaved_groups(orc, G, torch, out, groups, group, variant, st_all, combs):
    """Columns of the sampled groups against the oracle; advances st_all in place."""
    cols = np.concatenate([np.arange(gr * group, (gr + 1) * group) for gr in groups])
    got = G.as_u32(out.index_select(1, torch.from_numpy(cols).cuda()))      # (N, k)
    assert got.shape == (N, cols.size)
    for k, gr in enumerate(groups):
        rows = slice(int(gr) * group, (int(gr) + 1) * group)
        sub = st_all[rows].copy()
        want, _ = orc.generate(variant, sub, N, comb=combs)
        st_all[rows] = sub
        bad = np.argwhere(got[:, k * group:(k + 1) * group].T != want)
        assert bad.size == 0, f"group {gr}: first mismatch (stream in group, step) {bad[:3].tolist()}"
    return cols


def _headline(orc, G, torch, name, variant, group, combs, frac, calls=2):
    g = G.Generator(NS, name, seed=1, interleaved=True)
    try:
        assert g.get_tuning() == {k: 0 for k in g.get_tuning()}, "default tuning expected"
        out = torch.empty((N, NS), dtype=torch.int32, device="cuda")
        groups = _sample_groups(NS, group, frac, seed=20111223 + variant)
        st_all = np.zeros((NS, orc.state_words(variant)), dtype=np.uint32)
        for gr in groups:
            st_all[int(gr) * group:(int(gr) + 1) * group] = orc.seed(variant, 1, int(gr) * group, group)
        for _ in range(calls):
            g.generate(N, out=out)
            torch.cuda.synchronize()
            cols = _check_interleaved_groups(orc, G, torch, out, groups, group, variant, st_all, combs)
        dev = g.get_state()
        assert np.array_equal(dev[cols], st_all[cols]), "end states differ"
        del out
        return len(groups)
    finally:
        g.close()


def test_headline_v2_interleaved_full_size(orc, G, torch):
    # The configuration bench.py's headline times, exactly: default tuning
    # (1,024-stream x 16-step double-buffered tiles, LDS word exchange,
    # non-temporal stores, XCD-banded tile map).
    n_groups = _headline(orc, G, torch, "v2", 2, 32, orc.comb_tables(32), frac=0.01)
    assert n_groups > 5000          # 1% of 2^20 streams lands in ~9,000 of the 32,768 groups


@pytest.mark.parametrize("name,variant,group,frac", [("v0", 0, 1, 0.002), ("v1", 1, 1, 0.002),
                                                     ("v4", 4, 32, 0.002), ("v3", 3, 32, 0.0002)])
def test_other_variants_interleaved_full_size(orc, G, torch, name, variant, group, frac):
    combs = None
    if variant == 4:
        combs = orc.comb_tables(32)
    elif variant == 3:
        combs = orc.bbs_comb_tables(32)
    _headline(orc, G, torch, name, variant, group, combs, frac=frac)


def _stream_sample(lengths, frac, seed):
    from paper_1112_5239_amd import workloads
    ns = lengths.size
    return np.unique(np.concatenate([workloads.parity_sample(ns, frac, seed),
                                     [int(np.argmax(lengths)), int(np.argmin(lengths)), 0, ns - 1]]))


@pytest.mark.parametrize("tuned", [False, True])
def test_batched_v1_full_workload_auto_chunk(orc, G, torch, tuned):
    # default configuration, then the configuration the autotuner picks on
    # this workload (what bench.py's batched leg times)
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_lengths()
    ns = lengths.size
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    total = int(lengths.sum())
    assert total > (1 << 32)
    g = G.Generator(ns, "v1", seed=2)
    try:
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        if tuned:
            g.autotune_ragged(lengths, out=out)
            assert g.resolved_tuning_ragged(lengths)["source"] == "autotuned"
        pick = _stream_sample(lengths, 0.01, 101)
        st = orc.seed(1, 2, 0, ns)
        for call in range(2):
            g.generate_ragged(lengths, out=out)
            torch.cuda.synchronize()
            for s in pick:
                o, L = int(offs[s]), int(lengths[s])
                got = G.as_u32(out[o:o + L])
                one = st[s:s + 1].copy()
                want, _ = orc.generate(1, one, L)
                st[s] = one[0]
                bad = np.flatnonzero(got != want[0])
                assert bad.size == 0, f"call {call} stream {s} (length {L}): first mismatch at {bad[:3].tolist()}"
        assert np.array_equal(g.get_state()[pick], st[pick]), "end states differ"
        del out
    finally:
        g.close()


@pytest.mark.parametrize("tuned", [False, True])
def test_batched_v2_groups_full_workload_auto_chunk(orc, G, torch, tuned):
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_group_lengths()
    ns, Cg = lengths.size, 32
    gl = lengths[::Cg]
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    total = int(lengths.sum())
    combs = orc.comb_tables(Cg)
    g = G.Generator(ns, "v2", seed=2)
    try:
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        if tuned:
            g.autotune_ragged(lengths, out=out)
            assert g.resolved_tuning_ragged(lengths)["source"] == "autotuned"
        groups = np.unique(np.concatenate([workloads.parity_sample(gl.size, 0.01, 102),
                                           [int(np.argmax(gl)), int(np.argmin(gl))]]))
        st = orc.seed(2, 2, 0, ns)
        for call in range(2):
            g.generate_ragged(lengths, out=out)
            torch.cuda.synchronize()
            for gi in groups:
                rows = slice(int(gi) * Cg, (int(gi) + 1) * Cg)
                sub = st[rows].copy()
                L = int(gl[gi])
                want, _ = orc.generate(2, sub, L, comb=combs)
                st[rows] = sub
                o = int(offs[int(gi) * Cg])
                got = G.as_u32(out[o:o + Cg * L]).reshape(Cg, L)
                bad = np.argwhere(got != want)
                assert bad.size == 0, f"call {call} group {gi} (length {L}): first mismatch {bad[:3].tolist()}"
        rows = np.concatenate([np.arange(int(gi) * Cg, (int(gi) + 1) * Cg) for gi in groups])
        assert np.array_equal(g.get_state()[rows], st[rows]), "end states differ"
        del out
    finally:
        g.close()


def test_batched_v0_device_subset_full_workload(orc, G, torch):
    # The batched workload's 4,096 runs as a device-described subset
    # (cprng_generate_subset, default tuning), as the benchmark's ragged leg
    # times it: a 1% sample plus the longest and shortest streams, two calls.
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_lengths()
    ns = lengths.size
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    total = int(lengths.sum())
    g = G.Generator(ns, "v0", seed=2)
    try:
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        ids = torch.arange(ns, dtype=torch.int32, device="cuda")
        lens = torch.tensor(lengths.astype(np.int64), device="cuda")
        t_offs = torch.cumsum(lens, 0) - lens
        status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        pick = _stream_sample(lengths, 0.01, 103)
        st = orc.seed(0, 2, 0, ns)
        for call in range(2):
            g.generate_subset(ids, lens, t_offs, out, status)
            torch.cuda.synchronize()
            assert int(status.item()) == 0
            for s in pick:
                o, L = int(offs[s]), int(lengths[s])
                got = G.as_u32(out[o:o + L])
                one = st[s:s + 1].copy()
                want, _ = orc.generate(0, one, L)
                st[s] = one[0]
                bad = np.flatnonzero(got != want[0])
                assert bad.size == 0, f"call {call} stream {s} (length {L}): first mismatch at {bad[:3].tolist()}"
        assert np.array_equal(g.get_state()[pick], st[pick]), "end states differ"
        del out
    finally:
        g.close()
