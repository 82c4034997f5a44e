"""Per-stream seeds (CPRNG_F_SEED_PER_STREAM): stream s starts its SplitMix64
counter at seeds[s]; the oracle seeds one stream of base seed sigma, index j
at counter sigma*2^32 + j, so seeds[s] = sigma_s*2^32 + j_s must reproduce
those states, and seeds[s] = sigma*2^32 + s the single-seed handle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1112_5239_amd import generator
    return generator


@pytest.mark.parametrize("name,ov,kw", [("v0", 0, {}), ("v1", 1, {}), ("v1", 1, {"w32": True}), ("v2", 2, {}),
                                        ("v3", 3, {}), ("v4", 4, {})])
def test_per_stream_seeds_match_the_oracle(orc, G, name, ov, kw):
    ns = 64
    rng = np.random.default_rng(7)
    sig = rng.integers(0, 2**31, size=ns)
    idx = rng.integers(0, 2**32, size=ns)
    seeds = [int(a) * 2**32 + int(b) for a, b in zip(sig, idx)]
    W = 32 if kw.get("w32") else 64
    g = G.Generator(ns, name, seeds=seeds, **kw)
    try:
        got = g.get_state()
        assert got.nbytes == G.L.cprng_state_bytes(g.h)
    finally:
        g.close()
    for s in range(ns):
        want = orc.seed(ov, int(sig[s]), int(idx[s]), 1, W=W)
        assert np.array_equal(got[s], want[0]), f"stream {s}"


def test_per_stream_seeds_reproduce_the_single_seed_rule(G):
    ns = 256
    a = G.Generator(ns, "v2", seed=5)
    b = G.Generator(ns, "v2", seeds=[5 * 2**32 + s for s in range(ns)])
    try:
        assert np.array_equal(a.get_state(), b.get_state())
        assert np.array_equal(G.as_u32(a.generate(100)), G.as_u32(b.generate(100)))
    finally:
        a.close()
        b.close()
