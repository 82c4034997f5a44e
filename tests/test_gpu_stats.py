"""The statistical smoke battery on device outputs: every variant, 4,096
streams x 1,024 steps (stream-major rows), and a slice of the paper-shaped
interleaved V2 run read back as streams."""
import numpy as np
import pytest

from paper_1112_5239_amd import stats

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


@pytest.mark.parametrize("name,kw", [("v0", {}), ("v1", {}), ("v1", {"v1_xor64": True}), ("v1", {"w32": True}),
                                     ("v2", {}), ("v3", {}), ("v4", {})])
def test_battery_on_device_outputs(G, name, kw):
    g = G.Generator(4096, name, seed=123, **kw)
    try:
        w = G.as_u32(g.generate(1024))
    finally:
        g.close()
    p = stats.battery(w)
    assert stats.passes(p), p


def test_battery_on_paper_shaped_slice(G, torch):
    ns, n = 1 << 20, 1024
    g = G.Generator(ns, "v2", seed=1, interleaved=True)
    try:
        out = g.generate(n)
        torch.cuda.synchronize()
        w = G.as_u32(out[:, 123456:123456 + 4096].cpu()).T     # 4,096 consecutive streams
    finally:
        g.close()
    p = stats.battery(w)
    assert stats.passes(p), p
