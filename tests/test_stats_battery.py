"""The statistical smoke battery: it must reject gross defects (pinned on
sequences with known flaws) and accept the oracle's outputs of every variant.
The GPU outputs go through the same battery in the GPU tests."""
import numpy as np
import pytest

from paper_1112_5239_amd import stats


def _uniform(n, seed=1):
    return np.random.default_rng(seed).integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)


def test_accepts_independent_uniform_words():
    p = stats.battery(_uniform(1 << 20).reshape(256, 4096))
    assert stats.passes(p), p


def test_rejects_biased_bits():
    w = _uniform(1 << 18) | np.uint32(1 << 31)          # top bit stuck at 1
    assert stats.bit_positions(w) < 1e-6
    assert stats.monobit(w) < 1e-6


def test_rejects_skewed_bytes():
    w = _uniform(1 << 18) & np.uint32(0xFFFFFF7F)       # bit 7 of byte 0 never set
    assert stats.byte_chi2(w) < 1e-6


def test_rejects_correlated_successive_words():
    w = _uniform(1 << 18, seed=2)
    w[1::2] = w[0::2] ^ (_uniform(1 << 17, seed=3) & np.uint32(0xFFFF))   # every other word repeats the high half
    assert stats.serial_correlation(w.reshape(64, -1)) < 1e-6
    counter = np.arange(1 << 18, dtype=np.uint32) * np.uint32(16411)
    assert stats.serial_correlation(counter) < 1e-6


def test_rejects_correlated_streams():
    w = _uniform(1 << 18).reshape(64, -1)
    w[1::2] = w[0::2] ^ np.uint32(1)                    # odd streams copy even ones
    assert stats.cross_correlation(w) < 1e-6


@pytest.mark.parametrize("variant,extra", [(0, {}), (1, {}), (2, {}), (3, {}), (4, {}), (1, {"xor64": True})])
def test_oracle_outputs_pass(orc, variant, extra):
    ov = variant | (orc.F_XOR64 if extra.get("xor64") else 0)
    ns, n = 256, 4096
    st = orc.seed(ov, 99, 0, ns)
    out, _ = orc.generate(ov, st, n)
    p = stats.battery(out)
    assert stats.passes(p), p
