"""Seeded synthetic inputs of the benchmark workloads.

This module holds input recipes only (stream lengths, request arrivals and
sizes, parity samples); none of the generator's arithmetic.  Both the tests
and the benchmark draw their inputs from here.
"""
import numpy as np

# Batched uneven streams: 4,096 streams, lengths log-uniform in [1e3, 1e7].
RAGGED_STREAMS = 4096
RAGGED_LO, RAGGED_HI = 1e3, 1e7
RAGGED_SEED = 2


def ragged_lengths(n_streams: int = RAGGED_STREAMS, lo: float = RAGGED_LO, hi: float = RAGGED_HI,
                   seed: int = RAGGED_SEED) -> np.ndarray:
    """floor(lo * (hi/lo)^u), u uniform in [0,1) from numpy's PCG64 seeded with `seed`."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_streams)
    return np.floor(lo * np.power(hi / lo, u)).astype(np.uint64)


def ragged_group_lengths(n_groups: int = 128, group: int = 32, lo: float = RAGGED_LO, hi: float = RAGGED_HI,
                         seed: int = RAGGED_SEED) -> np.ndarray:
    """Per-stream lengths of batched uneven runs of the exchange variants: n_groups
    group lengths exp(U(ln lo, ln hi)) truncated to integers (numpy PCG64 seeded with
    `seed`), each repeated for the `group` streams of its group (a group's streams
    advance together)."""
    rng = np.random.default_rng(seed)
    gl = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_groups)).astype(np.uint64)
    return np.repeat(gl, group).astype(np.uint64)


def serving_trace(rate_hz: float = 2000.0, duration_s: float = 60.0, n_clients: int = 10000,
                  min_bytes: int = 1024, max_bytes: int = 256 << 20, seed: int = 5):
    """Poisson arrivals with log-uniform request sizes (bytes, multiple of 4).

    Returns (arrival_ns uint64, client uint32, n_numbers uint64), sorted by
    arrival time.
    """
    rng = np.random.default_rng(seed)
    expected = int(rate_hz * duration_s)
    gaps = rng.exponential(1.0 / rate_hz, size=expected + 8 * int(np.sqrt(expected) + 10))
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    n = t.size
    u = rng.random(n)
    size_bytes = np.floor(min_bytes * np.power(max_bytes / min_bytes, u)).astype(np.uint64)
    numbers = np.maximum(size_bytes // 4, 1).astype(np.uint64)
    clients = rng.integers(0, n_clients, size=n, dtype=np.uint32)
    return (t * 1e9).astype(np.uint64), clients, numbers


def parity_sample(n_items: int, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = max(1, int(n_items * frac))
    return np.sort(rng.choice(n_items, size=k, replace=False))
