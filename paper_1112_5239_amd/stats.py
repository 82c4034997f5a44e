"""A small statistical smoke battery for uint32 outputs.

A sanity check that catches gross defects (stuck or biased bits, skewed
bytes, correlated successive words, correlated neighbouring streams), not a
substitute for a full battery such as TestU01's BigCrush, which the paper
runs (Section 8) and which is not available here.

Every test returns a p-value under the hypothesis that the words are
independent and uniform on [0, 2^32); `battery` runs them all.  Host-side
numpy only: the words come from wherever the caller generated them.
"""
import numpy as np
from scipy import special, stats


def _u32(words):
    return np.ascontiguousarray(words, dtype=np.uint32).reshape(-1)


def _bit_counts(w):
    """Ones at each of the 32 bit positions."""
    b = np.unpackbits(w.view(np.uint8).reshape(-1, 4), axis=1, bitorder="little")
    return b.sum(axis=0, dtype=np.int64).reshape(4, 8).reshape(32)


def monobit(words) -> float:
    """Frequency test over all bits: the count of ones against N/2."""
    w = _u32(words)
    n = 32 * w.size
    ones = int(_bit_counts(w).sum())
    z = (ones - n / 2) / np.sqrt(n / 4)
    return float(special.erfc(abs(z) / np.sqrt(2)))


def bit_positions(words) -> float:
    """Each of the 32 bit positions balanced: chi-square, 32 degrees of freedom."""
    w = _u32(words)
    c = _bit_counts(w).astype(np.float64)
    z = (c - w.size / 2) / np.sqrt(w.size / 4)
    return float(stats.chi2.sf(float(np.sum(z * z)), 32))


def byte_chi2(words) -> float:
    """The 256 byte values equally likely (all four bytes of every word):
    chi-square, 255 degrees of freedom."""
    w = _u32(words)
    h = np.bincount(w.view(np.uint8), minlength=256).astype(np.float64)
    e = h.sum() / 256
    return float(stats.chi2.sf(float(np.sum((h - e) ** 2 / e)), 255))


def serial_correlation(words) -> float:
    """Lag-1 correlation of successive words of each row (as uniforms): for
    independent words sqrt(n) * r is close to standard normal."""
    w = np.atleast_2d(np.asarray(words, dtype=np.uint32))
    u = w.astype(np.float64) / 2.0 ** 32 - 0.5
    a, b = u[:, :-1].reshape(-1), u[:, 1:].reshape(-1)
    r = float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))
    z = r * np.sqrt(a.size)
    return float(special.erfc(abs(z) / np.sqrt(2)))


def cross_correlation(words) -> float:
    """Correlation of each row with the next row at the same step (rows are
    streams: neighbouring streams, e.g. members of one exchange group)."""
    w = np.atleast_2d(np.asarray(words, dtype=np.uint32))
    if w.shape[0] < 2:
        return 1.0
    u = w.astype(np.float64) / 2.0 ** 32 - 0.5
    a, b = u[:-1].reshape(-1), u[1:].reshape(-1)
    r = float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))
    z = r * np.sqrt(a.size)
    return float(special.erfc(abs(z) / np.sqrt(2)))


TESTS = {
    "monobit": monobit,
    "bit_positions": bit_positions,
    "byte_chi2": byte_chi2,
    "serial_correlation": serial_correlation,
    "cross_correlation": cross_correlation,
}


def battery(words) -> dict:
    """p-value of every test; words is (streams, steps) or flat."""
    return {name: f(words) for name, f in TESTS.items()}


def passes(pvalues: dict, alpha: float = 1e-6) -> bool:
    """True iff no p-value lies in either tail of width alpha."""
    return all(alpha < p < 1 - alpha for p in pvalues.values())
