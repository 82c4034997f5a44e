"""Pins of the oracle's xor64 pieces: the V4 variant (Algorithm 4 with xor64
as each thread's generator, the generator Section 7 names for its optimized
versions) and the xor64 alternative for Listing 1's first generator (V1 with
the F_XOR64 flag).

The xor64 triple is pinned by the first outputs of Marsaglia's own xor64
example (which also fixes the order of the shifts against the full-period
mirror triple) and by the primitivity of the recurrence its output bits obey
(a mistyped shift almost surely breaks it); the V4 wiring by a
brute-force lockstep simulation of Algorithm 4, the cancellation of equal
combination arrays and GF(2) linearity; the V1 alternative by composing the
three generators run alone.
"""
import numpy as np
import pytest

from tests import gf2
from tests.test_oracle_pins import _alg4_lockstep, _bits

V4 = 4


def _xor64_words(orc, y0, n):
    out, _ = orc.gen_outputs(3, 64, [int(y0)], n)
    return out.astype(np.uint64)


def test_xor64_marsaglia_example_outputs(orc):
    # Marsaglia, "Xorshift RNGs" (2003): xor64 with shifts left 13, right 7,
    # left 17 from the seed 88172645463325252, whose first outputs are
    # 8748534153485358512, 3040900993826735515, 3453997556048239312; the
    # mirror triple (17, 7, 13) gives other numbers from the first step.
    out = _xor64_words(orc, 88172645463325252, 3)
    assert [int(v) for v in out] == [8748534153485358512, 3040900993826735515, 3453997556048239312]


def test_xor64_primitive_degree_64(orc):
    # Marsaglia's xor64 has period 2^64 - 1: each output bit obeys one
    # primitive recurrence of degree 64.
    out = _xor64_words(orc, 88172645463325252, 512)
    polys = set()
    for b in (0, 17, 40, 63):
        L, Cx = gf2.berlekamp_massey(_bits(out, b))
        assert L == 64
        polys.add(gf2.reciprocal(Cx, L))
    assert len(polys) == 1
    assert gf2.is_primitive(polys.pop())


def test_xor64_is_not_the_alg2_triple(orc):
    # The alternative changes the generator: (13,7,17) and (13,17,5) differ
    # on 64-bit words from the first step.
    a = _xor64_words(orc, 0x0123456789ABCDEF, 4)
    b, _ = orc.gen_outputs(0, 64, [0x0123456789ABCDEF], 4)
    assert not np.array_equal(a, b.astype(np.uint64))


def test_v4_seeding_nonzero_and_reproducible(orc):
    a = orc.seed(V4, 5, 0, 256)
    b = orc.seed(V4, 5, 0, 256)
    assert np.array_equal(a, b)
    assert a.shape == (256, 4)
    assert np.all((a[:, 0] | a[:, 1]) != 0)
    assert len({(int(r[0]), int(r[1])) for r in a}) == 256
    # a stream's seed depends only on (seed, global stream id)
    assert np.array_equal(orc.seed(V4, 5, 100, 8), a[100:108])


def _u_words(orc, st, n):
    """Each thread's xor64 word halves xored, from the generator run alone."""
    u = np.zeros((st.shape[0], n), dtype=np.uint32)
    for s in range(st.shape[0]):
        y0 = int(st[s, 0]) | (int(st[s, 1]) << 32)
        w = _xor64_words(orc, y0, n)
        u[s] = ((w ^ (w >> np.uint64(32))) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return u


@pytest.mark.parametrize("Cg", [32, 5])
def test_v4_lockstep_simulation(orc, Cg):
    if Cg == 32:
        comb1, comb2 = orc.comb_tables(32)
    else:
        comb1 = np.array([3, 4, 0, 1, 2], dtype=np.uint32)
        comb2 = np.array([1, 3, 4, 2, 0], dtype=np.uint32)
    ns, n = 2 * Cg, 40
    st = orc.seed(V4, 21, 0, ns)
    u = _u_words(orc, st, n)
    want = _alg4_lockstep(u, st[:, 3].tolist(), st[:, 2].tolist(), comb1, comb2, Cg)
    got, _ = orc.generate(V4, st.copy(), n, comb=(comb1, comb2))
    assert np.array_equal(got, want)


def test_v4_equal_combs_reduce_to_xor64_halves(orc):
    # comb1 == comb2: the neighbour words cancel, so each output is the
    # prefix xor of the thread's own xor64 halves (Eq. Oplus).
    c = np.array([(j + 3) % 8 for j in range(8)], dtype=np.uint32)
    st = orc.seed(V4, 4, 0, 16)
    x0 = st[:, 2].copy()
    u = _u_words(orc, st, 100)
    got, _ = orc.generate(V4, st, 100, comb=(c, c))
    assert np.array_equal(got, np.bitwise_xor.accumulate(u, axis=1) ^ x0[:, None])


def test_v4_prefix_xor_and_group_invariant(orc):
    comb1, comb2 = orc.comb_tables(32)
    st = orc.seed(V4, 3, 0, 64)
    x0 = st[:, 2].copy()
    u = _u_words(orc, st, 200)
    out, S = orc.generate(V4, st, 200, comb=(comb1, comb2), want_strategy=True)
    assert np.array_equal(out, np.bitwise_xor.accumulate(S, axis=1) ^ x0[:, None])
    # the state written back holds the last output and the last shared word
    assert np.array_equal(st[:, 2], out[:, -1])
    assert np.array_equal(st[:, 3], S[:, -1])
    for g in range(2):
        rows = slice(32 * g, 32 * g + 32)
        assert np.array_equal(np.bitwise_xor.reduce(S[rows], axis=0), np.bitwise_xor.reduce(u[rows], axis=0))


def test_v4_superposition_and_continuation(orc):
    a = orc.seed(V4, 11, 0, 64)
    b = orc.seed(V4, 12, 0, 64)
    ab = a ^ b
    oa, _ = orc.generate(V4, a, 150)
    ob, _ = orc.generate(V4, b, 150)
    oab, _ = orc.generate(V4, ab, 150)
    assert np.array_equal(oab, oa ^ ob)
    c = orc.seed(V4, 13, 0, 64)
    d = c.copy()
    o1, _ = orc.generate(V4, c, 37)
    o2, _ = orc.generate(V4, c, 91)
    o, _ = orc.generate(V4, d, 128)
    assert np.array_equal(np.concatenate([o1, o2], axis=1), o)
    assert np.array_equal(c, d)


def test_v1_xor64_alternative_composition(orc):
    # Listing 1 with xor64 as its first generator: S is still the xor of the
    # six 32-bit halves, the first pair now from xor64.
    V1A = 1 | orc.F_XOR64
    st = orc.seed(V1A, 5, 0, 4)
    assert np.array_equal(st, orc.seed(1, 5, 0, 4))      # same draws, same layout
    for s in range(4):
        w = st[s].astype(np.uint64)
        g1 = int(w[0] | (w[1] << np.uint64(32)))
        g2 = [int(w[2 + 2 * k] | (w[3 + 2 * k] << np.uint64(32))) for k in range(4)]
        g3 = [int(w[10 + 2 * k] | (w[11 + 2 * k] << np.uint64(32))) for k in range(6)]
        t1 = _xor64_words(orc, g1, 100)
        t2, _ = orc.gen_outputs(1, 64, g2, 100)
        t3, _ = orc.gen_outputs(2, 64, g3, 100)
        halves = t1 ^ (t1 >> np.uint64(32)) ^ t2 ^ (t2 >> np.uint64(32)) ^ t3 ^ (t3 >> np.uint64(32))
        want_S = (halves & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        one = st[s:s + 1].copy()
        _, S = orc.generate(V1A, one, 100, want_strategy=True, want_out=False)
        assert np.array_equal(S[0], want_S)


def test_v1_xor64_alternative_needs_64bit_words(orc):
    with pytest.raises(Exception):
        orc.seed(1 | orc.F_XOR64, 5, 0, 4, W=32)
