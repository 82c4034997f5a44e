"""Pins of the oracle's BBS-based variant (Algorithm 5, Section 9.1) against
facts the paper and number theory fix, independent of the oracle's own code.

The paper prints no output of this generator, so the pins are: the moduli are
Blum integers below 2^16 (its stated requirements); one BBS step is modular
squaring (checked against Python's pow); seeded slots are quadratic residues
coprime to M; the bit layout of the strategy word on fixed points of the
squaring map (so every BBS output is a known constant); the direction of the
neighbour reads; how often each slot is stepped per output and the rotation of
the slots at the end of a call (closed form s^(2^(c n)) mod M); the prefix-xor
form of the chaotic iterations; and a monobit check.
"""
import math

import numpy as np
import pytest
import sympy

from oracle import oracle as O

V3 = 3


def _idempotents(M):
    """The four solutions of e^2 = e (mod M) for M = p*q: 0, 1 and the two CRT
    mixes (1 mod p, 0 mod q) and (0 mod p, 1 mod q)."""
    (p, _), (q, _) = sorted(sympy.factorint(M).items())
    e_p = (q * pow(q, -1, p)) % M      # 1 mod p, 0 mod q
    e_q = (p * pow(p, -1, q)) % M      # 0 mod p, 1 mod q
    return [0, 1, e_p, e_q]


def test_moduli_are_distinct_blum_integers_below_2_16():
    mods = [int(m) for m in O.bbs_moduli()]
    assert len(set(mods)) == 8
    for M in mods:
        f = sympy.factorint(M)
        assert sorted(f.values()) == [1, 1], M          # p*q, p != q
        for p in f:
            assert sympy.isprime(p) and p % 4 == 3       # Blum primes
            assert 200 < p < 260                         # "around 256"
        assert M < 1 << 16                                # x^2 fits 32 bits
        assert (M - 1) ** 2 < 1 << 32


def test_bbs_step_is_modular_squaring():
    rng = np.random.default_rng(11)
    mods = O.bbs_moduli()
    for k in range(8):
        for x in rng.integers(0, int(mods[k]), 200):
            assert O.bbs_step(int(x), k) == pow(int(x), 2, int(mods[k]))


def test_seeded_slots_are_coprime_quadratic_residues():
    st = O.seed(V3, 5, 0, 300)
    mods = [int(m) for m in O.bbs_moduli()]
    for row in st:
        for k in range(8):
            s, M = int(row[k]), mods[k]
            assert 0 < s < M and math.gcd(s, M) == 1
            for p in sympy.factorint(M):
                assert pow(s, (p - 1) // 2, p) == 1     # Euler: a square mod p


def test_idempotents_are_fixed_points():
    for M in O.bbs_moduli():
        for e in _idempotents(int(M)):
            assert pow(e, 2, int(M)) == e


def _fixed_states(want_low):
    """Slot states that are fixed points of their slot's squaring map, with
    the requested low bits where given (None: state 0)."""
    mods = [int(m) for m in O.bbs_moduli()]
    out = []
    for k in range(8):
        if want_low[k] is None:
            out.append(0)
            continue
        mask, val = want_low[k]
        cands = [e for e in _idempotents(mods[k]) if (e & mask) == val]
        assert cands, (k, want_low[k])
        out.append(cands[0])
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("slot", range(8))
def test_nibble_of_each_bbs_lands_in_its_place(slot):
    # Only slot `slot` outputs a nonzero low nibble (a fixed point of its
    # squaring map): the eight nibbles are shifted in four bits at a time,
    # BBS1 first, so BBS k's nibble ends up at bits 28-4(k-1) .. 31-4(k-1).
    # BBS3 and BBS7 also give the two extra shifts (their low two bits): for
    # those slots the word is further shifted left by that many bits, the
    # vacated bits taking BBS1's / BBS2's low bits, which are 0 here.
    mods = [int(m) for m in O.bbs_moduli()]
    cands = [e for e in _idempotents(mods[slot]) if e & 15]
    assert cands, slot
    e = cands[-1]
    st = np.zeros(8, dtype=np.uint32)
    st[slot] = e
    word, after = O.bbs_word(st)
    extra = (e & 3) if slot in (2, 6) else 0
    assert word == (((e & 15) << (28 - 4 * slot)) << extra) & 0xFFFFFFFF
    assert np.array_equal(after, st)                   # fixed points stay put


def test_extra_shifts_take_their_bits_from_bbs1_and_bbs2():
    # BBS3 and BBS7 at fixed points with low two bits s3, s7 shift t left by
    # s3 then s7 bits; the vacated low bits take BBS1's, then BBS2's, low
    # bits (masks 0, 1, 3, 7 for shifts 0..3).  Search the fixed points for
    # cases with nonzero shifts and compare with the bit placement the
    # paper describes.
    mods = [int(m) for m in O.bbs_moduli()]
    checked = 0
    for e3 in _idempotents(mods[2]):
        for e7 in _idempotents(mods[6]):
            for e1 in _idempotents(mods[0]):
                for e2 in _idempotents(mods[1]):
                    st = np.zeros(8, dtype=np.uint32)
                    st[0], st[1], st[2], st[6] = e1, e2, e3, e7
                    word, _ = O.bbs_word(st)
                    s3, s7 = e3 & 3, e7 & 3
                    nib = ((e1 & 15) << 28) | ((e2 & 15) << 24) | ((e3 & 15) << 20) | ((e7 & 15) << 4)
                    low1 = e1 & ((1 << s3) - 1)
                    low2 = e2 & ((1 << s7) - 1)
                    expect = ((((nib << s3) | low1) << s7) | low2) & 0xFFFFFFFF
                    assert word == expect, (e1, e2, e3, e7)
                    checked += (s3 > 0) + (s7 > 0)
    assert checked > 0


def test_word_from_random_states_matches_the_described_bit_placement():
    # Any states: BBS k's next output is pow(s_k, 2, M_k); the slots stepped a
    # second time in the step (BBS3, BBS1, BBS7, BBS2) give pow(s, 4, M).  The
    # word is the eight low nibbles (BBS1 highest), shifted left by the low two
    # bits of BBS3's second output with exactly that many low bits of BBS1's
    # second output put below, then the same with BBS7 and BBS2.  Random
    # states reach all four shift amounts.
    rng = np.random.default_rng(21)
    mods = [int(m) for m in O.bbs_moduli()]
    seen = set()
    for _ in range(400):
        st = np.array([rng.integers(2, mods[k]) for k in range(8)], dtype=np.uint32)
        word, _ = O.bbs_word(st)
        once = [pow(int(st[k]), 2, mods[k]) for k in range(8)]
        twice = {k: pow(int(st[k]), 4, mods[k]) for k in (0, 1, 2, 6)}
        t = 0
        for k in range(8):
            t = ((t << 4) | (once[k] & 15)) & 0xFFFFFFFF
        s3, s7 = twice[2] & 3, twice[6] & 3
        t = ((t << s3) | (twice[0] & ((1 << s3) - 1))) & 0xFFFFFFFF
        t = ((t << s7) | (twice[1] & ((1 << s7) - 1))) & 0xFFFFFFFF
        assert word == t
        seen.update((s3, s7))
    assert seen == {0, 1, 2, 3}


def test_neighbour_reads_follow_the_selected_arrays():
    # One step of a group of C = 8: t_new[j] = u[j] ^ t_prev[o1[j]] ^ t_prev[o2[j]]
    # with o1 = arrays[bbs1 & 7][j], o2 = arrays[8 + (bbs2 & 7)][j] taken at
    # the start of the call.  u[j] is the (separately pinned) BBS word; a
    # one-hot previous word per thread reveals which threads were read.
    Cg = 8
    arrays = O.bbs_comb_tables(Cg)
    st = O.seed(V3, 9, 0, Cg)
    st[:, 9] = 1 << np.arange(Cg, dtype=np.uint32)
    start = st.copy()
    _, strat = O.generate(V3, st, 1, comb=arrays, want_strategy=True)
    for j in range(Cg):
        u, _ = O.bbs_word(start[j, :8])
        read = int(strat[j, 0]) ^ u
        o1 = arrays[int(start[j, 0]) & 7][j]
        o2 = arrays[8 + (int(start[j, 1]) & 7)][j]
        assert read == (1 << int(o1)) ^ (1 << int(o2)), j


@pytest.mark.parametrize("n", [0, 1, 3])
def test_steps_per_slot_and_rotation_at_call_end(n):
    # Per output each BBS is stepped once for the nibbles, and BBS3, BBS1,
    # BBS7, BBS2 once more for the two extra shifts: 12 BBS numbers.  After
    # n outputs slot k holds s_k^(2^(c_k n)) mod M_k, c = (2,2,2,1,1,1,2,1),
    # and a call that produced outputs ends by storing slot k in slot k+1
    # (slot 8 in slot 1).  A call without outputs leaves the state alone.
    Cg = 8
    mods = [int(m) for m in O.bbs_moduli()]
    c = [2, 2, 2, 1, 1, 1, 2, 1]
    st = O.seed(V3, 4, 0, Cg)
    start = st.copy()
    O.generate(V3, st, n, comb=O.bbs_comb_tables(Cg))
    for j in range(Cg):
        stepped = [pow(int(start[j, k]), 1 << (c[k] * n), mods[k]) for k in range(8)]
        want = stepped[-1:] + stepped[:-1] if n > 0 else stepped
        assert [int(v) for v in st[j, :8]] == want, j


def test_outputs_are_the_prefix_xor_of_the_strategy():
    st = O.seed(V3, 2, 0, 64)
    x0 = st[:, 8].copy()
    out, strat = O.generate(V3, st, 50, want_strategy=True)
    acc = x0.copy()
    for i in range(50):
        acc ^= strat[:, i]
        assert np.array_equal(out[:, i], acc)


def test_arrangement_arrays_are_fixed_point_free_permutations_and_golden():
    arr = O.bbs_comb_tables(32)
    for a in range(16):
        assert sorted(arr[a].tolist()) == list(range(32))
        assert all(arr[a][j] != j for j in range(32))
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "bbs_comb_tables_c32.txt")
    rows = [line.split("=")[1].split() for line in open(path) if line.startswith("array")]
    assert np.array_equal(np.array(rows, dtype=np.uint32), arr)


def test_monobit():
    st = O.seed(V3, 3, 0, 256)
    out, _ = O.generate(V3, st, 4096)
    bits = np.unpackbits(out.view(np.uint8)).astype(np.int64)
    ones = int(bits.sum())
    nb = bits.size
    assert abs(ones - nb / 2) < 5 * math.sqrt(nb / 4)
