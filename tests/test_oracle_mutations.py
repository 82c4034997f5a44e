"""Mutation check of the oracle pins.

Each case plants one plausible mistake in a copy of the oracle's C source
(compiled here, on the CPU), points the oracle binding at the mutant and runs
the pins of test_oracle_pins.py.  Every mutant must make at least one pin
fail; the unmodified source must pass them all.  Mutants are never used for
anything else.
"""
import os
import subprocess

import pytest

from oracle import oracle as O
from tests import test_oracle_bbs_pins as B
from tests import test_oracle_pins as P
from tests import test_oracle_xor64_pins as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cprng_oracle.c")

# (name, original text, replacement) -- each original must occur in the source.
MUTATIONS = [
    ("xor128 left shift 11->12", "s[0] ^ ((s[0] << 11) & m)", "s[0] ^ ((s[0] << 12) & m)"),
    ("xor128 t>>8 -> t>>9", "(t ^ (t >> 8))", "(t ^ (t >> 9))"),
    ("xor128 w>>19 -> w>>18", "(s[3] ^ (s[3] >> 19))", "(s[3] ^ (s[3] >> 18))"),
    ("xorshift 13 -> 14", "orc_xs_step(&y, 13, 17, 5, 32)", "orc_xs_step(&y, 14, 17, 5, 32)"),
    ("xorwow Weyl 362437 -> 362439", "(s[5] + 362437ull)", "(s[5] + 362439ull)"),
    ("xorwow v<<4 -> v<<3", "((s[4] << 4) & m)", "((s[4] << 3) & m)"),
    ("step xor -> or", "return x ^ S;", "return x | S;"),
    ("listing drops t3", "fold32(t1 ^ t2 ^ t3)", "fold32(t1 ^ t2)"),
    ("listing drops hi(t3)", "fold32(t1 ^ t2 ^ t3)", "fold32(t1 ^ t2) ^ (uint32_t)t3"),
    ("listing high halves dropped", "{ return (uint32_t)v ^ (uint32_t)(v >> 32); }", "{ return (uint32_t)v; }"),
    ("alg4 reads comb2 twice", "u[j] ^ tprev[comb1[j]] ^ tprev[comb2[j]]", "u[j] ^ tprev[comb2[j]] ^ tprev[comb2[j]]"),
    ("alg4 index direction (inverse)",
     "for (uint32_t j = 0; j < C; ++j) tnext[j] = u[j] ^ tprev[comb1[j]] ^ tprev[comb2[j]];",
     "for (uint32_t j = 0; j < C; ++j) { tnext[comb1[j]] = 0; }\n"
     "        for (uint32_t j = 0; j < C; ++j) tnext[comb1[j]] ^= u[comb1[j]] ^ tprev[j];\n"
     "        for (uint32_t j = 0; j < C; ++j) tnext[comb2[j]] ^= tprev[j];"),
    ("alg4 gauss-seidel", "for (uint32_t j = 0; j < C; ++j) tnext[j] = u[j] ^ tprev[comb1[j]] ^ tprev[comb2[j]];",
     "for (uint32_t j = 0; j < C; ++j) { tnext[j] = u[j] ^ tprev[comb1[j]] ^ tprev[comb2[j]]; tprev[j] = tnext[j]; }"),
    ("consume <= 1", "if (s < 1.0f) ++hits;", "if (s <= 1.0f) ++hits;"),
    ("consume top 23 bits", "float u = (float)(r[k] >> 8) * 0x1p-24f;", "float u = (float)(r[k] >> 9) * 0x1p-23f;"),
    ("consume pairs (k,k+2)", "float v = (float)(r[k + 1] >> 8) * 0x1p-24f;",
     "float v = (float)(r[k + 1 < n ? k + 1 : k] >> 8) * 0x1p-24f; v = (float)(r[(k + 2) % n] >> 8) * 0x1p-24f;"),
    ("splitmix gamma", "#define ORC_SM64_GAMMA 0x9E3779B97F4A7C15ull", "#define ORC_SM64_GAMMA 0x9E3779B97F4A7C17ull"),
    ("splitmix shift 30 -> 31", "z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;", "z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;"),
    ("continuation loses state", "    st[4] = x;\n}", "    st[4] = x ^ 1u;\n}"),
    ("alg5 nibbles BBS8 first", "& 15u) << (28 - 4 * k);", "& 15u) << (4 * k);"),
    ("alg5 (8+bbs2)&7 precedence", "combs[(size_t)(8u + (s[1] & 7u)) * C + j]", "combs[(size_t)((8u + s[1]) & 7u) * C + j]"),
    ("alg5 o1 array from slot 2", "o1[j] = combs[(size_t)(s[0] & 7u) * C + j];", "o1[j] = combs[(size_t)(s[1] & 7u) * C + j];"),
    ("alg5 rotation backwards",
     "uint32_t last = s[7];\n            for (int k = 7; k > 0; --k) s[k] = s[k - 1];\n            s[0] = last;",
     "uint32_t first = s[0];\n            for (int k = 0; k < 7; ++k) s[k] = s[k + 1];\n            s[7] = first;"),
    ("alg5 fill mask of shift 3 one bit short", "orc_bbs_step(&b[0], 0) & ((1u << s1) - 1u)",
     "orc_bbs_step(&b[0], 0) & ((1u << (s1 < 3 ? s1 : 2)) - 1u)"),
    ("alg5 BBS2 not stepped again", "f2 = orc_bbs_step(&b[1], 1) & ((1u << s2) - 1u)", "f2 = b[1] & ((1u << s2) - 1u)"),
    ("alg5 fields swapped", "| (f1 << s2) | f2;", "| (f2 << s1) | f1;"),
    ("alg5 modulus 251*239 -> 251*241", "251u * 239u, 251u * 227u", "251u * 241u, 251u * 227u"),
    ("alg5 seed not squared", "st[k] = (uint32_t)((r * r) % M);", "st[k] = (uint32_t)r;"),
    ("xor64 triple 7 -> 8", "orc_xs_step(y, 13, 7, 17, 64)", "orc_xs_step(y, 13, 8, 17, 64)"),
    ("v4 word is the low half only", "tnext[j] = (uint32_t)v ^ (uint32_t)(v >> 32);", "tnext[j] = (uint32_t)v;"),
    ("v4 reads comb1 twice", "tnext[j] ^= tprev[comb1[j]] ^ tprev[comb2[j]];", "tnext[j] ^= tprev[comb1[j]] ^ tprev[comb1[j]];"),
    ("v4 loses t at call end", "st[j * 4 + 3] = tprev[j];", "st[j * 4 + 3] = tprev[j] ^ 1u;"),
    ("v1 alternative ignored", "alt ? orc_xor64_step(&g1) : orc_xs_step(&g1, 13, 17, 5, W)", "orc_xs_step(&g1, 13, 17, 5, W)"),
]
# Not listed: dropping the all-zero redraw of the seeding is an equivalent
# mutant in practice (four zero draws have probability 2^-128); the seeding
# draw order is a documented convention, checked by oracle/library agreement.
# Nor the mirrored xor64 triple (17,7,13): it is also a full-period xor64, so
# no property the paper fixes separates it from (13,7,17); the order is the
# reading's convention (Marsaglia lists the triple as (13,7,17)).


def _pins(orc):
    """The CPU pins, each a callable raising AssertionError on failure."""
    t = []
    t.append(lambda: P.test_table1_worked_example(orc))
    for N in (3, 5):
        t.append(lambda N=N: P.test_general_ci_bruteforce_small(orc, N))
    t.append(lambda: P.test_general_ci_bruteforce_n10(orc))
    t.append(lambda: _period_quick(orc))
    t.append(lambda: P.test_xor128_32_primitive_degree_128(orc))
    t.append(lambda: P.test_xorwow_32_core_primitive_degree_160(orc))
    t.append(lambda: P.test_generators_64bit_are_gf2_linear_and_width_generic(orc))
    t.append(lambda: P.test_xorshift64_13_17_5_reduces_to_alg2_on_low_word_prefix(orc))
    t.append(lambda: P.test_splitmix_gamma_is_golden_ratio(orc))
    t.append(lambda: P.test_splitmix_mix_bijective(orc))
    t.append(lambda: P.test_seeding_reproducible_nonzero_distinct(orc))
    for v in (0, 1, 2):
        t.append(lambda v=v: P.test_prefix_xor_form(orc, v))
        t.append(lambda v=v: P.test_continuation(orc, v))
    for v in (0, 2):
        t.append(lambda v=v: P.test_superposition_linear_variants(orc, v))
        t.append(lambda v=v: P.test_consume_counts_match_numpy_float32(orc, v))
    t.append(lambda: P.test_superposition_fails_for_v1(orc))
    for W in (64, 32):
        t.append(lambda W=W: P.test_listing1_composition(orc, W))
    t.append(lambda: P.test_comb_tables_are_valid_derangement_pairs(orc))
    t.append(lambda: P.test_alg4_index_direction_one_hot(orc))
    for Cg in (32, 5):
        t.append(lambda Cg=Cg: P.test_alg4_lockstep_simulation(orc, Cg))
    t.append(lambda: P.test_alg4_group_xor_invariant(orc))
    t.append(lambda: P.test_alg4_equal_combs_reduces_to_v0(orc))
    t.append(lambda: P.test_consume_predicate_edges(orc))
    t.append(B.test_moduli_are_distinct_blum_integers_below_2_16)
    t.append(B.test_bbs_step_is_modular_squaring)
    t.append(B.test_seeded_slots_are_coprime_quadratic_residues)
    for slot in range(8):
        t.append(lambda slot=slot: B.test_nibble_of_each_bbs_lands_in_its_place(slot))
    t.append(B.test_extra_shifts_take_their_bits_from_bbs1_and_bbs2)
    t.append(B.test_word_from_random_states_matches_the_described_bit_placement)
    t.append(B.test_neighbour_reads_follow_the_selected_arrays)
    for n in (0, 1, 3):
        t.append(lambda n=n: B.test_steps_per_slot_and_rotation_at_call_end(n))
    t.append(B.test_outputs_are_the_prefix_xor_of_the_strategy)
    t.append(B.test_arrangement_arrays_are_fixed_point_free_permutations_and_golden)
    t.append(B.test_monobit)
    t.append(lambda: X.test_xor64_primitive_degree_64(orc))
    for Cg in (32, 5):
        t.append(lambda Cg=Cg: X.test_v4_lockstep_simulation(orc, Cg))
    t.append(lambda: X.test_v4_equal_combs_reduce_to_xor64_halves(orc))
    t.append(lambda: X.test_v4_prefix_xor_and_group_invariant(orc))
    t.append(lambda: X.test_v4_superposition_and_continuation(orc))
    t.append(lambda: X.test_v1_xor64_alternative_composition(orc))
    return t


def _period_quick(orc):
    # Algorithm 2's period is 2^32 - 1; a shorter orbit from 1 shows a wrong
    # triple quickly (the full exhaustive check lives in test_oracle_pins).
    n, hit_zero = orc.xs32_orbit(1, 1 << 24)
    assert n == 1 << 24 and not hit_zero


def _build(tmp_path, name, src_text):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-w",
                           "-o", str(so), str(c)])
    return str(so)


def _failures(path):
    failed = 0
    with O.use_library(path):
        for pin in _pins(O):
            try:
                pin()
            except (AssertionError, ValueError):
                failed += 1
    return failed


def test_unmodified_oracle_passes_every_pin(tmp_path):
    so = _build(tmp_path, "orig", open(SRC).read())
    assert _failures(so) == 0


@pytest.mark.parametrize("name,orig,repl", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_every_planted_mistake_is_caught(tmp_path, name, orig, repl):
    src = open(SRC).read()
    assert orig in src, f"mutation anchor not found: {orig!r}"
    so = _build(tmp_path, "mutant", src.replace(orig, repl, 1))
    assert _failures(so) > 0, f"no pin caught: {name}"
