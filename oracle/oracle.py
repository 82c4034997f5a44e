"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this module.  The product library neither imports nor links it.

All arrays are numpy; states are array-of-structures uint32 words per stream
(V0: 5 words, V2: 6, V1: 23, V3: 10, V4: 4; layout in cprng_oracle.c).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

V0, V1, V2, V3, V4 = 0, 1, 2, 3, 4
F_XOR64 = 0x100        # V1 modifier: xor64 (13,7,17) as Listing 1's first generator

_lib = None
_override = None


class use_library:
    """Context manager: route every call of this module to another build of
    the oracle (used by the mutation tests, which compile planted mistakes)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _override
        self.prev = _override
        _override = _bind(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _override
        _override = self.prev


def lib():
    if _override is not None:
        return _override
    return _default_lib()


def _default_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


def _bind(L):
    """Declare the C signatures on a loaded oracle library."""
    u64, u32, i32, p = C.c_uint64, C.c_uint32, C.c_int, C.c_void_p
    L.orc_sm64_mix.restype = u64
    L.orc_sm64_mix.argtypes = [u64]
    L.orc_sm64_draws.restype = None
    L.orc_sm64_draws.argtypes = [u64, u64, p]
    L.orc_gen_outputs.restype = i32
    L.orc_gen_outputs.argtypes = [i32, i32, p, u64, p]
    L.orc_xs32_orbit.restype = u64
    L.orc_xs32_orbit.argtypes = [u32, u64, C.POINTER(i32)]
    L.orc_ci_step.restype = u32
    L.orc_ci_step.argtypes = [u32, u32]
    L.orc_ci_step_batch.restype = None
    L.orc_ci_step_batch.argtypes = [p, p, p, u64]
    L.orc_state_words.restype = i32
    L.orc_state_words.argtypes = [i32]
    L.orc_seed.restype = i32
    L.orc_seed.argtypes = [i32, i32, u64, u64, u64, p]
    L.orc_comb_tables.restype = i32
    L.orc_comb_tables.argtypes = [u32, p, p]
    L.orc_generate.restype = i32
    L.orc_generate.argtypes = [i32, i32, u64, p, u64, p, p, u32, p, p]
    L.orc_consume_qc.restype = i32
    L.orc_consume_qc.argtypes = [i32, i32, u64, p, u64, p, u32, p, p]
    L.orc_qc_hit.restype = i32
    L.orc_qc_hit.argtypes = [u32, u32]
    L.orc_bbs_moduli.restype = None
    L.orc_bbs_moduli.argtypes = [p]
    L.orc_bbs_step.restype = u32
    L.orc_bbs_step.argtypes = [p, i32]
    L.orc_bbs_word.restype = u32
    L.orc_bbs_word.argtypes = [p]
    L.orc_bbs_comb_tables.restype = i32
    L.orc_bbs_comb_tables.argtypes = [u32, p]
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def sm64_mix(z: int) -> int:
    return int(lib().orc_sm64_mix(z))


def sm64_draws(z: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_sm64_draws(z, n, _ptr(out))
    return out


def gen_outputs(kind: int, W: int, state, n: int):
    """kind 0 = xorshift(13,17,5), 1 = xor128, 2 = xorwow.  Returns (outputs, new state)."""
    st = np.array(state, dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint64)
    _check(lib().orc_gen_outputs(kind, W, _ptr(st), n, _ptr(out)), "gen_outputs")
    return out, st


def xs32_orbit(y0: int, limit: int):
    hz = C.c_int(0)
    n = lib().orc_xs32_orbit(y0, limit, C.byref(hz))
    return int(n), bool(hz.value)


def ci_step(x: int, S: int) -> int:
    return int(lib().orc_ci_step(x, S))


def ci_step_batch(x: np.ndarray, S: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint32)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    out = np.zeros_like(x)
    lib().orc_ci_step_batch(_ptr(x), _ptr(S), _ptr(out), x.size)
    return out


def state_words(variant: int) -> int:
    return int(lib().orc_state_words(variant))


def seed(variant: int, sigma: int, first_stream: int, n_streams: int, W: int = 64) -> np.ndarray:
    nw = state_words(variant)
    st = np.zeros((n_streams, nw), dtype=np.uint32)
    _check(lib().orc_seed(variant, W, sigma, first_stream, n_streams, _ptr(st)), "seed")
    return st


def comb_tables(Cg: int = 32):
    c1 = np.zeros(Cg, dtype=np.uint32)
    c2 = np.zeros(Cg, dtype=np.uint32)
    _check(lib().orc_comb_tables(Cg, _ptr(c1), _ptr(c2)), "comb_tables")
    return c1, c2


def bbs_moduli() -> np.ndarray:
    out = np.zeros(8, dtype=np.uint32)
    lib().orc_bbs_moduli(_ptr(out))
    return out


def bbs_step(x: int, slot: int) -> int:
    """One BBS step of slot 0..7; returns the new state."""
    v = C.c_uint32(x)
    return int(lib().orc_bbs_step(C.byref(v), slot))


def bbs_word(states):
    """Strategy bits of one step of Algorithm 5 from 8 slot states (before the
    neighbour mixing).  Returns (word, new states)."""
    b = np.ascontiguousarray(states, dtype=np.uint32).copy()
    w = int(lib().orc_bbs_word(_ptr(b)))
    return w, b


def bbs_comb_tables(Cg: int = 32) -> np.ndarray:
    """The sixteen arrangement arrays, shape (16, C)."""
    out = np.zeros(16 * Cg, dtype=np.uint32)
    _check(lib().orc_bbs_comb_tables(Cg, _ptr(out)), "bbs_comb_tables")
    return out.reshape(16, Cg)


def _comb_args(variant, comb):
    """(C, comb1, comb2) for the C entry points: V2 takes (comb1, comb2), V3 the
    (16, C) arrangement arrays."""
    if (variant & 0xFF) in (V2, V4):
        c1, c2 = comb if comb is not None else comb_tables(32)
        c1 = np.ascontiguousarray(c1, dtype=np.uint32)
        c2 = np.ascontiguousarray(c2, dtype=np.uint32)
        return c1.size, c1, c2
    if variant == V3:
        arr = np.ascontiguousarray(comb if comb is not None else bbs_comb_tables(32), dtype=np.uint32)
        return arr.shape[1], arr.reshape(-1), None
    return 0, None, None


def generate(variant: int, state: np.ndarray, n: int, W: int = 64, comb=None,
             want_out: bool = True, want_strategy: bool = False):
    """Advance `state` (modified in place) by n steps (one call of the paper's
    kernel).

    Returns (out, strategy), each shape (n_streams, n) or None.
    """
    assert state.dtype == np.uint32 and state.flags.c_contiguous
    ns = state.shape[0]
    out = np.zeros((ns, n), dtype=np.uint32) if want_out else None
    strat = np.zeros((ns, n), dtype=np.uint32) if want_strategy else None
    Cg, c1, c2 = _comb_args(variant, comb)
    _check(lib().orc_generate(variant, W, ns, _ptr(state), n, _ptr(out), _ptr(strat),
                              Cg, _ptr(c1), _ptr(c2)), "generate")
    return out, strat


def consume_qc(variant: int, state: np.ndarray, n: int, W: int = 64, comb=None) -> np.ndarray:
    assert state.dtype == np.uint32 and state.flags.c_contiguous
    ns = state.shape[0]
    counts = np.zeros(ns, dtype=np.uint64)
    Cg, c1, c2 = _comb_args(variant, comb)
    _check(lib().orc_consume_qc(variant, W, ns, _ptr(state), n, _ptr(counts), Cg,
                                _ptr(c1), _ptr(c2)), "consume_qc")
    return counts


def qc_hit(r1: int, r2: int) -> bool:
    return bool(lib().orc_qc_hit(r1, r2))
