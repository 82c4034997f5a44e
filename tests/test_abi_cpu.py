"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function include/cprng.h declares, and
reject invalid arguments that are checked before any device work.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cprng.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(cprng_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1112_5239_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    declared = _declared_functions()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(L.EXPORTED) == declared


def test_status_strings(L):
    assert L.cprng_strerror(0) == "ok"
    assert L.cprng_strerror(-1) == "invalid argument"
    assert L.cprng_strerror(-4) == "unsupported"


def test_invalid_arguments_rejected_before_device_work(L):
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 0, 0)                      # n_streams == 0
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 64, 7)                     # unknown variant
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 100, L.V2_SHMEM)           # 100 % 32 != 0
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create_ex(L.V2_SHMEM, 96, 0, group=3)  # group not a power of two
    assert e.value.status == L.E_UNSUPPORTED
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 64, L.V0_PLAIN | L.F_V1_W32)  # W32 flag on V0
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 64, L.V1_NAIVE3 | L.F_V1_W32 | L.F_V1_XOR64)  # xor64 needs 64-bit words
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 64, L.V4_XOR64 | L.F_V1_XOR64)  # V1 flag on V4
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create(0, 100, L.V4_XOR64)           # 100 % 32 != 0
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.CprngError) as e:
        L.cprng_create_ex(L.V0_PLAIN | L.F_SEED_PER_STREAM, 64, 0)   # flag without the seeds array
    assert e.value.status == L.E_INVAL
    assert L.lib().cprng_state_bytes(None) == 0
    with pytest.raises(L.CprngError) as e:
        L.cprng_create_ex(L.V2_SHMEM, 64, 0, group=4, comb1=[1, 2, 3, 9], comb2=[2, 3, 0, 1])
    assert e.value.status == L.E_INVAL
    lib = L.lib()
    assert lib.cprng_generate(None, None, 4, None) == L.E_INVAL
    assert lib.cprng_consume_qc(None, None, 4, None) == L.E_INVAL
    assert lib.cprng_state_words(None) == L.E_INVAL
    assert lib.cprng_last_kernel_ms(None) < 0
    assert lib.cprng_probe_valu(5, 16, 256, 1, None) == L.E_INVAL      # no such class
    assert lib.cprng_probe_valu(0, 16, 100, 1, None) == L.E_INVAL      # not a multiple of 256
    assert lib.cprng_probe_valu(0, None, 256, 1, None) == L.E_INVAL
    lib.cprng_destroy(None)                          # no-op


def test_default_combs_match_the_oracle_reading(L, orc):
    # Two independent implementations of the same reading of Algorithm 4's
    # unspecified combination arrays must agree.
    for Cg in (4, 8, 16, 32, 64):
        c1, c2 = L.cprng_default_combs(Cg)
        o1, o2 = orc.comb_tables(Cg)
        assert c1 == o1.tolist() and c2 == o2.tolist()
    with pytest.raises(L.CprngError):
        L.cprng_default_combs(2)


def test_default_bbs_arrays_match_the_oracle_reading(L, orc):
    # Algorithm 5's sixteen arrangement arrays: library and oracle draw them
    # independently from the same reading.
    for Cg in (4, 8, 16, 32, 64):
        assert L.cprng_default_bbs_combs(Cg) == orc.bbs_comb_tables(Cg).tolist()
    with pytest.raises(L.CprngError):
        L.cprng_default_bbs_combs(3)


def test_header_is_plain_c(tmp_path):
    # The boundary header compiles as C99 on its own (no HIP or torch types).
    src = tmp_path / "t.c"
    src.write_text('#include "cprng.h"\nint main(void){cprng_params_t p; (void)p; return 0;}\n')
    import subprocess
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(tmp_path / "t")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("J", [0, 1, 777, 123457])
def test_group_jump_ahead_selftest(L, J):
    # The ragged paths' jump polynomials, checked on the host: X^J mod q of
    # the group map reproduces J steps (V2 and V4, default and custom arrays).
    L.cprng_jump_selftest(L.V2_SHMEM, 32, J=J)
    L.cprng_jump_selftest(L.V4_XOR64, 16, J=J)
    L.cprng_jump_selftest(L.V2_SHMEM, 8, comb1=[3, 4, 0, 1, 7, 6, 2, 5], comb2=[1, 3, 4, 2, 0, 7, 5, 6], J=J)


@pytest.mark.parametrize("J", [0, 1, 4096, 99991])
def test_v1_jump_ahead_and_aggregate_selftest(L, J):
    for flags in (0, L.F_V1_W32, L.F_V1_XOR64):
        L.cprng_jump_selftest(L.V1_NAIVE3 | flags, J=J)


def test_jump_selftest_rejects_bad_arguments(L):
    for args in ((L.V3_BBS, 32), (L.V2_SHMEM, 7), (L.V1_NAIVE3 | L.F_V1_W32 | L.F_V1_XOR64, 0)):
        with pytest.raises(L.CprngError) as e:
            L.cprng_jump_selftest(*args, J=10)
        assert e.value.status == L.E_INVAL


def test_tuning_queries_and_replay_reject_null_before_device_work(L):
    lib = L.lib()
    t = L.Tuning()
    src = C.c_int(-1)
    assert lib.cprng_resolved_tuning(None, 64, C.byref(t), C.byref(src)) == L.E_INVAL
    lengths = np.ones(4, dtype=np.uint64)
    assert lib.cprng_resolved_tuning_ragged(None, lengths.ctypes.data, C.byref(t), C.byref(src)) == L.E_INVAL
    res = (L.Completion * 1)()
    z64 = np.zeros(1, dtype=np.uint64)
    z32 = np.zeros(1, dtype=np.uint32)
    keep = np.zeros(1, dtype=np.uint8)
    assert lib.cprng_server_replay_keep(None, z64.ctypes.data, z32.ctypes.data, z64.ctypes.data, 1,
                                        keep.ctypes.data, res) == L.E_INVAL
    assert lib.cprng_autotune(None, None, 64, None) == L.E_INVAL
    assert lib.cprng_autotune_ragged(None, None, lengths.ctypes.data, None, None) == L.E_INVAL


def test_subset_rejects_null_handle_before_device_work(L):
    lib = L.lib()
    z64 = np.zeros(1, dtype=np.uint64)
    z32 = np.zeros(1, dtype=np.uint32)
    assert lib.cprng_generate_subset(None, z32.ctypes.data, z64.ctypes.data, z64.ctypes.data, 1,
                                     z32.ctypes.data, None, None) == L.E_INVAL
