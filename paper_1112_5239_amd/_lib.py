"""ctypes binding of libcprng.so (argument marshalling only).

Every function here has the name of the C entry point it calls and raises
CprngError when the call returns a negative status.  There is no fallback:
if the HIP library is not built, loading fails with an error.
"""
import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcprng.so")

V0_PLAIN, V1_NAIVE3, V2_SHMEM, V3_BBS, V4_XOR64 = 0, 1, 2, 3, 4
F_INTERLEAVED = 1 << 8
F_V1_W32 = 1 << 9
F_SEED_PER_STREAM = 1 << 10
F_V1_XOR64 = 1 << 11

OK, E_INVAL, E_NOMEM, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4

STORE_AUTO, STORE_DIRECT, STORE_LDS, STORE_DIRECT_NT, STORE_LDS_NT = 0, 1, 2, 3, 4


class CprngError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("variant", C.c_uint32), ("n_streams", C.c_uint32),
                ("group", C.c_uint32), ("seed", C.c_uint64), ("comb1", C.POINTER(C.c_uint32)),
                ("comb2", C.POINTER(C.c_uint32)), ("device", C.c_int32), ("reserved", C.c_uint32),
                ("seeds", C.POINTER(C.c_uint64))]


class Request(C.Structure):
    _fields_ = [("stream", C.c_uint32), ("reserved", C.c_uint32), ("length", C.c_uint64),
                ("out", C.c_void_p)]


class ServerParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_gpu_streams", C.c_uint32), ("budget_bytes", C.c_uint64),
                ("max_batch", C.c_uint32), ("reserved", C.c_uint32)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("client", C.c_uint32), ("status", C.c_int32), ("length", C.c_uint64),
                ("out", C.c_void_p), ("t_submit_ns", C.c_uint64), ("t_admit_ns", C.c_uint64),
                ("t_done_ns", C.c_uint64)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_uint32), ("unroll", C.c_uint32), ("store", C.c_uint32),
                ("chunk", C.c_uint32), ("waves_per_cu", C.c_uint32), ("streams_per_lane", C.c_uint32),
                ("exchange", C.c_uint32), ("reserved", C.c_uint32)]


EXPORTED = [
    "cprng_create", "cprng_create_ex", "cprng_destroy", "cprng_generate", "cprng_consume_qc",
    "cprng_generate_ragged", "cprng_generate_ragged_noalloc", "cprng_generate_requests", "cprng_generate_subset",
    "cprng_state_words", "cprng_state_bytes", "cprng_get_state",
    "cprng_set_state", "cprng_checkpoint_bytes", "cprng_checkpoint_save", "cprng_checkpoint_load",
    "cprng_n_streams", "cprng_variant", "cprng_default_combs", "cprng_default_bbs_combs", "cprng_jump_selftest",
    "cprng_set_tuning", "cprng_get_tuning", "cprng_autotune", "cprng_autotune_ragged",
    "cprng_resolved_tuning", "cprng_resolved_tuning_ragged",
    "cprng_enable_timing", "cprng_last_kernel_ms", "cprng_probe_fill", "cprng_probe_copy", "cprng_probe_valu",
    "cprng_strerror", "cprng_last_error", "cprng_now_ns", "cprng_server_create", "cprng_server_submit",
    "cprng_server_poll", "cprng_server_release", "cprng_server_stats", "cprng_server_replay",
    "cprng_server_replay_keep",
    "cprng_server_destroy",
]

_lib = None


def lib():
    """Load libcprng.so (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is not built; run paper_1112_5239_amd/build.py "
                      "(the HIP library has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sig = {
        "cprng_create": (i32, [vp, u32, u32, vp]),
        "cprng_create_ex": (i32, [C.POINTER(Params), vp]),
        "cprng_destroy": (None, [vp]),
        "cprng_generate": (i32, [vp, vp, u64, vp]),
        "cprng_consume_qc": (i32, [vp, vp, u64, vp]),
        "cprng_generate_ragged": (i32, [vp, vp, vp, vp, vp]),
        "cprng_generate_ragged_noalloc": (i32, [vp, vp, vp, vp, vp]),
        "cprng_generate_requests": (i32, [vp, C.POINTER(Request), u32, vp]),
        "cprng_generate_subset": (i32, [vp, vp, vp, vp, u32, vp, vp, vp]),
        "cprng_state_words": (i32, [vp]),
        "cprng_state_bytes": (C.c_size_t, [vp]),
        "cprng_get_state": (i32, [vp, vp, C.c_size_t]),
        "cprng_set_state": (i32, [vp, vp, C.c_size_t]),
        "cprng_checkpoint_bytes": (C.c_size_t, [vp]),
        "cprng_checkpoint_save": (i32, [vp, vp, C.c_size_t]),
        "cprng_checkpoint_load": (i32, [vp, vp, C.c_size_t]),
        "cprng_n_streams": (u32, [vp]),
        "cprng_variant": (u32, [vp]),
        "cprng_default_combs": (i32, [u32, vp, vp]),
        "cprng_default_bbs_combs": (i32, [u32, vp]),
        "cprng_jump_selftest": (i32, [u32, u32, vp, vp, u64]),
        "cprng_set_tuning": (i32, [vp, C.POINTER(Tuning)]),
        "cprng_get_tuning": (i32, [vp, C.POINTER(Tuning)]),
        "cprng_autotune": (i32, [vp, vp, u64, vp]),
        "cprng_autotune_ragged": (i32, [vp, vp, vp, vp, vp]),
        "cprng_resolved_tuning": (i32, [vp, u64, C.POINTER(Tuning), vp]),
        "cprng_resolved_tuning_ragged": (i32, [vp, vp, C.POINTER(Tuning), vp]),
        "cprng_enable_timing": (i32, [vp, i32]),
        "cprng_last_kernel_ms": (C.c_double, [vp]),
        "cprng_probe_fill": (i32, [vp, u64, u32, vp]),
        "cprng_probe_copy": (i32, [vp, vp, u64, vp]),
        "cprng_probe_valu": (i32, [u32, vp, u32, u32, vp]),
        "cprng_strerror": (C.c_char_p, [i32]),
        "cprng_last_error": (C.c_char_p, []),
        "cprng_now_ns": (u64, []),
        "cprng_server_create": (i32, [vp, C.POINTER(ServerParams), vp]),
        "cprng_server_submit": (i32, [vp, u32, u64, u64, u64]),
        "cprng_server_poll": (i32, [vp, C.POINTER(Completion), u32, C.POINTER(u32)]),
        "cprng_server_release": (i32, [vp, vp]),
        "cprng_server_stats": (i32, [vp, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]),
        "cprng_server_replay": (i32, [vp, vp, vp, vp, u32, i32, C.POINTER(Completion)]),
        "cprng_server_replay_keep": (i32, [vp, vp, vp, vp, u32, vp, C.POINTER(Completion)]),
        "cprng_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc, where):
    if rc < 0:
        L = lib()
        raise CprngError(rc, where, f"{L.cprng_strerror(rc).decode()}: {L.cprng_last_error().decode()}")
    return rc


def _addr(x):
    """Device or host address of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def cprng_create(seed: int, n_streams: int, variant: int) -> int:
    h = C.c_void_p()
    s = (C.c_uint64 * 1)(seed)
    _check(lib().cprng_create(C.cast(s, C.c_void_p), n_streams, variant, C.byref(h)), "cprng_create")
    return h.value


def cprng_create_ex(variant: int, n_streams: int, seed: int, group: int = 0, comb1=None, comb2=None,
                    device: int = -1, seeds=None) -> int:
    """seeds: optional n_streams per-stream SplitMix64 start counters (sets
    F_SEED_PER_STREAM)."""
    p = Params()
    p.struct_size = C.sizeof(Params)
    p.variant = variant
    p.n_streams = n_streams
    p.group = group
    p.seed = seed
    p.device = device
    keep = []
    if comb1 is not None:
        a1 = (C.c_uint32 * len(comb1))(*[int(v) for v in comb1])
        a2 = (C.c_uint32 * len(comb2))(*[int(v) for v in comb2])
        keep += [a1, a2]
        p.comb1 = C.cast(a1, C.POINTER(C.c_uint32))
        p.comb2 = C.cast(a2, C.POINTER(C.c_uint32))
    if seeds is not None:
        sa = (C.c_uint64 * len(seeds))(*[int(v) for v in seeds])
        keep.append(sa)
        p.seeds = C.cast(sa, C.POINTER(C.c_uint64))
        p.variant = variant | F_SEED_PER_STREAM
    h = C.c_void_p()
    _check(lib().cprng_create_ex(C.byref(p), C.byref(h)), "cprng_create_ex")
    return h.value


def cprng_destroy(h: int) -> None:
    lib().cprng_destroy(h)


def cprng_generate(h: int, out, n_per_stream: int, stream=None) -> None:
    _check(lib().cprng_generate(h, _addr(out), n_per_stream, _addr(stream)), "cprng_generate")


def cprng_consume_qc(h: int, counts, n_per_stream: int, stream=None) -> None:
    _check(lib().cprng_consume_qc(h, _addr(counts), n_per_stream, _addr(stream)), "cprng_consume_qc")


def cprng_generate_ragged(h: int, out, lengths, offsets=None, stream=None) -> None:
    """lengths/offsets: host uint64 numpy arrays of n_streams entries."""
    _check(lib().cprng_generate_ragged(h, _addr(out), _addr(lengths), _addr(offsets), _addr(stream)),
           "cprng_generate_ragged")


def cprng_generate_ragged_noalloc(h: int, out, lengths, offsets=None, stream=None) -> None:
    """As cprng_generate_ragged (V0 handles), allocating no device memory."""
    _check(lib().cprng_generate_ragged_noalloc(h, _addr(out), _addr(lengths), _addr(offsets), _addr(stream)),
           "cprng_generate_ragged_noalloc")


def cprng_generate_requests(h: int, reqs, stream=None) -> None:
    """reqs: sequence of (stream_id, length, out) with out a device address or tensor."""
    arr = (Request * max(1, len(reqs)))()
    for i, (s, n, o) in enumerate(reqs):
        arr[i].stream = s
        arr[i].length = n
        arr[i].out = _addr(o)
    _check(lib().cprng_generate_requests(h, arr, len(reqs), _addr(stream)), "cprng_generate_requests")


def cprng_generate_subset(h: int, ids, lens, out_offsets, count: int, out_base, status=None, stream=None) -> None:
    """ids (uint32), lens and out_offsets (uint64): device addresses or tensors
    of `count` entries; status: optional device int32 (address or tensor)."""
    _check(lib().cprng_generate_subset(h, _addr(ids), _addr(lens), _addr(out_offsets), count, _addr(out_base),
                                       _addr(status), _addr(stream)), "cprng_generate_subset")


def cprng_state_bytes(h: int) -> int:
    return int(lib().cprng_state_bytes(h))


def cprng_state_words(h: int) -> int:
    return _check(lib().cprng_state_words(h), "cprng_state_words")


def cprng_get_state(h: int, host_words) -> None:
    _check(lib().cprng_get_state(h, _addr(host_words), host_words.size), "cprng_get_state")


def cprng_set_state(h: int, host_words) -> None:
    _check(lib().cprng_set_state(h, _addr(host_words), host_words.size), "cprng_set_state")


def cprng_checkpoint_bytes(h: int) -> int:
    return int(lib().cprng_checkpoint_bytes(h))


def cprng_checkpoint_save(h: int) -> bytes:
    """The handle's versioned checkpoint image."""
    n = cprng_checkpoint_bytes(h)
    buf = (C.c_ubyte * n)()
    _check(lib().cprng_checkpoint_save(h, buf, n), "cprng_checkpoint_save")
    return bytes(buf)


def cprng_checkpoint_load(h: int, image: bytes) -> None:
    buf = (C.c_ubyte * len(image)).from_buffer_copy(image)
    _check(lib().cprng_checkpoint_load(h, buf, len(image)), "cprng_checkpoint_load")


def cprng_n_streams(h: int) -> int:
    return int(lib().cprng_n_streams(h))


def cprng_variant(h: int) -> int:
    return int(lib().cprng_variant(h))


def cprng_jump_selftest(variant: int, Cg: int = 0, comb1=None, comb2=None, J: int = 1000) -> None:
    """Host-only check of the jump-ahead (raises CprngError on failure)."""
    keep = []
    p1 = p2 = None
    if comb1 is not None:
        a1 = (C.c_uint32 * len(comb1))(*[int(v) for v in comb1])
        a2 = (C.c_uint32 * len(comb2))(*[int(v) for v in comb2])
        keep += [a1, a2]
        p1, p2 = C.cast(a1, C.c_void_p), C.cast(a2, C.c_void_p)
    _check(lib().cprng_jump_selftest(variant, Cg, p1, p2, J), "cprng_jump_selftest")


def cprng_default_bbs_combs(Cg: int):
    """The library's 16 arrangement arrays of the BBS variant, as 16 lists of Cg."""
    arr = (C.c_uint32 * (16 * Cg))()
    _check(lib().cprng_default_bbs_combs(Cg, C.cast(arr, C.c_void_p)), "cprng_default_bbs_combs")
    return [list(arr[a * Cg:(a + 1) * Cg]) for a in range(16)]


def cprng_default_combs(Cg: int):
    a1 = (C.c_uint32 * Cg)()
    a2 = (C.c_uint32 * Cg)()
    _check(lib().cprng_default_combs(Cg, C.cast(a1, C.c_void_p), C.cast(a2, C.c_void_p)), "cprng_default_combs")
    return list(a1), list(a2)


def cprng_set_tuning(h: int, block=0, unroll=0, store=0, chunk=0, waves_per_cu=0,
                     streams_per_lane=0, exchange=0) -> None:
    t = Tuning(block, unroll, store, chunk, waves_per_cu, streams_per_lane, exchange)
    _check(lib().cprng_set_tuning(h, C.byref(t)), "cprng_set_tuning")


def cprng_get_tuning(h: int) -> dict:
    t = Tuning()
    _check(lib().cprng_get_tuning(h, C.byref(t)), "cprng_get_tuning")
    return {"block": t.block, "unroll": t.unroll, "store": t.store, "chunk": t.chunk,
            "waves_per_cu": t.waves_per_cu, "streams_per_lane": t.streams_per_lane,
            "exchange": t.exchange}


def _tuning_dict(t) -> dict:
    return {"block": t.block, "unroll": t.unroll, "store": t.store, "chunk": t.chunk,
            "waves_per_cu": t.waves_per_cu, "streams_per_lane": t.streams_per_lane,
            "exchange": t.exchange}


_SOURCES = {0: "default", 1: "autotuned", 2: "explicit"}


def cprng_resolved_tuning(h: int, n_per_stream: int) -> dict:
    t, src = Tuning(), C.c_int(-1)
    _check(lib().cprng_resolved_tuning(h, n_per_stream, C.byref(t), C.byref(src)), "cprng_resolved_tuning")
    return {**_tuning_dict(t), "source": _SOURCES.get(src.value, src.value)}


def cprng_resolved_tuning_ragged(h: int, lengths) -> dict:
    t, src = Tuning(), C.c_int(-1)
    _check(lib().cprng_resolved_tuning_ragged(h, _addr(lengths), C.byref(t), C.byref(src)),
           "cprng_resolved_tuning_ragged")
    return {**_tuning_dict(t), "source": _SOURCES.get(src.value, src.value)}


def cprng_autotune(h: int, scratch, n_per_stream: int, stream=None) -> None:
    _check(lib().cprng_autotune(h, _addr(scratch), n_per_stream, _addr(stream)), "cprng_autotune")


def cprng_autotune_ragged(h: int, out, lengths, offsets=None, stream=None) -> None:
    _check(lib().cprng_autotune_ragged(h, _addr(out), _addr(lengths), _addr(offsets), _addr(stream)),
           "cprng_autotune_ragged")


def cprng_enable_timing(h: int, on: bool) -> None:
    _check(lib().cprng_enable_timing(h, 1 if on else 0), "cprng_enable_timing")


def cprng_last_kernel_ms(h: int) -> float:
    return float(lib().cprng_last_kernel_ms(h))


def cprng_probe_fill(dst, n_words: int, value: int, stream=None) -> None:
    _check(lib().cprng_probe_fill(_addr(dst), n_words, value, _addr(stream)), "cprng_probe_fill")


def cprng_probe_copy(dst, src, n_words: int, stream=None) -> None:
    _check(lib().cprng_probe_copy(_addr(dst), _addr(src), n_words, _addr(stream)), "cprng_probe_copy")


def cprng_probe_valu(kind: int, out, n_threads: int, iters: int, stream=None) -> None:
    _check(lib().cprng_probe_valu(kind, _addr(out), n_threads, iters, _addr(stream)), "cprng_probe_valu")


def cprng_strerror(status: int) -> str:
    return lib().cprng_strerror(status).decode()


def cprng_last_error() -> str:
    return lib().cprng_last_error().decode()


# ---------------------------------------------------------------------------
# Serving loop.
# ---------------------------------------------------------------------------
def cprng_now_ns() -> int:
    return int(lib().cprng_now_ns())


def cprng_server_create(h: int, n_gpu_streams: int = 0, budget_bytes: int = 0, max_batch: int = 0) -> int:
    p = ServerParams(C.sizeof(ServerParams), n_gpu_streams, budget_bytes, max_batch, 0)
    s = C.c_void_p()
    _check(lib().cprng_server_create(h, C.byref(p), C.byref(s)), "cprng_server_create")
    return s.value


def cprng_server_submit(s: int, client: int, length: int, tag: int, t_submit_ns: int = 0) -> None:
    _check(lib().cprng_server_submit(s, client, length, tag, t_submit_ns), "cprng_server_submit")


def cprng_server_poll(s: int, max_done: int = 256):
    buf = (Completion * max_done)()
    n = C.c_uint32(0)
    _check(lib().cprng_server_poll(s, buf, max_done, C.byref(n)), "cprng_server_poll")
    return [buf[i] for i in range(n.value)]


def cprng_server_release(s: int, out: int) -> None:
    _check(lib().cprng_server_release(s, out), "cprng_server_release")


def cprng_server_stats(s: int):
    w, f, b = C.c_uint64(0), C.c_uint64(0), C.c_uint64(0)
    _check(lib().cprng_server_stats(s, C.byref(w), C.byref(f), C.byref(b)), "cprng_server_stats")
    return {"waiting": w.value, "in_flight": f.value, "bytes_in_use": b.value}


def cprng_server_replay(s: int, arrival_ns, client, length, release_results: bool):
    """arrival_ns/length: uint64 numpy arrays, client: uint32 numpy array.
    Returns a ctypes array of Completion, indexed by request."""
    n = len(arrival_ns)
    res = (Completion * max(1, n))()
    _check(lib().cprng_server_replay(s, _addr(arrival_ns), _addr(client), _addr(length), n,
                                     1 if release_results else 0, res), "cprng_server_replay")
    return res


def cprng_server_replay_keep(s: int, arrival_ns, client, length, keep):
    """As cprng_server_replay with results released as they complete, except
    those with keep[i] != 0 (uint8 numpy array)."""
    n = len(arrival_ns)
    res = (Completion * max(1, n))()
    _check(lib().cprng_server_replay_keep(s, _addr(arrival_ns), _addr(client), _addr(length), n,
                                          _addr(keep), res), "cprng_server_replay_keep")
    return res


def cprng_server_destroy(s: int) -> None:
    lib().cprng_server_destroy(s)
