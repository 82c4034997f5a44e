"""Torch-facing wrapper of one cprng handle.

torch provides device memory and the current HIP stream; every number is
produced by the library's HIP kernels through the C ABI.
"""
import numpy as np

from . import _lib as L

_VARIANTS = {"v0": L.V0_PLAIN, "plain": L.V0_PLAIN, "v1": L.V1_NAIVE3, "naive3": L.V1_NAIVE3,
             "v2": L.V2_SHMEM, "shmem": L.V2_SHMEM, "v3": L.V3_BBS, "bbs": L.V3_BBS,
             "v4": L.V4_XOR64, "xor64": L.V4_XOR64}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the cprng library needs a HIP device (no CPU fallback)")
    return torch


def _stream(stream):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    return _torch().cuda.current_stream().cuda_stream


class Generator:
    def __init__(self, n_streams: int, variant="v0", seed: int = 0, group: int = 0, comb=None,
                 interleaved: bool = False, w32: bool = False, v1_xor64: bool = False, device: int = -1,
                 seeds=None):
        _torch()
        v = _VARIANTS[variant] if isinstance(variant, str) else int(variant)
        if interleaved:
            v |= L.F_INTERLEAVED
        if w32:
            v |= L.F_V1_W32
        if v1_xor64:
            v |= L.F_V1_XOR64
        c1, c2 = (comb if comb is not None else (None, None))
        if seeds is not None and len(seeds) != n_streams:
            raise ValueError("seeds needs one entry per stream")
        self.h = L.cprng_create_ex(v, n_streams, seed, group=group, comb1=c1, comb2=c2, device=device,
                                   seeds=seeds)
        self.n_streams = n_streams
        self.variant = v & 0xFF
        self.flags = v & ~0xFF

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            L.cprng_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- hot path -----------------------------------------------------------
    def generate(self, n: int, out=None, stream=None):
        """n outputs per stream; returns an int32 tensor holding the uint32 bits,
        shape [n_streams, n] (or [n, n_streams] with the interleaved flag)."""
        torch = _torch()
        shape = (n, self.n_streams) if self.flags & L.F_INTERLEAVED else (self.n_streams, n)
        if out is None:
            out = torch.empty(shape, dtype=torch.int32, device="cuda")
        L.cprng_generate(self.h, out, n, _stream(stream))
        return out

    def consume_qc(self, n: int, counts=None, stream=None):
        torch = _torch()
        if counts is None:
            counts = torch.empty(self.n_streams, dtype=torch.int64, device="cuda")
        L.cprng_consume_qc(self.h, counts, n, _stream(stream))
        return counts

    def generate_ragged(self, lengths, offsets=None, out=None, stream=None):
        torch = _torch()
        lengths = np.ascontiguousarray(lengths, dtype=np.uint64)
        if offsets is not None:
            offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
            total = int((offsets + lengths).max()) if lengths.size else 0
        else:
            total = int(lengths.sum())
        if out is None:
            out = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        L.cprng_generate_ragged(self.h, out, lengths, offsets, _stream(stream))
        return out

    def generate_requests(self, reqs, stream=None):
        """reqs: list of (stream_id, length, out_tensor_or_address)."""
        L.cprng_generate_requests(self.h, reqs, _stream(stream))

    def generate_subset(self, ids, lens, out_offsets, out, status=None, stream=None):
        """Device-described subset (cprng_generate_subset): ids (int32 tensor
        viewed as uint32), lens and out_offsets (int64 tensors) on the device,
        out the uint32 output base, status an optional one-element int32
        device tensor."""
        L.cprng_generate_subset(self.h, ids, lens, out_offsets, int(ids.numel()), out, status, _stream(stream))

    # -- state ----------------------------------------------------------------
    def state_words(self) -> int:
        return L.cprng_state_words(self.h)

    def get_state(self) -> np.ndarray:
        w = np.zeros((self.n_streams, self.state_words()), dtype=np.uint32)
        L.cprng_get_state(self.h, w)
        return w

    def set_state(self, words: np.ndarray) -> None:
        w = np.ascontiguousarray(words, dtype=np.uint32)
        L.cprng_set_state(self.h, w)

    def checkpoint(self) -> bytes:
        """Versioned, hashed image of every stream's state (cprng_checkpoint_save)."""
        return L.cprng_checkpoint_save(self.h)

    def restore(self, image: bytes) -> None:
        L.cprng_checkpoint_load(self.h, image)

    # -- tuning / timing ------------------------------------------------------
    def set_tuning(self, **kw):
        L.cprng_set_tuning(self.h, **kw)

    def get_tuning(self):
        return L.cprng_get_tuning(self.h)

    def autotune(self, n: int, scratch=None, stream=None):
        torch = _torch()
        if scratch is None:
            scratch = torch.empty(self.n_streams * n, dtype=torch.int32, device="cuda")
        L.cprng_autotune(self.h, scratch, n, _stream(stream))

    def autotune_ragged(self, lengths, offsets=None, out=None, stream=None):
        lengths = np.ascontiguousarray(lengths, dtype=np.uint64)
        if offsets is not None:
            offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        L.cprng_autotune_ragged(self.h, out, lengths, offsets, _stream(stream))

    def resolved_tuning(self, n: int) -> dict:
        """Launch configuration the next generate(n) uses, and its source."""
        return L.cprng_resolved_tuning(self.h, n)

    def resolved_tuning_ragged(self, lengths) -> dict:
        lengths = np.ascontiguousarray(lengths, dtype=np.uint64)
        return L.cprng_resolved_tuning_ragged(self.h, lengths)

    def enable_timing(self, on: bool = True):
        L.cprng_enable_timing(self.h, on)

    def last_kernel_ms(self) -> float:
        return L.cprng_last_kernel_ms(self.h)


def as_u32(t) -> np.ndarray:
    """Host numpy uint32 view of an int32 tensor produced by the library."""
    return t.detach().cpu().numpy().view(np.uint32)
