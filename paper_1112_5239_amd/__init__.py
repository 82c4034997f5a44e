"""MI355X (gfx950) chaotic-iteration PRNG (Bahi, Couturier, Guyeux, Heam,
arXiv 1112.5239): HIP kernels behind a C ABI (include/cprng.h), bound here
with ctypes.  PyTorch is used only for device memory and streams.

    from paper_1112_5239_amd import Generator
    g = Generator(n_streams=1 << 20, variant="v2", seed=1)
    out = g.generate(1024)              # torch uint32 tensor [n_streams, 1024] on cuda
"""
from ._lib import (  # noqa: F401
    CprngError, F_INTERLEAVED, F_V1_W32, V0_PLAIN, V1_NAIVE3, V2_SHMEM, lib,
)
from .generator import Generator  # noqa: F401
