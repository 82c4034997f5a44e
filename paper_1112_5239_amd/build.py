"""Build libcprng.so in-tree for gfx950 with hipcc.

    python -m paper_1112_5239_amd.build        (or: python paper_1112_5239_amd/build.py)

Every source is compiled on every call (objects under _build/, in parallel)
and linked into paper_1112_5239_amd/libcprng.so.  Device code is built with
packed-FP32 instructions disabled and without floating-point contraction
(the consumption predicate rounds each product and the sum separately).
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libcprng.so")
ARCH = os.environ.get("CPRNG_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-ffp-contract=off"] + NO_PACKED_FP32
# Host sources include the HIP runtime headers; hipcc compiles them in HIP mode.
HOST = ["-D__HIP_PLATFORM_AMD__=1", f"--offload-arch={ARCH}"] + NO_PACKED_FP32


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [_hipcc()] + COMMON + DEVICE + ["-c", src, "-o", obj]
    else:
        cmd = [_hipcc()] + COMMON + HOST + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs + \
          ["-Wl,--no-undefined", "-Wl,-soname,libcprng.so"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
