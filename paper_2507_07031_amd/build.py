"""Build the gfx950 shared library libzk.so in-tree with hipcc.

    python -m paper_2507_07031_amd.build

Each .hip file is compiled separately (in parallel) and linked into one
shared library next to this file.  Packed-FP32 instruction selection is
disabled for every HIP compile (the kernels use no floating point).
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libzk.so")
SOURCES = ["api.hip", "ntt.hip", "msm.hip", "msm_accumulate.hip", "msm_tiny.hip", "prof.hip", "validate.hip", "open.hip", "quotient.hip", "accum.hip", "g2msm.hip"]
HIPCC = os.environ.get("HIPCC", "hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
