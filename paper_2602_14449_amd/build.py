"""Build libtho.so (gfx950) in-tree with hipcc.

Usage: python paper_2602_14449_amd/build.py  (a plain script: it must not import
the package, whose import loads the library being rebuilt).
Every HIP translation unit is compiled with
  --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops
(the last flag keeps the compiler from emitting packed FP32 instructions).
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtho.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["k_small.hip", "k_tsqr.hip", "k_stream.hip", "k_lowp.hip", "k_batched.hip", "k_complex.hip", "tho_host.cpp", "tho_api.cpp", "tho_bcgs.cpp",
           "tho_backward.cpp", "tho_batched.cpp", "tho_complex.cpp", "tho_noalloc.hip", "k_pchoice.hip", "k_checks.hip", "tho_block.cpp", "k_weighted.hip", "tho_weighted.cpp", "k_zleaf.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _compile(src):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
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
