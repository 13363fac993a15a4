"""Build libblockalif.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_2311_11390_amd.build          # or build() from Python
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libblockalif.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["alif_api.hip", "alif_blocks.hip", "alif_blocks_s1.hip", "alif_blocks_s2.hip",
           "alif_blocks_s4.hip", "alif_blocks_s8.hip", "alif_blocks_s8_long.hip", "alif_blocks_s8_xl.hip",
           "alif_recurrent_g2.hip", "alif_recurrent_g4.hip", "alif_recurrent_wgrad.hip",
           "alif_seq.hip", "alif_gemm.hip", "alif_gemm_big.hip", "alif_readout.hip", "alif_server.hip", "alif_fit.hip",
           "alif_events.hip"]
ARCH = os.environ.get("ALIF_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: every FMA in the kernels is written explicitly, so the forward
# and the backward recompute the same rounding sequence.
# -packed-fp32-ops: no v_pk_*_f32 instructions are generated.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-I", INCLUDE]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
