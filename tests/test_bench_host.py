"""Host-side checks of bench.py (no GPU): the block-kernel sources it hashes to
match the committed HBM counters all exist, the built library's sources cover
them, and the CLI refuses more than one GPU."""
import os
import subprocess
import sys

import bench
from paper_2311_11390_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_sources_exist_and_hash():
    csrc = os.path.join(ROOT, "paper_2311_11390_amd", "csrc")
    for name in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name
    d = bench.kernel_sources_digest()
    assert isinstance(d, str) and len(d) == 64
    # every compiled block-kernel source is hashed
    for src in build.SOURCES:
        if src.startswith("alif_blocks"):
            assert src in bench.KERNEL_SOURCES, src


def test_measured_traffic_parses_or_is_empty():
    t = bench.measured_traffic()
    assert t == {} or set(t) == {"block_fwd", "block_bwd"}
    for v in t.values():
        assert v > 1e8


def test_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
