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


def _fake_result():
    """A detail record shaped like bench.py's, with every leg present and long."""
    k = {"avg_ms": 0.6, "bytes_per_launch": 2.7e9, "achieved_GBs": 4500.0, "frac_of_peak": 0.56}
    mode = {"p50_ms": 1.5, "p99_ms": 9.2, "mean_ms": 2.0, "max_ms": 30.0, "neuron_steps_per_s": 5.3e9,
            "span_s": 10.0, "failed": 0}
    sl = {"blocks_in_sequence": 500, "steps_in_sequence": 1000, "T_R": 2, "block_fwd_ms": 0.05,
          "sequential_fwd_ms": 0.2, "spikes": 1234, "block_equals_sequential": True,
          "block_us_per_dependent_block": 0.1, "speedup_vs_sequential": 4.0}
    return {
        "metric": "neuron-steps/s fwd+bwd, block-wise vs sequential ALIF on 1 GPU; p99 latency",
        "value": 3.3e11, "unit": "neuron-steps/s", "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": 1.0,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fine-DT fit: 256 ALIF neurons x batch 64, T=20000, DT=0.05 ms, ARP=2.0 ms "
                               "(T_R=40), OU current, forward+backward",
                   "batch": 64, "neurons": 256, "T": 20000, "dt_ms": 0.05, "arp_ms": 2.0, "T_R": 40,
                   "firing_rate_hz": 2.3},
        "roofline": {"bound": "hbm", "kernel": "block_bwd", "achieved": 4500.0, "peak": 8000.0, "unit": "GB/s",
                     "frac": 0.5625, "traffic": 2.7e9, "algorithmic_bytes_per_launch": 2.7e9},
        "kernels": {"block_fwd": k, "block_bwd": k},
        "sequential": {"value": 2.8e10, "ms_per_step": 11.6, "fwd_ms": 5.0, "bwd_ms": 6.6, "steps": 5,
                       "kind": "x" * 200, "per_step_launch_fwd_ms": 71.0},
        "speedup_vs_sequential": 11.6,
        "cpu_baseline": {"value": 1.4e9, "unit": "neuron-steps/s", "cores": 192, "kind": "oracle",
                         "cgroup_cpu_quota": 16.0,
                         "sample": "the whole workload (16384 (batch, neuron) rows x 20000 steps), forward + "
                                   "backward, 45 passes on 192 threads: 10.00 s wall, 160.0 CPU-s",
                         "one_core": {"value": 1.1e8, "cores": 1, "sample": "y" * 100}},
        "layers": {"three_layer": {"rows": ["z" * 100] * 200}},
        "recurrent": {"workload": "w" * 300},
        "speedup_sweep": {"rows": [{"T": 512, "x": "v" * 100}] * 40},
        "fits": {"rows": ["u" * 200] * 40},
        "serving": {"requests": 2000, "arrival_rate_hz": 200.0, "realtime": mode, "saturated": mode,
                    "stream": "s" * 300},
        "single_layer": {"as_specified": sl, "driven": sl, "workload": "t" * 200},
    }


def test_headline_is_compact_and_parses():
    import json
    line = json.dumps(bench.headline(_fake_result()))
    assert len(line) < 2048, len(line)
    h = json.loads(line)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in h, key
    assert set(h["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert h["config"]["workload"].startswith("fine-DT fit")
    assert h["cpu_baseline"]["cores"] == 192 and h["cpu_baseline"]["kind"] == "oracle"
    assert h["serving"]["realtime"]["p99_ms"] == 9.2
    assert h["single_layer"]["as_specified"]["blocks_in_sequence"] == 500


def test_headline_without_optional_legs():
    import json
    r = _fake_result()
    for k in ("cpu_baseline", "sequential", "serving", "single_layer"):
        r[k] = None
    h = json.loads(json.dumps(bench.headline(r)))
    assert "serving" not in h and h["value"] == 3.3e11
