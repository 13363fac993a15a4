#!/usr/bin/env python3
"""Benchmark of the block-wise ALIF hot path on one MI355X.

Workload (the fine-DT fitting configuration): 256 independent ALIF neurons x
batch 64, T = 20000 steps at DT = 0.05 ms, ARP = 2 ms (40-step blocks), driven
by an Ornstein-Uhlenbeck current (tau 5 ms, mean 0.8, sd 0.5), per-neuron
tau_mem ~ U[10, 30] ms, tau_adapt ~ U[100, 300] ms, d = 1.8, theta0 = 1. The
input current is resident in HBM before timing starts.

One step = alif_forward (block integrate + first crossing + carry, spikes and
block carries written) + alif_backward (recompute + reverse adjoint, gradients
for tau_mem, tau_adapt, d, theta0 and bias) on that input. The upstream
gradient dL/dS is the gradient of a Gaussian-smoothed (sigma 2 ms) MSE against
target trains simulated with perturbed parameters; it is computed once before
timing (the loss is not part of the ALIF path).

Printed JSON (last stdout line): whole-job neuron-steps/s (B * N * T / step
time), the sequential per-step GPU kernels on the same work, per-kernel HIP
event durations, the HBM roofline of the dominant kernel and the FP64 oracle on
host cores over a bounded sample of rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(TR):
    """Bytes per neuron-step the method must move (see the design notes):
    forward: read I (4) + write S (1) + block carry (9 B per neuron-block);
    backward: read I (4) + read dL/dS (4) + read block carry."""
    return {"fwd": 4.0 + 1.0 + 9.0 / TR, "bwd": 8.0 + 9.0 / TR}


def smoothed_mse_grad(S, S_tgt, sigma_steps):
    """d/dS of mean((G*S - G*S_tgt)^2), G a unit-sum Gaussian (+-4 sigma), 'same'
    convolution along time; computed with torch on the GPU."""
    import torch
    h = int(np.ceil(4 * sigma_steps))
    k = torch.exp(-0.5 * (torch.arange(-h, h + 1, device=S.device, dtype=torch.float32) / sigma_steps) ** 2)
    k = k / k.sum()
    B, T, N = S.shape
    nfft = 1 << int(np.ceil(np.log2(T + 2 * h + 1)))
    kf = torch.fft.rfft(k, n=nfft)

    def conv(x):   # 'same' linear convolution along time via FFT
        y = torch.fft.irfft(torch.fft.rfft(x.float(), n=nfft, dim=1) * kf.view(1, -1, 1), n=nfft, dim=1)
        return y[:, h:h + T, :]

    diff = conv(S.float()) - conv(S_tgt.float())
    g = conv(2.0 * diff / diff.numel())
    return g.contiguous()


def time_steps(fn_fwd, fn_bwd, steps, warmup):
    import torch
    for _ in range(warmup):
        fn_fwd()
        fn_bwd()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record()
        fn_fwd()
        e1.record()
        fn_bwd()
        e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = [a.elapsed_time(b) for a, b, _ in ev]
    bwd = [b.elapsed_time(c) for _, b, c in ev]
    return wall, np.array(fwd), np.array(bwd)


def cpu_baseline(w, rows, threads):
    """FP64 oracle fwd + bwd on the first `rows` (batch, neuron) rows, full T."""
    import oracle
    from oracle import _to_rows
    I = w.inputs["I"]
    B, T, N = I.shape
    nb = max(1, rows // N)
    Irows = _to_rows(I[:nb].astype(np.float64))
    lp = w.layers[0]
    tile = lambda q: np.tile(np.asarray(q, np.float64), nb)
    prm = [tile(lp.tau_mem), tile(lp.tau_adapt), tile(lp.d), tile(lp.theta0)]
    g = np.random.default_rng(1).standard_normal(Irows.shape)
    TR = oracle.refractory_steps(w.dt, w.arp)
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    fw = oracle.forward_rows(Irows, *prm, w.dt, TR)
    oracle.backward_rows(fw, *prm, w.dt, 10.0, gS=g, want_gI=False)
    el = time.perf_counter() - t0
    return Irows.size / el, el, Irows.shape[0]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=8192)
    ap.add_argument("--B", type=int, default=64)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--T", type=int, default=20000)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (a kernel of known "
                         "traffic, for scaling HBM byte counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); the path would "
              "shard independent (batch, neuron) rows across GPUs with no exchange, which is not run here.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L.load()
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calibrate_copy_mib} MiB read + {args.calibrate_copy_mib} MiB written")
        del src, dst
    log("[bench] generating the fine-DT OU workload")
    w = synth.fine_dt_fit(seed=0, B=args.B, N=args.N, T=args.T)
    B, T, N = w.inputs["I"].shape
    TR = alif.refractory_steps(w.dt, w.arp)
    I = torch.from_numpy(w.inputs["I"]).to(dev)
    P = alif.Params.from_numpy(w.layers[0], dev)
    Ptgt = alif.Params.from_numpy(w.extra["target_params"], dev)
    torch.cuda.synchronize()

    log("[bench] target trains and loss gradient")
    S = alif.forward(I, P, w.dt, w.arp, spike_dtype=L.SPIKES_F32)["spikes"]
    S_tgt = alif.forward(I, Ptgt, w.dt, w.arp, spike_dtype=L.SPIKES_F32)["spikes"]
    gS = smoothed_mse_grad(S, S_tgt, w.extra["sigma_steps"])
    rate_hz = float(S.sum().item()) / (B * N * T * w.dt * 1e-3)
    del S, S_tgt
    torch.cuda.synchronize()

    def make(algo):
        desc = alif.make_desc(B, T, N, w.dt, w.arp, algo=algo)
        out = {"spikes": torch.empty(B, T, N, dtype=torch.uint8, device=dev),
               "carries": torch.empty(alif.carry_bytes(desc), dtype=torch.uint8, device=dev)}
        ws = torch.empty(alif.backward_workspace_bytes(desc), dtype=torch.uint8, device=dev)
        st = {}

        def fwd():
            st["f"] = alif.forward(I, P, w.dt, w.arp, algo=algo, save=True, out=out)

        def bwd():
            alif.backward(st["f"], I, P, grad_spikes=gS, workspace=ws)
        return fwd, bwd

    log(f"[bench] block-wise fwd+bwd: warmup {args.warmup}, steps {args.steps}")
    fb, bb = make(L.ALGO_BLOCKS)
    wall, fwd_ms, bwd_ms = time_steps(fb, bb, args.steps, args.warmup)
    ms_step = wall / args.steps * 1e3
    ns = float(B) * N * T
    value = ns / (wall / args.steps)
    log(f"[bench] blocks: {ms_step:.3f} ms/step, fwd {np.mean(fwd_ms):.3f} ms, bwd {np.mean(bwd_ms):.3f} ms")

    ab = algorithmic_bytes(TR)
    k_fwd = {"avg_ms": float(np.mean(fwd_ms)), "bytes_per_launch": ab["fwd"] * ns}
    k_bwd = {"avg_ms": float(np.mean(bwd_ms)), "bytes_per_launch": ab["bwd"] * ns}
    for k in (k_fwd, k_bwd):
        k["achieved_GBs"] = k["bytes_per_launch"] / (k["avg_ms"] * 1e-3) / 1e9
        k["frac_of_peak"] = k["achieved_GBs"] / HBM_PEAK_GBS
    dom_name, dom = max((("block_bwd", k_bwd), ("block_fwd", k_fwd)), key=lambda kv: kv[1]["avg_ms"])

    seq = None
    if not args.no_sequential:
        log("[bench] sequential fused fwd+bwd")
        fs, bs = make(L.ALGO_SEQUENTIAL)
        steps_seq = max(3, args.steps // 4)
        wall_s, fwd_s, bwd_s = time_steps(fs, bs, steps_seq, 2)
        seq = {"value": ns / (wall_s / steps_seq), "ms_per_step": wall_s / steps_seq * 1e3,
               "fwd_ms": float(np.mean(fwd_s)), "bwd_ms": float(np.mean(bwd_s)), "steps": steps_seq,
               "kind": "one thread per (batch, neuron), fused loop over t, FP64 state"}
        log(f"[bench] sequential: {seq['ms_per_step']:.3f} ms/step")
        # per-step launches (forward only; context)
        desc = alif.make_desc(B, T, N, w.dt, w.arp, algo=L.ALGO_SEQUENTIAL_STEP)
        car = torch.empty(alif.carry_bytes(desc), dtype=torch.uint8, device=dev)
        sp = torch.empty(B, T, N, dtype=torch.uint8, device=dev)
        alif.forward(I, P, w.dt, w.arp, algo=L.ALGO_SEQUENTIAL_STEP, out={"spikes": sp, "carries": car})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alif.forward(I, P, w.dt, w.arp, algo=L.ALGO_SEQUENTIAL_STEP, out={"spikes": sp, "carries": car})
        torch.cuda.synchronize()
        seq["per_step_launch_fwd_ms"] = (time.perf_counter() - t0) * 1e3
        del car, sp

    cpu = None
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        threads = min(threads, 16)
        log(f"[bench] oracle CPU baseline on {args.cpu_rows} rows x {T} steps, {threads} threads")
        rate, el, rows = cpu_baseline(w, args.cpu_rows, threads)
        cpu = {"value": rate, "unit": "neuron-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"first {rows} (batch, neuron) rows of the workload, all {T} steps, "
                         f"forward + backward, {el:.2f} s wall"}

    res = {
        "metric": "neuron-steps/s fwd+bwd, block-wise vs sequential ALIF on 1 GPU; p99 latency",
        "value": value,
        "unit": "neuron-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fine-DT fit: {N} ALIF neurons x batch {B}, T={T}, DT={w.dt} ms, "
                               f"ARP={w.arp} ms (T_R={TR}), OU current, forward+backward",
                   "batch": B, "neurons": N, "T": T, "dt_ms": w.dt, "arp_ms": w.arp, "T_R": TR,
                   "firing_rate_hz": rate_hz},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": dom["achieved_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["frac_of_peak"], "traffic": None},
        "kernels": {"block_fwd": k_fwd, "block_bwd": k_bwd},
        "sequential": seq,
        "speedup_vs_sequential": (value / seq["value"]) if seq else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
