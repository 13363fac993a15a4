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

Output. The last stdout line is a compact JSON headline (under 2 KB): whole-job
neuron-steps/s (B * N * T / step time), ms per step, the HBM roofline of the
dominant kernel (HIP events on the launch stream), the FP64 oracle on the host's
cores over the same workload, the fused sequential GPU kernels on the same work,
the serving leg's p50 / p99 latency and throughput (a Poisson stream of 2000
uneven requests under continuous batching) and the latency-bound single-layer
forward (200 -> 100, batch 1, T 1000: time and sequential depth). Every leg's
full results go to --detail-out: per-kernel durations, the three-layer BF16
and SHD-shaped training legs (each GEMM timed alone against the MFMA peak), the
recurrent leg, the block-vs-sequential speedup sweep and the speed-accuracy
sweeps. Progress and one-line summaries go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # MI355X dense, published


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(TR):
    """Bytes per neuron-step the method must move: forward reads I (4 B) and writes
    the spike (1 B) and, once per T_R-step block, the block's carry-in (V0 and a
    as float, the previous spike step as a byte: 9 B); the backward reads I and
    dL/dS (4 + 4 B) and the carries. Traces, gradients of I and anything the
    method could avoid are not counted."""
    return {"fwd": 4.0 + 1.0 + 9.0 / TR, "bwd": 8.0 + 9.0 / TR}


HERE = os.path.dirname(os.path.abspath(__file__))
COUNTERS = os.path.join(HERE, "profiles", "block_fwd_bwd_fine_dt_hbm_counters.md")
KERNEL_SOURCES = ["alif_blocks.hip", "alif_blocks_impl.h", "alif_blocks_s1.hip", "alif_blocks_s2.hip",
                  "alif_blocks_s4.hip", "alif_blocks_s8.hip", "alif_blocks_s8_long.hip", "alif_blocks_s8_xl.hip",
                  "alif_common.h", "alif_kernels.h"]


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in sorted(KERNEL_SOURCES):
        h.update(name.encode())
        try:
            with open(os.path.join(HERE, "paper_2311_11390_amd", "csrc", name), "rb") as f:
                h.update(f.read())
        except OSError:
            return None   # a listed source is gone: the counters cannot be matched
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by a copy kernel of known size), or {} when the kernel
    sources have changed since those counters were taken."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return {}
    digest, traffic = None, {}
    for line in text.splitlines():
        if line.startswith("kernel_sources_sha256:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch:"):
            for kv in line.split(":", 1)[1].split():
                k, v = kv.split("=")
                traffic[k] = float(v)
    cur = kernel_sources_digest()
    return traffic if cur is not None and digest == cur else {}


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


def _event_ms(fn, reps):
    """Average duration of fn() over reps calls, HIP events on the current stream
    (the library launches on it)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def three_layer_leg(steps, warmup, seed=4):
    """Three-layer spike-input network 700 -> 1024 -> 1024 -> 20, B 128, T 2000,
    DT 0.5 ms (T_R = 4), driven by a bias, BF16 GEMMs with FP32 accumulation.
    One step = the three forward layers (Eq. 3 GEMM + block kernels) and the
    backward chain of loss = sum of last-layer spikes (block backward, then
    dW = gI^T x and dx = gI W per layer). Also times every GEMM of the step on
    its own, against the BF16 MFMA peak, and each layer's forward current from
    its active inputs alone (the event kernel) beside the GEMM."""
    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif
    from paper_2311_11390_amd.synth import three_layer
    w = three_layer(seed=seed, driven=True)
    dev = "cuda"
    B, T = w.B, w.T
    x = torch.as_tensor(w.inputs["x"], device=dev)
    Ws = [torch.as_tensor(W, device=dev) for W in w.weights]
    Ps = [alif.Params.from_numpy(lp, dev) for lp in w.layers]
    prec = L.GEMM_BF16
    st = {}

    def step():
        h, fs, ins = x, [], []
        for W, P in zip(Ws, Ps):
            f = alif.forward(h, P, w.dt, w.arp, W, gemm_precision=prec, spike_dtype=L.SPIKES_U8, save=True)
            fs.append(f)
            ins.append(h)
            h = f["spikes"]
        g = torch.ones(h.shape, dtype=torch.float32, device=dev)
        for li in reversed(range(len(Ws))):
            gr = alif.backward(fs[li], ins[li], Ps[li], Ws[li], grad_spikes=g, want_grad_input=li > 0,
                               want_grad_W=True)
            g = gr["grad_input"] if li > 0 else None
        st["fs"], st["ins"] = fs, ins

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    neurons = sum(W.shape[0] for W in Ws)
    spikes = [int(f["spikes"].sum().item()) for f in st["fs"]]
    # the same step with each forward current from the active inputs (event kernel, FP32 weights; W transposed
    # in the step, as after every optimiser update); the backward is the block backward to gI and the same BF16
    # dW / dx GEMMs
    def step_events():
        h, fs, ins, curs = x, [], [], []
        for W, P in zip(Ws, Ps):
            cur = alif.input_current_events(h, alif.transpose(W))
            f = alif.forward(cur, P, w.dt, w.arp, spike_dtype=L.SPIKES_U8, save=True)
            fs.append(f)
            ins.append(h)
            curs.append(cur)
            h = f["spikes"]
        g = torch.ones(h.shape, dtype=torch.float32, device=dev)
        for li in reversed(range(len(Ws))):
            gI = alif.backward(fs[li], curs[li], Ps[li], grad_spikes=g, want_grad_current=True)["grad_current"]
            alif.weight_grad(gI, ins[li], gemm_precision=prec)
            g = alif.input_grad(gI, Ws[li], L.INPUT_SPIKES_U8, gemm_precision=prec) if li > 0 else None
        st["ev_fs"] = fs

    for _ in range(warmup):
        step_events()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_events()
    torch.cuda.synchronize()
    ms_ev = (time.perf_counter() - t0) / steps * 1e3
    st["ev_spikes"] = [int(f["spikes"].sum().item()) for f in st.pop("ev_fs")]

    gemms, events = {}, {}
    for li, (W, h) in enumerate(zip(Ws, st["ins"])):
        N, K = W.shape
        M = B * T
        flops = 2.0 * M * N * K
        gI = torch.randn(B, T, N, device=dev)
        calls = {f"L{li + 1} I = x W^T ({K} -> {N})": lambda: alif.input_current(h, W, None, gemm_precision=prec),
                 f"L{li + 1} dW = gI^T x": lambda: alif.weight_grad(gI, h, gemm_precision=prec)}
        if li > 0:
            calls[f"L{li + 1} dx = gI W"] = lambda: alif.input_grad(gI, W, L.INPUT_SPIKES_U8, gemm_precision=prec)
        for name, fn in calls.items():
            t = _event_ms(fn, 5)
            tf = flops / (t * 1e-3) / 1e12
            gemms[name] = {"ms": t, "tflops": tf, "frac_of_peak": tf / MFMA_PEAK_TFLOPS["bf16"]}
        # the same current from the active inputs only (FP32 weights, W transposed once)
        WT = alif.transpose(W)
        t = _event_ms(lambda: alif.input_current_events(h, WT), 20)
        t_gemm = gemms[f"L{li + 1} I = x W^T ({K} -> {N})"]["ms"]
        ev_bytes = M * (K * h.element_size() + 4 * N)     # inputs read + current written (HBM)
        events[f"L{li + 1} ({K} -> {N})"] = {"ms": t, "active_fraction": float((h != 0).float().mean().item()),
                                             "speedup_vs_bf16_gemm": t_gemm / t,
                                             "algorithmic_bytes": ev_bytes,
                                             "hbm_gbps": ev_bytes / (t * 1e-3) / 1e9,
                                             "frac_of_hbm_peak": ev_bytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del gI, WT
    del st["fs"], st["ins"]
    torch.cuda.synchronize()
    return {"workload": "three-layer 700 -> 1024 -> 1024 -> 20, B 128, T 2000, DT 0.5 ms, T_R 4, driven; "
                        "loss = sum of last-layer spikes; BF16 GEMMs (FP32 accumulate), uint8 spikes",
            "ms_per_step": ms, "value": B * T * neurons / (ms * 1e-3), "unit": "neuron-steps/s",
            "steps": steps, "spikes_per_layer": spikes,
            "gemm_peak_tflops": MFMA_PEAK_TFLOPS["bf16"], "gemms": gemms, "event_current": events,
            "event_forward_step": {"ms_per_step": ms_ev, "value": B * T * neurons / (ms_ev * 1e-3),
                                   "spikes_per_layer": st["ev_spikes"],
                                   "kind": "forward currents by the event kernel (FP32 W), backward as above"}}


def shd_like_leg(steps, warmup, seed=3):
    """SHD-shaped training step: 700 Bernoulli channels -> 512 ALIF -> 20 leaky
    readout, B 32, T 1000, DT 1 ms, driven by a bias, FP32 GEMMs; forward,
    cross-entropy and backward through torch.autograd with the library's ops."""
    import torch

    from paper_2311_11390_amd import alif
    from paper_2311_11390_amd.synth import shd_like_training
    w = shd_like_training(seed=seed, driven=True)
    dev = "cuda"
    lp = w.layers[0]
    xt = torch.as_tensor(w.inputs["x"], device=dev)
    Wt = torch.as_tensor(w.weights[0], device=dev).requires_grad_()
    P = {k: torch.as_tensor(getattr(lp, k), device=dev).requires_grad_()
         for k in ("tau_mem", "tau_adapt", "d", "theta0", "bias")}
    Wrt = torch.as_tensor(w.extra["readout_W"], device=dev).requires_grad_()
    trt = torch.as_tensor(w.extra["readout_tau"], device=dev).requires_grad_()
    labels = torch.as_tensor(w.inputs["labels"], device=dev)
    cfg = {"dt": w.dt, "arp": w.arp}

    def step():
        S, _, _ = alif.BlockALIF.apply(xt, Wt, P["tau_mem"], P["tau_adapt"], P["d"], P["theta0"], P["bias"], cfg)
        o = alif.Readout.apply(S, Wrt, trt, w.dt)
        loss = torch.nn.functional.cross_entropy(o, labels)
        loss.backward()
        return S

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    return {"workload": "SHD-shaped 700 -> 512 ALIF -> 20 readout, B 32, T 1000, DT 1 ms, T_R 2, driven; "
                        "cross-entropy; FP32 GEMMs; torch.autograd over the library's ops",
            "ms_per_step": ms, "value": w.B * w.T * 512 / (ms * 1e-3), "unit": "neuron-steps/s",
            "steps": steps, "spikes": int(S.sum().item())}


def speedup_sweep(steps=5, warmup=2):
    """Training-step speedup of the block kernels over the fused sequential kernels
    in the shapes of the paper's speed benchmarks: the synthetic Poisson spike
    dataset (rate per batch element ~ U[0, 200] Hz, one step = 1 ms), 200 inputs,
    ALIF layers with loss = total last-layer spike count, forward and backward
    (FP32 GEMMs, dW for every layer, dx between layers), B 64.
      * T in {512, 2048} x T_R in {2, 5, 10, 20, 40, 64, 80, 100, 120} (the sequential
        backward stages a block in LDS, which fits T_R <= 121), one layer of 256;
      * T = 1024, T_R = 40: 1-3 layers of 128, 256 or 512 units;
      * the supplementary's single-layer forward shape: 200 -> 100, T 1000, B 128, T_R 50.
    Both algorithms run the same GEMMs; only the ALIF kernels differ. Each row also
    times the forward alone against the per-step-launch forward (one kernel launch
    per time step, the cost structure of a step-by-step framework loop)."""
    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif
    from paper_2311_11390_amd.synth import speed_benchmark
    dev = "cuda"
    configs = [(T, TR, (256,), 64) for T in (512, 2048) for TR in (2, 5, 10, 20, 40, 64, 80, 100, 120)]
    configs += [(1024, 40, (h,) * n, 64) for n in (1, 2, 3) for h in (128, 256, 512)]
    configs += [(1000, 50, (100,), 128)]   # the single-layer forward timing shape of the supplementary
    rows = []
    for T, TR, hidden, B in configs:
        w = speed_benchmark(seed=T + TR + len(hidden) * hidden[0], B=B, T=T, hidden=hidden, TR=TR)
        x = torch.as_tensor(w.inputs["x"], device=dev)
        Ws = [torch.as_tensor(W, device=dev) for W in w.weights]
        Ps = [alif.Params.from_numpy(lp, dev) for lp in w.layers]
        res = {}
        for name, algo in (("block", L.ALGO_BLOCKS), ("sequential", L.ALGO_SEQUENTIAL)):
            def step():
                h, fs, ins = x, [], []
                for W, P in zip(Ws, Ps):
                    f = alif.forward(h, P, w.dt, w.arp, W, algo=algo, spike_dtype=L.SPIKES_U8, save=True)
                    fs.append(f)
                    ins.append(h)
                    h = f["spikes"]
                g = torch.ones(h.shape, dtype=torch.float32, device=dev)
                for li in reversed(range(len(Ws))):
                    gr = alif.backward(fs[li], ins[li], Ps[li], Ws[li], grad_spikes=g, want_grad_input=li > 0,
                                       want_grad_W=True)
                    g = gr["grad_input"] if li > 0 else None
                return fs
            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fs = step()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) / steps * 1e3
            if name == "block":
                res["spikes_last_layer"] = int(fs[-1]["spikes"].sum().item())
        for name, algo in (("block_fwd", L.ALGO_BLOCKS), ("per_step_fwd", L.ALGO_SEQUENTIAL_STEP)):
            def fwd():
                h = x
                for W, P in zip(Ws, Ps):
                    h = alif.forward(h, P, w.dt, w.arp, W, algo=algo, spike_dtype=L.SPIKES_U8)["spikes"]
            fwd()
            torch.cuda.synchronize()
            reps = 1 if algo == L.ALGO_SEQUENTIAL_STEP else steps
            t0 = time.perf_counter()
            for _ in range(reps):
                fwd()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) / reps * 1e3
        rows.append({"T": T, "T_R": TR, "layers": len(hidden), "hidden": hidden[0], "batch": B,
                     "block_ms": res["block"], "sequential_ms": res["sequential"],
                     "speedup": res["sequential"] / res["block"],
                     "block_fwd_ms": res["block_fwd"], "per_step_fwd_ms": res["per_step_fwd"],
                     "fwd_speedup_vs_per_step": res["per_step_fwd"] / res["block_fwd"],
                     "spikes_last_layer": res["spikes_last_layer"]})
        log(f"[bench] speedup B={B} T={T} T_R={TR} layers={len(hidden)}x{hidden[0]}: block {res['block']:.3f} ms, "
            f"sequential {res['sequential']:.3f} ms, x{rows[-1]['speedup']:.1f}; forward {res['block_fwd']:.3f} "
            f"ms vs per-step {res['per_step_fwd']:.2f} ms, x{rows[-1]['fwd_speedup_vs_per_step']:.0f}")
        del x, Ws, Ps
    return {"workload": "synthetic Poisson spikes (rate per batch element ~ U[0, 200] Hz), 200 inputs -> ALIF "
                        "layers, B 64, DT 1 ms, ARP = T_R ms, driven; loss = last-layer spike count; forward + "
                        "backward with FP32 GEMMs",
            "comparator": "fused sequential kernels (one thread per (batch, neuron), loop over t)",
            "steps": steps, "rows": rows}


def dt_error_sweep(reps=3, seed=21):
    """The speed-accuracy trade-off of simulating one layer at a coarser DT (the
    problem overview figure, panel b): 16 x 256 ALIF neurons with fixed input
    weights driven by 200 Poisson channels for 1 s (synth.dt_sweep_layer), the
    same input events binned at DT in {0.025, 0.05, 0.1, 0.2, 0.25, 0.5, 1} ms, ARP
    2 ms. Per DT: forward time (FP32 input GEMM + ALIF) of the block kernels, of
    the fused sequential kernels and of one launch per step, and the error of the
    spike trains against the DT = 0.025 ms run (its trains summed into the coarser
    bins): mean van Rossum distance at tau_R = 10 ms and 100 ms, and the relative
    error of the spike count."""
    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif, synth
    dev = "cuda"
    w = synth.dt_sweep_layer(seed)
    x_fine = w.inputs["x"]
    B, Tf, _ = x_fine.shape
    W = torch.as_tensor(w.weights[0], device=dev)
    P = alif.Params.from_numpy(w.layers[0], dev)
    N = W.shape[0]
    rows, ref = [], None
    for dt in (0.025, 0.05, 0.1, 0.2, 0.25, 0.5, 1.0):
        s = int(round(dt / w.dt))
        x = torch.as_tensor(synth.bin_counts(x_fine, s) if s > 1 else x_fine, device=dev)
        T = x.shape[1]
        Wd = (W / dt).contiguous()
        out = {"spikes": torch.empty(B, T, N, dtype=torch.uint8, device=dev),
               "current": torch.empty(B, T, N, dtype=torch.float32, device=dev)}
        row = {"dt_ms": dt, "T": T, "T_R": alif.refractory_steps(dt, w.arp)}
        for name, algo, n in (("sequential", L.ALGO_SEQUENTIAL, reps), ("per_step", L.ALGO_SEQUENTIAL_STEP, 1),
                              ("block", L.ALGO_BLOCKS, reps)):
            o = dict(out)
            if algo == L.ALGO_SEQUENTIAL_STEP:
                desc = alif.make_desc(B, T, N, dt, w.arp, x.shape[2], L.INPUT_SPIKES_U8, algo=algo)
                o["carries"] = torch.empty(alif.carry_bytes(desc), dtype=torch.uint8, device=dev)
            row[name + "_fwd_ms"] = _event_ms(lambda: alif.forward(x, P, dt, w.arp, Wd, algo=algo, out=o), n)
        S = out["spikes"]            # the block run's trains
        if ref is None:
            ref = S.clone()
        tgt = ref.view(B, T, s, N).sum(dim=2).to(torch.uint8).contiguous()
        for tau in (10.0, 100.0):
            d, _, _ = alif.van_rossum(S, tgt, dt, tau, want_grad=False)
            row[f"van_rossum_{tau:g}ms"] = float(d.mean().item())
        n_ref = float(ref.sum().item())
        row["spike_count_rel_err"] = abs(float(S.sum().item()) - n_ref) / n_ref
        row["rate_hz"] = float(S.sum().item()) / (B * N * w.T * w.dt * 1e-3)
        rows.append(row)
        log(f"[bench] dt sweep DT={dt}: block {row['block_fwd_ms']:.3f} ms, sequential "
            f"{row['sequential_fwd_ms']:.3f} ms, per-step {row['per_step_fwd_ms']:.1f} ms; van Rossum "
            f"{row['van_rossum_10ms']:.3f} (10 ms) {row['van_rossum_100ms']:.3f} (100 ms), "
            f"count err {row['spike_count_rel_err']:.3f}")
        del x, out, S
    return {"workload": f"{B} x {N} ALIF, 200 Poisson inputs (rate per batch element ~ U[20, 80] Hz), "
                        f"W ~ U[0, 0.26], 1 s, ARP 2 ms; error against DT {w.dt} ms",
            "reps": reps, "rows": rows}


FIT_GROUPS = (  # parameter, Adam learning rate, projection bounds
    ("tau_mem", 0.5, 1.0, 200.0), ("tau_adapt", 5.0, 5.0, 2000.0), ("d", 0.01, 0.0, 5.0),
    ("theta0", 0.01, 0.05, 10.0), ("bias", 0.01, -5.0, 5.0))


FIT_CONFIGS = ((0.1, 2.0), (0.1, 4.0), (0.1, 8.0), (0.2, 2.0), (0.5, 2.0), (1.0, 2.0), (2.0, 4.0), (4.0, 8.0))


def fit_sweep(epochs=100, seq_epochs=5, N=2048, seed=31, configs=FIT_CONFIGS):
    """Fitting ALIF neurons to recorded spike trains by minimising the van Rossum
    distance (tau_R 100 ms) with Adam, full batch, at several DT and ARP (the
    neural-fit figure's accuracy-versus-ARP and accuracy-versus-DT panels), on
    synthetic recordings (synth.neuron_fit): N ground-truth neurons simulated at
    DT 0.05 ms, ARP 2 ms, 4 fitting + 4 held-out OU stimuli of 2 s, 4 repeats each
    with independent intrinsic noise. Every fit starts from the same initial
    parameters; one epoch = forward on the fitting stimuli, van Rossum loss and
    gradient against all repeats, surrogate-gradient backward, one Adam step per
    parameter vector. Per configuration: ms per epoch, the mean distance on the
    fitting set (last epoch) and on the held-out set before and after fitting, the
    repeat-to-repeat distance of the recordings themselves (the floor), and the
    relative error of the recovered tau_mem and theta0; the held-out distance and
    the floor are also given at tau_R 10 ms, which weighs spike timing more. The DT 0.1 ms, ARP 2 ms fit
    is also timed with the fused sequential kernels."""
    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif, synth
    dev = "cuda"
    fs = synth.neuron_fit(seed, N=N)
    Tg = int(round(fs.duration_ms / fs.dt_ms))
    nb, R, ns = 2 * fs.n_stim, fs.repeats, fs.n_stim
    stim = torch.empty(nb, Tg, N, dtype=torch.float32, device=dev)
    for b in range(nb):
        alif.ou_current(Tg, N, fs.dt_ms, fs.stim_tau_ms, fs.amplitudes[b], fs.stim_sd, fs.seed * 1000 + b,
                        out=stim[b])
    gt = torch.empty(nb, R, Tg, N, dtype=torch.uint8, device=dev)
    Pt = alif.Params.from_numpy(fs.truth, dev)
    cur = torch.empty(R, Tg, N, dtype=torch.float32, device=dev)
    for b in range(nb):
        for r in range(R):
            alif.ou_current(Tg, N, fs.dt_ms, fs.noise_tau_ms, 0.0, fs.noise_sd, fs.seed * 1000 + 100 + b * R + r,
                            out=cur[r])
        cur += stim[b]
        alif.forward(cur, Pt, fs.dt_ms, fs.arp_ms, out={"spikes": gt[b]})
    del cur
    torch.cuda.synchronize()
    gt_rate = float(gt.sum().item()) / (nb * R * N * fs.duration_ms * 1e-3)
    log(f"[bench] fit: ground truth {nb} stimuli x {R} repeats x {N} neurons, {gt_rate:.1f} Hz")
    truth_tm = torch.as_tensor(fs.truth.tau_mem, device=dev)
    truth_th = torch.as_tensor(fs.truth.theta0, device=dev)

    def run(dt, arp, n_epochs, algo=L.ALGO_BLOCKS):
        s = int(round(dt / fs.dt_ms))
        Tc = Tg // s
        I_tr = stim[:ns].view(ns, Tc, s, N).mean(dim=2).contiguous()
        I_te = stim[ns:].view(ns, Tc, s, N).mean(dim=2).contiguous()
        y = gt.view(nb, R, Tc, s, N).sum(dim=3).to(torch.uint8)
        y_tr, y_te = y[:ns].contiguous(), y[ns:].contiguous()
        del y
        P = alif.Params.from_numpy(fs.init, dev)
        opt = {k: (torch.zeros(N, device=dev), torch.zeros(N, device=dev)) for k, *_ in FIT_GROUPS}
        desc = alif.make_desc(ns, Tc, N, dt, arp, algo=algo)
        out = {"spikes": torch.empty(ns, Tc, N, dtype=torch.uint8, device=dev),
               "carries": torch.empty(alif.carry_bytes(desc), dtype=torch.uint8, device=dev)}
        bws = torch.empty(max(1, alif.backward_workspace_bytes(desc)), dtype=torch.uint8, device=dev)
        vws = alif.van_rossum_workspace(ns, R, Tc, N, dev)
        gS = torch.empty(ns, Tc, N, dtype=torch.float32, device=dev)
        dist = torch.empty(ns, R, N, dtype=torch.float32, device=dev)

        def test_distance(tau):
            S = alif.forward(I_te, P, dt, arp, algo=algo)["spikes"]
            d, _, _ = alif.van_rossum(S, y_te, dt, tau, want_grad=False, workspace=vws)
            return float(d.mean().item())

        def floor(tau):
            d, _, _ = alif.van_rossum(y_te[:, 0].contiguous(), y_te[:, 1:].contiguous(), dt, tau, want_grad=False)
            return float(d.mean().item())

        row = {"dt_ms": dt, "arp_ms": arp, "T": Tc, "T_R": alif.refractory_steps(dt, arp)}
        if algo == L.ALGO_BLOCKS:
            row["test_distance_init"] = test_distance(100.0)
            row["repeat_floor"] = floor(100.0)
            row["repeat_floor_10ms"] = floor(10.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for ep in range(1, n_epochs + 1):
            f = alif.forward(I_tr, P, dt, arp, algo=algo, save=True, out=out)
            alif.van_rossum(f["spikes"], y_tr, dt, 100.0, scale=1.0 / (ns * R), dist=dist, grad=gS, workspace=vws)
            g = alif.backward(f, I_tr, P, grad_spikes=gS, workspace=bws)
            for name, lr, lo, hi in FIT_GROUPS:
                m, v = opt[name]
                alif.adam_step(getattr(P, name), g["grad_" + name], m, v, ep, lr, lo=lo, hi=hi)
            if ep == 1:
                d_first = dist.mean()
        e1.record()
        torch.cuda.synchronize()
        row["ms_per_epoch"] = e0.elapsed_time(e1) / n_epochs
        row["epochs"] = n_epochs
        if algo == L.ALGO_BLOCKS:
            # the loss alone (three kernels, one launch each), against the bytes it must
            # move: the model spikes and every target once (1 + R bytes) and the gradient
            # (4 bytes) per element
            S = out["spikes"]
            ms = _event_ms(lambda: alif.van_rossum(S, y_tr, dt, 100.0, scale=1.0 / (ns * R), dist=dist, grad=gS,
                                                   workspace=vws), 5)
            nbytes = float(ns) * Tc * N * (1 + R + 4)
            row["loss"] = {"avg_ms": ms, "bytes_per_launch": nbytes, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
                           "frac_of_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        row["train_distance_first"] = float(d_first.item())
        row["train_distance_last"] = float(dist.mean().item())
        if algo == L.ALGO_BLOCKS:
            row["test_distance_fit"] = test_distance(100.0)
            row["test_distance_fit_10ms"] = test_distance(10.0)
            row["tau_mem_rel_err"] = float(((P.tau_mem - truth_tm).abs() / truth_tm).mean().item())
            row["theta0_rel_err"] = float(((P.theta0 - truth_th).abs() / truth_th).mean().item())
            row["rate_hz"] = float(out["spikes"].sum().item()) / (ns * N * fs.duration_ms * 1e-3)
        del I_tr, I_te, y_tr, y_te, out, bws, vws, gS
        return row

    rows = []
    for dt, arp in configs:
        row = run(dt, arp, epochs)
        rows.append(row)
        log(f"[bench] fit DT={dt} ARP={arp}: {row['ms_per_epoch']:.2f} ms/epoch, train D "
            f"{row['train_distance_first']:.3f} -> {row['train_distance_last']:.3f}, test D "
            f"{row['test_distance_init']:.3f} -> {row['test_distance_fit']:.3f} (floor {row['repeat_floor']:.3f}; "
            f"at tau_R 10 ms {row['test_distance_fit_10ms']:.3f}, floor {row['repeat_floor_10ms']:.3f}), "
            f"tau_mem err {row['tau_mem_rel_err']:.3f}, theta0 err {row['theta0_rel_err']:.3f}, {row['rate_hz']:.1f} Hz; "
            f"loss {row['loss']['avg_ms']:.3f} ms = {row['loss']['frac_of_peak']:.2f} of HBM peak")
        torch.cuda.empty_cache()
    dt0, arp0 = configs[0]
    seq = run(dt0, arp0, seq_epochs, algo=L.ALGO_SEQUENTIAL) if seq_epochs > 0 else None
    if seq:
        log(f"[bench] fit DT={dt0} ARP={arp0} with the sequential kernels: {seq['ms_per_epoch']:.2f} ms/epoch")
    del stim, gt
    torch.cuda.empty_cache()
    return {"workload": f"{N} synthetic neurons, {ns} fitting + {ns} held-out OU stimuli of {fs.duration_ms:g} ms "
                        f"x {R} noisy repeats, ground truth at DT {fs.dt_ms} ms, ARP {fs.arp_ms} ms "
                        f"({gt_rate:.1f} Hz); van Rossum tau_R 100 ms; Adam, full batch",
            "adam_groups": [{"param": k, "lr": lr, "lo": lo, "hi": hi} for k, lr, lo, hi in FIT_GROUPS],
            "rows": rows,
            "sequential": None if seq is None else {
                "dt_ms": dt0, "arp_ms": arp0, "ms_per_epoch": seq["ms_per_epoch"], "epochs": seq_epochs,
                "speedup_block": seq["ms_per_epoch"] / rows[0]["ms_per_epoch"]}}


def recurrent_leg(w, I, P, gS, steps=3):
    """The fine-DT workload as a recurrent network: the OU current plus
    W_rec S[t - T_R] (W_rec ~ N(0, 0.5^2 / N)), T_R = 40, so 500 blocks run one
    after another inside one launch (a workgroup per batch element gathers each
    block's recurrent input from the previous block's spikes). Times the
    forward eagerly and as a captured HIP graph replay (torch.cuda.CUDAGraph on
    the library's launches), and the detached backward with dW_rec, next to the
    feedforward forward of the same shape."""
    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif
    B, T, N = I.shape
    g = np.random.default_rng(11)
    W_rec = torch.as_tensor((g.standard_normal((N, N)) * 0.5 / np.sqrt(N)).astype(np.float32), device="cuda")
    f = alif.forward_recurrent(I, P, w.dt, w.arp, W_rec)
    ws = f["workspace"]
    torch.cuda.synchronize()

    def fwd():
        return alif.forward_recurrent(I, P, w.dt, w.arp, W_rec, workspace=ws)

    t0 = time.perf_counter()
    for _ in range(steps):
        f = fwd()
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / steps * 1e3
    spikes = int(f["spikes"].sum().item())
    graph_ms = None
    try:
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            fg = fwd()
        cg.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            cg.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) / steps * 1e3
        assert torch.equal(fg["spikes"], f["spikes"]), "graph replay differs from the eager run"
        del cg, fg
    except Exception as e:   # report, keep the eager numbers
        log(f"[bench] recurrent graph capture failed: {e}")
    out = alif.backward_recurrent(f, I, P, grad_spikes=gS)   # warm-up (output allocations)
    del out
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = alif.backward_recurrent(f, I, P, grad_spikes=gS)
    torch.cuda.synchronize()
    bwd = (time.perf_counter() - t0) / steps * 1e3
    del out
    ff = alif.forward(I, P, w.dt, w.arp, save=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ff = alif.forward(I, P, w.dt, w.arp, save=True)
    torch.cuda.synchronize()
    ff_ms = (time.perf_counter() - t0) / steps * 1e3
    NB = (T + 39) // 40
    return {"workload": f"fine-DT shape as a recurrent network: {B} x {N} neurons, T {T}, T_R 40 ({NB} blocks in "
                        "sequence), OU current + W_rec S[t - T_R], W_rec ~ N(0, 0.25 / N), FP32 GEMMs",
            "forward_eager_ms": eager, "forward_graph_ms": graph_ms, "backward_ms": bwd,
            "feedforward_forward_ms": ff_ms, "spikes": spikes,
            "value": B * N * T / ((graph_ms or eager) + bwd) * 1e3, "unit": "neuron-steps/s (fwd + bwd)"}


def single_layer_leg(reps=50, seed=0):
    """The single-layer forward as specified: 200 Bernoulli(0.02) channels -> 100
    ALIF neurons, batch 1, T 1000, DT 1 ms, ARP 2 ms (T_R 2), FP32 input GEMM;
    and its driven variant (bias b ~ U[1, 2]), which fires. 100 neurons cannot
    fill the GPU: the time is the latency of 500 dependent blocks (1000 dependent
    steps for the sequential kernels), so no roofline applies. Each forward
    (GEMM + block kernel, or GEMM + sequential kernel) is timed with HIP events
    over ``reps`` calls."""
    import torch

    from paper_2311_11390_amd import _lib as L
    from paper_2311_11390_amd import alif
    from paper_2311_11390_amd.synth import single_layer
    out = {}
    for driven in (False, True):
        w = single_layer(seed=seed, driven=driven)
        x = torch.as_tensor(w.inputs["x"], device="cuda")
        W = torch.as_tensor(w.weights[0], device="cuda")
        P = alif.Params.from_numpy(w.layers[0], "cuda")
        B, T, N = w.B, w.T, W.shape[0]
        TR = alif.refractory_steps(w.dt, w.arp)
        row = {"blocks_in_sequence": -(-T // TR), "steps_in_sequence": T, "T_R": TR}
        sp = {}
        for name, algo in (("block", L.ALGO_BLOCKS), ("sequential", L.ALGO_SEQUENTIAL)):
            o = {"spikes": torch.empty(B, T, N, dtype=torch.uint8, device="cuda"),
                 "current": torch.empty(B, T, N, dtype=torch.float32, device="cuda")}
            row[name + "_fwd_ms"] = _event_ms(lambda: alif.forward(x, P, w.dt, w.arp, W, algo=algo, out=o), reps)
            sp[name] = o["spikes"]
        row["spikes"] = int(sp["block"].sum().item())
        row["block_equals_sequential"] = bool(torch.equal(sp["block"], sp["sequential"]))
        row["block_us_per_dependent_block"] = row["block_fwd_ms"] * 1e3 / row["blocks_in_sequence"]
        row["speedup_vs_sequential"] = row["sequential_fwd_ms"] / row["block_fwd_ms"]
        out["driven" if driven else "as_specified"] = row
        log(f"[bench] single layer{' (driven)' if driven else ''}: block fwd {row['block_fwd_ms'] * 1e3:.1f} us "
            f"({row['blocks_in_sequence']} blocks in sequence), sequential fwd {row['sequential_fwd_ms'] * 1e3:.1f} us "
            f"({T} steps), {row['spikes']} spikes")
    out["workload"] = ("single layer 200 -> 100, batch 1, T 1000, DT 1 ms, ARP 2 ms (T_R 2), Bernoulli(0.02) "
                       "input, FP32 input GEMM; latency-bound, time and sequential depth only")
    return out


def cgroup_cpu_quota():
    """CPUs the process's cgroup may use (cpu.max quota / period), or None."""
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        return None if q == "max" else float(q) / float(per)
    except (OSError, ValueError):
        return None


def cpu_baseline(w, cpu_seconds, threads):
    """FP64 oracle fwd + bwd over the whole workload (every (batch, neuron) row, all
    T steps), repeated in whole passes until `cpu_seconds` of CPU time (summed
    over the threads) have been spent."""
    import oracle
    from oracle import _to_rows
    I = w.inputs["I"]
    Irows = _to_rows(I.astype(np.float64))
    B, T, N = I.shape
    lp = w.layers[0]
    tile = lambda q: np.tile(np.asarray(q, np.float64), B)
    prm = [tile(lp.tau_mem), tile(lp.tau_adapt), tile(lp.d), tile(lp.theta0)]
    g = np.random.default_rng(1).standard_normal(Irows.shape)
    TR = oracle.refractory_steps(w.dt, w.arp)
    oracle.set_threads(threads)
    passes, c0, t0 = 0, time.process_time(), time.perf_counter()
    while passes == 0 or time.process_time() - c0 < cpu_seconds:
        fw = oracle.forward_rows(Irows, *prm, w.dt, TR)
        oracle.backward_rows(fw, *prm, w.dt, 10.0, gS=g, want_gI=False)
        del fw
        passes += 1
    el, cpu = time.perf_counter() - t0, time.process_time() - c0
    return Irows.size * passes / el, el, cpu, passes, Irows.shape[0]


def cpu_baseline_one_core(w, rows):
    """The same oracle on one thread over the first `rows` (batch, neuron) rows
    (all of them by default), one forward + backward pass."""
    import oracle
    from oracle import _to_rows
    I = w.inputs["I"]
    B, T, N = I.shape
    Irows = _to_rows(I.astype(np.float64))[:rows]
    lp = w.layers[0]
    tile = lambda q: np.tile(np.asarray(q, np.float64), B)[:rows]
    prm = [tile(lp.tau_mem), tile(lp.tau_adapt), tile(lp.d), tile(lp.theta0)]
    g = np.random.default_rng(1).standard_normal(Irows.shape)
    TR = oracle.refractory_steps(w.dt, w.arp)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    fw = oracle.forward_rows(Irows, *prm, w.dt, TR)
    oracle.backward_rows(fw, *prm, w.dt, 10.0, gS=g, want_gI=False)
    el = time.perf_counter() - t0
    return Irows.size / el, el, Irows.shape[0]


def serve_leg(n_requests, rate_hz, max_slots, budget_gib, output="events", seed=1):
    """Replay a Poisson request stream (uneven N, T and DT; OU current drawn on the
    device) against the library's server in real time, then the same stream
    submitted all at once. Latency = completion - submission on the server's
    clock; throughput = neuron-steps of all requests / (last completion - first
    submission)."""
    from paper_2311_11390_amd import serving, synth
    stream = synth.request_stream(seed=seed, n=n_requests + 8, rate_hz=rate_hz)
    warm, stream = stream[:8], stream[8:]
    t_shift = stream[0].arrival_s

    def req(q):
        lp = synth.request_params(q)
        TR = int(round(q.arp / q.dt))
        cap = max(1024, -(-q.T // TR) * q.N // 4) if output == "events" else 0
        return serving.Request(T=q.T, dt=q.dt, arp=q.arp, tau_mem=lp.tau_mem, tau_adapt=lp.tau_adapt,
                               d=lp.d, theta0=lp.theta0, seed=q.seed, want_spikes=output == "raster",
                               events_capacity=cap, **{"ou_" + k: v for k, v in synth.REQUEST_OU.items()})

    reqs = [req(q) for q in stream]
    work = float(sum(q.N * q.T for q in stream))
    out = {"requests": len(stream), "arrival_rate_hz": rate_hz, "max_slots": max_slots,
           "budget_GiB": budget_gib, "neuron_steps": work,
           "stream": "Poisson arrivals; N ~ U{64..2048}, T ~ U{500..50000}, DT in {1, 0.1, 0.05} ms, "
                     "ARP 2 ms; OU current (tau 5 ms, mean 0.8, sd 0.5) drawn on the device; "
                     + ("spikes returned as event lists (flat t * N + n indices)" if output == "events" else
                        "spikes returned as dense [T][N] rasters"),
           "output": output}
    with serving.Server(int(budget_gib * (1 << 30)), max_slots=max_slots) as srv:
        for t in [srv.submit(req(q)) for q in warm]:     # pool and staging warm-up
            srv.wait(t, timeout=120)
        for mode in ("realtime", "saturated"):
            pending, results = {}, []
            t0 = time.perf_counter()
            for i, (q, r) in enumerate(zip(stream, reqs)):
                if mode == "realtime":
                    while time.perf_counter() - t0 < q.arrival_s - t_shift:
                        for tk in list(pending):
                            res = srv.poll(tk)
                            if res is not None:
                                res.spikes = res.events = None
                                results.append(res)
                                del pending[tk]
                        time.sleep(2e-4)
                pending[srv.submit(r)] = i
            while pending:
                for tk in list(pending):
                    res = srv.poll(tk)
                    if res is not None:
                        res.spikes = res.events = None
                        results.append(res)
                        del pending[tk]
                time.sleep(2e-4)
            bad = [r.status for r in results if r.status != 0 or r.events_truncated]
            lat = np.array([r.latency for r in results]) * 1e3
            span = max(r.t_done for r in results) - min(r.t_submit for r in results)
            out[mode] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                         "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                         "neuron_steps_per_s": work / span, "span_s": span, "failed": len(bad)}
            log(f"[bench] serving {mode}: p50 {out[mode]['p50_ms']:.2f} ms, p99 {out[mode]['p99_ms']:.2f} ms, "
                f"{out[mode]['neuron_steps_per_s']:.3e} neuron-steps/s over {span:.2f} s")
            del results
    return out


def copy_rate(torch, dev, mib=512, reps=5):
    """What a plain device-to-device copy reaches on this GPU (torch's copy, timed
    with HIP events on torch's stream): bytes read plus bytes written per second,
    in GB/s. Context for the HBM roofline, whose peak stays the published 8 TB/s."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def headline(res):
    """The compact result line (well under 2 KB): the contract's keys, the roofline
    and CPU baseline of the timed step, the sequential comparator, and one-line
    summaries of the serving and single-layer legs. Everything else stays in the
    detail file."""
    r3 = lambda v: None if v is None else float(f"{v:.4g}")
    out = {k: res[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                               "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    c = res["config"]
    out["config"] = {"workload": c["workload"], "global_batch": c["batch"], "neurons": c["neurons"],
                     "seq_len": c["T"], "T_R": c["T_R"], "parallelism": "single GPU"}
    rf = res["roofline"]
    out["roofline"] = {"bound": rf["bound"], "kernel": rf["kernel"], "achieved": r3(rf["achieved"]),
                       "peak": rf["peak"], "unit": rf["unit"], "frac": r3(rf["frac"]),
                       "traffic": rf["traffic"], "copy_GBs": r3(rf.get("copy_GBs")),
                       "frac_of_copy": r3(rf.get("frac_of_copy"))}
    out["kernels_ms"] = {k: r3(v["avg_ms"]) for k, v in res["kernels"].items()}
    cpu = res.get("cpu_baseline")
    if cpu:
        out["cpu_baseline"] = {"value": r3(cpu["value"]), "unit": cpu["unit"], "cores": cpu["cores"],
                               "kind": cpu["kind"], "sample": cpu["sample"],
                               "one_core": r3(cpu["one_core"]["value"])}
    seq = res.get("sequential")
    if seq:
        out["sequential"] = {"value": r3(seq["value"]), "ms_per_step": r3(seq["ms_per_step"]),
                             "speedup": r3(res["speedup_vs_sequential"])}
    sv = res.get("serving")
    if sv:
        out["serving"] = {"requests": sv["requests"], "rate_hz": sv["arrival_rate_hz"]}
        for mode in ("realtime", "saturated"):
            m = sv.get(mode)
            if m:
                out["serving"][mode] = {"p50_ms": r3(m["p50_ms"]), "p99_ms": r3(m["p99_ms"]),
                                        "neuron_steps_per_s": r3(m["neuron_steps_per_s"]), "failed": m["failed"]}
    sl = res.get("single_layer")
    if sl:
        out["single_layer"] = {k: {"block_fwd_ms": r3(v["block_fwd_ms"]), "sequential_fwd_ms": r3(v["sequential_fwd_ms"]),
                                   "blocks_in_sequence": v["blocks_in_sequence"], "spikes": v["spikes"]}
                               for k, v in sl.items() if isinstance(v, dict)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--no-layers", action="store_true",
                    help="skip the three-layer and SHD-shaped training legs")
    ap.add_argument("--no-recurrent", action="store_true", help="skip the recurrent-network leg")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the block-vs-sequential speedup sweep over T, T_R, layers and width")
    ap.add_argument("--no-fit", action="store_true",
                    help="skip the DT error sweep and the neural-fit sweep over DT and ARP")
    ap.add_argument("--fit-epochs", type=int, default=100)
    ap.add_argument("--fit-configs", default=",".join(f"{d:g}:{a:g}" for d, a in FIT_CONFIGS),
                    help="DT:ARP pairs (ms) of the neural-fit sweep; the first is also fitted with the "
                         "sequential kernels")
    ap.add_argument("--fit-seq-epochs", type=int, default=5)
    ap.add_argument("--no-dt-sweep", action="store_true", help="skip the simulation-error-versus-DT sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU time (summed over threads) the oracle baseline runs for, in whole passes")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests in the serving leg (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--serve-output", choices=("events", "raster"), default="events")
    ap.add_argument("--B", type=int, default=64)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--T", type=int, default=20000)
    ap.add_argument("--no-single-layer", action="store_true",
                    help="skip the latency-bound single-layer forward (200 -> 100, B 1, T 1000)")
    ap.add_argument("--detail-out", default=os.path.join(HERE, "gpurun_out", "bench_detail.json"),
                    help="file the full per-leg results are written to (the last stdout line is a compact "
                         "headline); empty to skip")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (a kernel of known "
                         "traffic, for scaling HBM byte counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (got --gpus {args.gpus}); the path would "
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
    copy_gbs = copy_rate(torch, dev)
    log(f"[bench] device-to-device copy: {copy_gbs:.0f} GB/s (bytes read + written)")
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

    recurrent = None
    if not args.no_recurrent:
        log("[bench] recurrent network on the fine-DT shape")
        recurrent = recurrent_leg(w, I, P, gS)
        log(f"[bench] recurrent: forward {recurrent['forward_eager_ms']:.2f} ms eager, "
            f"{recurrent['forward_graph_ms']} ms graph; backward {recurrent['backward_ms']:.2f} ms")
        torch.cuda.empty_cache()

    layers = None
    if not args.no_layers:
        log("[bench] three-layer BF16 training step")
        layers = {"three_layer": three_layer_leg(max(3, args.steps // 4), 2)}
        log(f"[bench] three-layer: {layers['three_layer']['ms_per_step']:.3f} ms/step")
        log("[bench] SHD-shaped training step")
        layers["shd_like"] = shd_like_leg(max(5, args.steps // 2), 2)
        log(f"[bench] SHD-shaped: {layers['shd_like']['ms_per_step']:.3f} ms/step")
        torch.cuda.empty_cache()

    sweep = None
    if not args.no_sweep:
        log("[bench] block-vs-sequential speedup sweep")
        sweep = speedup_sweep()
        torch.cuda.empty_cache()

    fits = None
    if not args.no_fit:
        fits = {}
        if not args.no_dt_sweep:
            log("[bench] simulation error versus DT")
            fits["dt_error"] = dt_error_sweep()
            torch.cuda.empty_cache()
        log("[bench] neural fits versus DT and ARP")
        cfgs = tuple(tuple(float(v) for v in c.split(":")) for c in args.fit_configs.split(","))
        fits["neuron_fit"] = fit_sweep(args.fit_epochs, args.fit_seq_epochs, configs=cfgs)
        torch.cuda.empty_cache()

    single = None
    if not args.no_single_layer:
        log("[bench] single-layer forward (latency-bound)")
        single = single_layer_leg()

    cpu = None
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        quota = cgroup_cpu_quota()
        log(f"[bench] oracle CPU baseline: whole workload, {threads} threads (every core in the affinity "
            f"mask; cgroup CPU quota {quota}), >= {args.cpu_seconds} CPU-s")
        rate, el, cpu_s, passes, rows = cpu_baseline(w, args.cpu_seconds, threads)
        log(f"[bench] oracle on {threads} threads: {rate:.3e} neuron-steps/s")
        r1, el1, rows1 = cpu_baseline_one_core(w, rows)
        log(f"[bench] oracle on one core: {r1:.3e} neuron-steps/s")
        cpu = {"value": rate, "unit": "neuron-steps/s", "cores": threads, "kind": "oracle",
               "cgroup_cpu_quota": quota,
               "sample": f"the whole workload ({rows} (batch, neuron) rows x {T} steps), forward + "
                         f"backward, {passes} passes on {threads} threads: {el:.2f} s wall, {cpu_s:.1f} CPU-s",
               "one_core": {"value": r1, "cores": 1,
                            "sample": f"the whole workload ({rows1} rows x {T} steps), forward + backward, "
                                      f"one pass on one thread: {el1:.2f} s"}}

    serve = None
    if args.serve_requests > 0:
        del I, P, Ptgt, gS, fb, bb
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"[bench] serving: {args.serve_requests} requests at {args.serve_rate}/s")
        serve = serve_leg(args.serve_requests, args.serve_rate, args.serve_slots, args.serve_budget_gib,
                          args.serve_output)

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
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["frac_of_peak"],
                     "traffic": measured_traffic().get(dom_name),
                     "algorithmic_bytes_per_launch": dom["bytes_per_launch"],
                     "copy_GBs": copy_gbs, "frac_of_copy": dom["achieved_GBs"] / copy_gbs},
        "kernels": {"block_fwd": k_fwd, "block_bwd": k_bwd},
        "sequential": seq,
        "speedup_vs_sequential": (value / seq["value"]) if seq else None,
        "cpu_baseline": cpu,
        "layers": layers,
        "recurrent": recurrent,
        "speedup_sweep": sweep,
        "fits": fits,
        "serving": serve,
        "single_layer": single,
    }
    if args.detail_out:
        try:
            os.makedirs(os.path.dirname(os.path.abspath(args.detail_out)), exist_ok=True)
            with open(args.detail_out, "w") as f:
                json.dump(res, f, indent=1)
            log(f"[bench] full results written to {args.detail_out}")
        except OSError as e:
            log(f"[bench] could not write {args.detail_out}: {e}")
    print(json.dumps(headline(res)), flush=True)


if __name__ == "__main__":
    main()
