"""Shared pieces of the GPU parity tests: seeded driven inputs and runners.

Inputs come from numpy PCG64 (no ALIF arithmetic here); the same arrays feed the
GPU library and, upcast to float64, the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np

from paper_2311_11390_amd.synth import LayerParams, rng


def log(msg: str) -> None:
    """Print and flush before a GPU step, so a crash still names its case."""
    print(msg, flush=True)
    sys.stdout.flush()
    sys.stderr.flush()


def driven_current(seed, B, T, N, lo=-0.5, hi=3.0, burst_p=0.03, burst=3.0):
    g = rng(seed)
    I = g.uniform(lo, hi, (B, T, N)).astype(np.float32)
    I += (g.random((B, T, N)) < burst_p).astype(np.float32) * np.float32(burst)
    return I


def random_params(seed, N, tm=(5.0, 30.0), ta=(50.0, 300.0), d=(0.0, 1.8), th=(0.8, 1.2),
                  bias=None) -> LayerParams:
    g = rng(seed + 1000)
    f = lambda lo_hi: g.uniform(lo_hi[0], lo_hi[1], N).astype(np.float32)
    return LayerParams(f(tm), f(ta), f(d), f(th), None if bias is None else f(bias))


def to_dev(prm: LayerParams):
    import torch

    from paper_2311_11390_amd.alif import Params
    return Params.from_numpy(prm, "cuda")


def gpu_forward(I, prm, dt, arp, algo=0, traces=True, save=False, init=None, want_final=False,
                spike_dtype=0, surrogate=0, grad_policy=0):
    import torch

    from paper_2311_11390_amd import alif
    It = torch.as_tensor(I, device="cuda").contiguous()
    P = to_dev(prm)
    f = alif.forward(It, P, dt, arp, algo=algo, want_v=traces, want_theta=traces, save=save,
                     init=init, want_final=want_final, spike_dtype=spike_dtype, surrogate=surrogate,
                     grad_policy=grad_policy)
    torch.cuda.synchronize()
    return f, It, P


def np_(t):
    return None if t is None else t.detach().float().cpu().numpy() if t.dtype in (
        __import__("torch").bfloat16,) else t.detach().cpu().numpy()
