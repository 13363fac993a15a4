"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws random numbers and nothing else: it holds none of the ALIF
arithmetic, so the GPU path and the FP64 oracle can both be fed from it. All
draws use numpy's PCG64 with an explicit seed and are returned as the exact
float32 / uint8 arrays the GPU consumes (the oracle upcasts them).

Workload shapes:

* Bernoulli input spikes per step (the supplementary "Synthetic spike dataset"
  draws a homogeneous Poisson train per sample; the workloads here fix the rate
  per step or per channel instead).
* Ornstein-Uhlenbeck injected current, exact discretisation
  I[t+1] = mu + (I[t] - mu) e + sd sqrt(1 - e^2) xi,  e = exp(-DT/tau),
  with I[0] drawn from the stationary law N(mu, sd^2).
* Per-neuron time constants drawn uniformly, Normal(0, 1/sqrt(fan_in)) weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def bernoulli_spikes(g: np.random.Generator, shape, prob) -> np.ndarray:
    """uint8 0/1 spikes; ``prob`` is a scalar or broadcasts against ``shape``."""
    u = g.random(shape, dtype=np.float32)
    return (u < np.asarray(prob, dtype=np.float32)).astype(np.uint8)


def ou_current(g: np.random.Generator, B: int, T: int, N: int, dt_ms: float,
               tau_ms: float = 5.0, mu: float = 0.8, sd: float = 0.5) -> np.ndarray:
    """Ornstein-Uhlenbeck current [B][T][N] float32 (exact discretisation)."""
    e = np.exp(-dt_ms / tau_ms)
    s = sd * np.sqrt(1.0 - e * e)
    out = np.empty((B, T, N), dtype=np.float32)
    x = mu + sd * g.standard_normal((B, N))
    out[:, 0, :] = x
    chunk = 256
    for t0 in range(1, T, chunk):
        t1 = min(T, t0 + chunk)
        xi = g.standard_normal((B, t1 - t0, N))
        for k in range(t1 - t0):
            x = mu + (x - mu) * e + s * xi[:, k, :]
            out[:, t0 + k, :] = x
    return out


def normal_weights(g: np.random.Generator, n_out: int, n_in: int) -> np.ndarray:
    """W ~ N(0, sd = 1/sqrt(n_in)), [n_out][n_in] float32."""
    return (g.standard_normal((n_out, n_in)) / np.sqrt(n_in)).astype(np.float32)


def uniform(g: np.random.Generator, lo: float, hi: float, n: int) -> np.ndarray:
    return g.uniform(lo, hi, n).astype(np.float32)


def const(v: float, n: int) -> np.ndarray:
    return np.full(n, v, dtype=np.float32)


@dataclass
class LayerParams:
    """Per-neuron ALIF parameters, float32 [N] each. ``d`` is the adaptation scalar
    (the paper's d; the workload tables call it "beta")."""
    tau_mem: np.ndarray
    tau_adapt: np.ndarray
    d: np.ndarray
    theta0: np.ndarray
    bias: np.ndarray | None = None


def layer_params(g, N, tau_mem=(20.0, 20.0), tau_adapt=(200.0, 200.0), d=1.8, theta0=1.0,
                 bias=None) -> LayerParams:
    tm = uniform(g, *tau_mem, N) if tau_mem[0] != tau_mem[1] else const(tau_mem[0], N)
    ta = uniform(g, *tau_adapt, N) if tau_adapt[0] != tau_adapt[1] else const(tau_adapt[0], N)
    b = None if bias is None else uniform(g, bias[0], bias[1], N)
    return LayerParams(tm, ta, const(d, N), const(theta0, N), b)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    B: int
    T: int
    dt: float
    arp: float
    sizes: list          # [n_in, n1, n2, ...]; n_in == 0 means injected current
    inputs: dict = field(default_factory=dict)
    layers: list = field(default_factory=list)
    weights: list = field(default_factory=list)
    extra: dict = field(default_factory=dict)


def single_layer(seed=0, driven=False, B=1, T=1000) -> Workload:
    """200 Bernoulli(0.02) channels -> 100 ALIF, DT 1 ms, ARP 2 ms, T=1000.

    ``driven`` adds a bias b ~ U[1, 2] (Eq. 3's constant source) so that the layer
    fires; without it this layer stays below threshold."""
    g = rng(seed)
    x = bernoulli_spikes(g, (B, T, 200), 0.02)
    W = normal_weights(g, 100, 200)
    lp = layer_params(g, 100, bias=(1.0, 2.0) if driven else None)
    return Workload("single_layer_200x100" + ("_driven" if driven else ""), B, T, 1.0, 2.0,
                    [200, 100], {"x": x}, [lp], [W])


def shd_like_training(seed=0, driven=False, B=32, T=1000) -> Workload:
    """700 Bernoulli channels (rate_j ~ U[0,50] Hz) -> 512 ALIF -> 20 leaky readout,
    DT 1 ms, ARP 2 ms, per-neuron tau_m ~ U[10,30], tau_a ~ U[100,300], random labels."""
    g = rng(seed)
    dt = 1.0
    rates_hz = g.uniform(0.0, 50.0, 700)
    x = bernoulli_spikes(g, (B, T, 700), (rates_hz * dt * 1e-3).astype(np.float32))
    W = normal_weights(g, 512, 700)
    lp = layer_params(g, 512, tau_mem=(10.0, 30.0), tau_adapt=(100.0, 300.0),
                      bias=(1.0, 2.0) if driven else None)
    Wr = normal_weights(g, 20, 512)
    labels = g.integers(0, 20, B)
    return Workload("shd_like_700x512x20" + ("_driven" if driven else ""), B, T, dt, 2.0,
                    [700, 512], {"x": x, "labels": labels}, [lp], [W],
                    {"readout_W": Wr, "readout_tau": const(20.0, 20)})


def fine_dt_fit(seed=0, B=64, N=256, T=20000, dt=0.05) -> Workload:
    """N independent ALIF neurons driven by OU current (tau 5 ms, mean 0.8, sd 0.5),
    DT 0.05 ms, ARP 2 ms (40-step blocks), per-neuron tau_m ~ U[10,30],
    tau_a ~ U[100,300], d = 1.8, theta0 = 1."""
    g = rng(seed)
    I = ou_current(g, B, T, N, dt)
    lp = layer_params(g, N, tau_mem=(10.0, 30.0), tau_adapt=(100.0, 300.0))
    # perturbed parameters for the target trains of the fitting loss
    tgt = LayerParams(
        np.maximum(lp.tau_mem * (1 + 0.1 * g.standard_normal(N)), 1e-3).astype(np.float32),
        np.maximum(lp.tau_adapt * (1 + 0.1 * g.standard_normal(N)), 1e-3).astype(np.float32),
        np.maximum(lp.d * (1 + 0.1 * g.standard_normal(N)), 0.0).astype(np.float32),
        np.maximum(lp.theta0 * (1 + 0.05 * g.standard_normal(N)), 1e-3).astype(np.float32))
    return Workload(f"fine_dt_fit_B{B}_N{N}_T{T}_dt{dt}", B, T, dt, 2.0, [0, N], {"I": I},
                    [lp], [], {"target_params": tgt, "sigma_steps": 2.0 / dt})


def three_layer(seed=0, driven=False, B=128, T=2000) -> Workload:
    """700 -> 1024 -> 1024 -> 20 ALIF, Bernoulli 10 Hz input at DT 0.5 ms, ARP 2 ms,
    single-layer parameters, loss = total final-layer spike count."""
    g = rng(seed)
    dt = 0.5
    x = bernoulli_spikes(g, (B, T, 700), 10.0 * dt * 1e-3)
    sizes = [700, 1024, 1024, 20]
    Ws = [normal_weights(g, sizes[i + 1], sizes[i]) for i in range(3)]
    lps = [layer_params(g, sizes[i + 1], bias=(1.0, 2.0) if driven else None) for i in range(3)]
    return Workload("three_layer_700x1024x1024x20" + ("_driven" if driven else ""), B, T, dt,
                    2.0, sizes, {"x": x}, lps, Ws)


def speed_benchmark(seed=0, B=64, T=1024, n_in=200, hidden=(256,), TR=40, driven=True) -> Workload:
    """The speed-benchmark network: a synthetic spike dataset in which each batch
    element b fires at r_b ~ U[0, 200] Hz on every input channel (homogeneous
    Poisson, one step = 1 ms), feeding ALIF layers of the given widths with
    W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), tau_mem 20 ms, tau_adapt 150 ms,
    d 1.8 (supplementary "Speed benchmarks" and "Weight initialisation");
    loss = total last-layer spike count. DT = 1 ms and ARP = T_R ms, so the
    refractory period spans T_R steps. ``driven`` adds a bias b ~ U[1, 2] so that
    every layer fires (with zero bias the deeper layers fall silent)."""
    g = rng(seed)
    rates = g.uniform(0.0, 200.0, B).astype(np.float32)
    x = bernoulli_spikes(g, (B, T, n_in), (rates * 1e-3)[:, None, None])
    sizes = [n_in, *hidden]
    Ws, lps = [], []
    for i in range(len(hidden)):
        lim = 1.0 / np.sqrt(sizes[i])
        Ws.append(g.uniform(-lim, lim, (sizes[i + 1], sizes[i])).astype(np.float32))
        lps.append(layer_params(g, sizes[i + 1], tau_mem=(20.0, 20.0), tau_adapt=(150.0, 150.0),
                                bias=(1.0, 2.0) if driven else None))
    return Workload(f"speed_{n_in}x{'x'.join(map(str, hidden))}_B{B}_T{T}_TR{TR}", B, T, 1.0, float(TR),
                    sizes, {"x": x}, lps, Ws)


def bin_counts(x: np.ndarray, s: int) -> np.ndarray:
    """Sum [B][T][n] uint8 counts over consecutive groups of s steps: the same events
    on a grid s times coarser (T must be a multiple of s)."""
    B, T, n = x.shape
    return x.reshape(B, T // s, s, n).sum(axis=2, dtype=np.uint16).astype(np.uint8)


def dt_sweep_layer(seed=21, B=16, N=256, n_in=200, duration_ms=1000.0, dt_ms=0.025) -> Workload:
    """One ALIF layer with fixed input weights driven by Poisson spikes, for the
    simulation-error-versus-DT trade-off (the problem overview figure, panel b).
    Input channel spikes are drawn on the finest grid (dt_ms; Bernoulli per step
    with p = rate dt, rate per batch element ~ U[20, 80] Hz) and summed into
    coarser bins for every coarser DT, so all DTs see the same events. The
    synaptic current is I[t] = b + sum_j W_ij counts_j[t] / DT (each input spike
    delivers the same charge at every DT); W_ij ~ U[0, 0.26] gives a mean drive
    of about 0.5 to 2 against theta0 = 1. tau_mem ~ U[10, 30] ms, tau_adapt ~
    U[100, 300] ms, d ~ U[0.05, 0.5], bias ~ U[-0.1, 0.1]. ARP 2 ms at every DT."""
    g = rng(seed)
    T = int(round(duration_ms / dt_ms))
    rates = g.uniform(20.0, 80.0, B).astype(np.float32)
    x = bernoulli_spikes(g, (B, T, n_in), (rates * dt_ms * 1e-3)[:, None, None])
    W = g.uniform(0.0, 0.26, (N, n_in)).astype(np.float32)
    lp = LayerParams(uniform(g, 10.0, 30.0, N), uniform(g, 100.0, 300.0, N), uniform(g, 0.05, 0.5, N),
                     const(1.0, N), uniform(g, -0.1, 0.1, N))
    return Workload(f"dt_sweep_{n_in}x{N}_B{B}_{duration_ms:g}ms", B, T, dt_ms, 2.0, [n_in, N], {"x": x},
                    [lp], [W], {"rates_hz": rates})


@dataclass
class FitSetup:
    """Synthetic stand-in for the neural-fit experiments (supplementary "Neural fits"):
    ground-truth ALIF neurons with their own parameters, each injected with
    Ornstein-Uhlenbeck currents at several amplitudes (stimuli; the first half for
    fitting, the second half held out), each stimulus repeated ``repeats`` times
    with independent intrinsic noise (a second, weaker OU current) so that the
    recorded trains vary from repeat to repeat. The ground truth runs at dt_ms and
    ARP 2 ms; models start from the paper's initialisation."""
    N: int
    n_stim: int
    repeats: int
    duration_ms: float
    dt_ms: float
    arp_ms: float
    amplitudes: list          # OU mean of each stimulus (fit stimuli, then held-out ones)
    stim_tau_ms: float
    stim_sd: float
    noise_tau_ms: float
    noise_sd: float
    truth: LayerParams
    init: LayerParams
    seed: int


def neuron_fit(seed=31, N=2048, n_stim=4, repeats=4, duration_ms=2000.0, dt_ms=0.05) -> FitSetup:
    """Ground truth tau_mem ~ U[8, 40] ms, tau_adapt ~ U[50, 400] ms, d ~ U[0.02, 0.4],
    theta0 ~ U[0.8, 1.2], bias ~ U[-0.1, 0.1]; stimuli OU (tau 5 ms, sd 0.5) with
    means 1.0, 1.2, 1.4, 1.6 (then the same means for the held-out set); intrinsic
    noise OU (tau 2 ms, sd 0.05). Initial model: tau_mem 20 ms, tau_adapt 100 ms,
    d 0.1, theta0 1, bias 0 (the supplementary's initial time constants; d and
    theta0 in this model's units)."""
    g = rng(seed)
    truth = LayerParams(uniform(g, 8.0, 40.0, N), uniform(g, 50.0, 400.0, N), uniform(g, 0.02, 0.4, N),
                        uniform(g, 0.8, 1.2, N), uniform(g, -0.1, 0.1, N))
    init = LayerParams(const(20.0, N), const(100.0, N), const(0.1, N), const(1.0, N), const(0.0, N))
    amps = [1.0 + 0.2 * (i % 4) for i in range(n_stim)]
    return FitSetup(N, n_stim, repeats, duration_ms, dt_ms, 2.0, amps + amps, 5.0, 0.5, 2.0, 0.05,
                    truth, init, seed)


@dataclass
class Request:
    """One serving request: a single ALIF layer of N neurons over T steps fed by
    an OU current that the server draws on the device from ``seed``."""
    rid: int
    arrival_s: float
    N: int
    T: int
    dt: float
    arp: float
    seed: int


def request_stream(seed=0, n=2000, rate_hz=200.0, n_range=(64, 2048),
                   t_range=(500, 50000), dts=(1.0, 0.1, 0.05)) -> list:
    """Poisson arrivals at ``rate_hz``; N ~ U{n_range}, T ~ U{t_range}, DT from ``dts``."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_hz, n)
    t = np.cumsum(gaps) - gaps[0]
    Ns = g.integers(n_range[0], n_range[1] + 1, n)
    Ts = g.integers(t_range[0], t_range[1] + 1, n)
    D = g.choice(np.asarray(dts), n)
    seeds = g.integers(1, 2**62, n)
    return [Request(i, float(t[i]), int(Ns[i]), int(Ts[i]), float(D[i]), 2.0, int(seeds[i]))
            for i in range(n)]


# OU current of a serving request (the same process as the fine-DT workload)
REQUEST_OU = dict(tau=5.0, mean=0.8, sd=0.5)


def request_params(req: Request) -> LayerParams:
    """Per-neuron parameters of a serving request, drawn from its seed:
    tau_m ~ U[10, 30] ms, tau_a ~ U[100, 300] ms, d = 1.8, theta0 = 1."""
    g = rng(req.seed % (2**63))
    return layer_params(g, req.N, tau_mem=(10.0, 30.0), tau_adapt=(100.0, 300.0))
