"""FP64 CPU oracle for block-wise ALIF -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it; the two
share no code. Every function here computes the plain standard ALIF model of the
paper (Section 2, Equations 1-5) step by step in double precision, or a plain
definition the paper states (readout, losses), so that it can be checked by eye.

Layout conventions of the wrapper: arrays handed in by callers use the same
``[B][T][N]`` (batch, step, neuron) layout as the GPU library; the C core works
on independent rows ``[R][T]`` (one row per (batch, neuron) pair) and the
wrapper transposes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alif_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i8p = ctypes.POINTER(ctypes.c_int8)
_i64 = ctypes.c_int64


def build() -> str:
    """Compile the C oracle with gcc (IEEE double, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
           "-fPIC", "-Wall", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_refractory_steps.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_refractory_steps.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_input_current.argtypes = [_i64, _i64, _i64, _u8p, _f64p, _f64p, _f64p]
    lib.oracle_alif_forward.argtypes = [_i64, _i64, _f64p, _f64p, _f64p, _f64p, _f64p,
                                        ctypes.c_double, ctypes.c_int, _i8p,
                                        _u8p, _f64p, _f64p, _f64p, _u8p]
    lib.oracle_alif_backward.argtypes = [_i64, _i64, _f64p, _f64p, _f64p, _f64p, _f64p,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                         _u8p, _f64p, _f64p, _f64p, _u8p,
                                         _f64p, _f64p, _f64p,
                                         _f64p, _f64p, _f64p, _f64p, _f64p]
    lib.oracle_alif_forward_recurrent.argtypes = [_i64, _i64, _i64, _f64p, _f64p, _f64p, _f64p, _f64p,
                                                  _f64p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                  _i8p, _u8p, _f64p, _f64p, _f64p, _u8p, _f64p]
    lib.oracle_surrogate.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.oracle_surrogate.restype = ctypes.c_double
    lib.oracle_readout_forward.argtypes = [_i64, _i64, _f64p, _f64p, ctypes.c_double,
                                           _f64p, _f64p]
    lib.oracle_readout_backward.argtypes = [_i64, _i64, _f64p, _f64p, ctypes.c_double,
                                            _f64p, _f64p, _f64p]
    _lib = lib
    return lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def refractory_steps(dt_ms: float, arp_ms: float) -> int:
    """T_R = ARP/DT as a whole number of steps, or -1 if it is not one."""
    return int(_load().oracle_refractory_steps(float(dt_ms), float(arp_ms)))


def input_current(x: np.ndarray, W: np.ndarray, bias=None) -> np.ndarray:
    """Eq. 3 feedforward current b + W x for binary spikes x[..., n_in] -> [..., n]."""
    x = np.ascontiguousarray(x, dtype=np.uint8)
    W = _c64(W)
    lead = x.shape[:-1]
    M = int(np.prod(lead)) if lead else 1
    n, n_in = W.shape
    out = np.empty((M, n), dtype=np.float64)
    b = None if bias is None else _c64(bias)
    _load().oracle_input_current(M, n, n_in, _p(x, ctypes.c_uint8), _p(W, ctypes.c_double),
                                 _p(b, ctypes.c_double), _p(out, ctypes.c_double))
    return out.reshape(*lead, n)


def input_current_values(x: np.ndarray, W: np.ndarray, bias=None) -> np.ndarray:
    """Eq. 3's projection b + W x with real-valued inputs x[..., n_in] in place of binary
    spikes (spike counts per step, or graded values): one FP64 matrix product. For 0/1
    inputs it is the spike sum of input_current."""
    out = np.asarray(x, dtype=np.float64) @ _c64(W).T
    if bias is not None:
        out = out + _c64(bias)
    return out


def weight_grad(gI: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gradient with respect to W of the Eq. 3 projection I = b + W x, given the
    current gradient gI[..., n]: dL/dW[n][i] = sum over (b, t) of gI[n] x[i]
    (one FP64 matrix product; x may be spikes or any real input)."""
    gI = np.asarray(gI, np.float64)
    x = np.asarray(x, np.float64)
    return gI.reshape(-1, gI.shape[-1]).T @ x.reshape(-1, x.shape[-1])


def input_grad(gI: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Gradient with respect to the input x of the Eq. 3 projection I = b + W x:
    dL/dx[..., i] = sum over n of gI[..., n] W[n][i] (one FP64 matrix product)."""
    return np.asarray(gI, np.float64) @ np.asarray(W, np.float64)


def forward_rows(I, tau_m, tau_a, d, theta0, dt, TR, force=None):
    """Standard ALIF (Eqs. 1-5) on independent rows I[R][T]; params are [R].

    Returns dict with S (uint8), V, TH, A (float64) and MASK (uint8), all [R][T].
    ``force`` [R][T] int8 (-1 free, 0/1 imposed) re-runs on given decisions.
    """
    I = _c64(I)
    R, T = I.shape
    pr = [_c64(np.broadcast_to(q, (R,))) for q in (tau_m, tau_a, d, theta0)]
    S = np.empty((R, T), np.uint8)
    V = np.empty((R, T))
    TH = np.empty((R, T))
    A = np.empty((R, T))
    M = np.empty((R, T), np.uint8)
    f = None if force is None else np.ascontiguousarray(force, dtype=np.int8)
    _load().oracle_alif_forward(R, T, _p(I, ctypes.c_double), *[_p(q, ctypes.c_double) for q in pr],
                                float(dt), int(TR), _p(f, ctypes.c_int8),
                                _p(S, ctypes.c_uint8), _p(V, ctypes.c_double),
                                _p(TH, ctypes.c_double), _p(A, ctypes.c_double),
                                _p(M, ctypes.c_uint8))
    return {"S": S, "V": V, "TH": TH, "A": A, "MASK": M, "I": I}


# surrogate kinds (supplementary "Surrogate gradient"); the library's enum uses the same numbers
SURROGATES = {"fast_sigmoid": 0, "boxcar": 1, "multi_gaussian": 2}


def _sg_kind(surrogate) -> int:
    return SURROGATES[surrogate] if isinstance(surrogate, str) else int(surrogate)


def surrogate(kind, u: float, slope: float = 10.0) -> float:
    """Surrogate derivative dS/du at u = V - th: fast sigmoid (slope |u| + 1)^-2,
    boxcar 0.5 on |u| <= 0.5, or the multi-Gaussian mixture as printed."""
    return float(_load().oracle_surrogate(_sg_kind(kind), float(u), float(slope)))


def backward_rows(fw, tau_m, tau_a, d, theta0, dt, slope=10.0, gS=None, gV=None, gTH=None,
                  want_gI=True, surrogate="fast_sigmoid", attached=False):
    """Sequential surrogate-gradient adjoint of ``forward_rows`` under the detached
    policy, or with ``attached`` the spike's own effect through reset and adaptation
    (supplementary "Detaching gradients").

    Returns dict with gI [R][T] (or None) and g_tau_m, g_tau_a, g_d, g_theta0 [R].
    """
    I = fw["I"]
    R, T = I.shape
    pr = [_c64(np.broadcast_to(q, (R,))) for q in (tau_m, tau_a, d, theta0)]
    gS = None if gS is None else _c64(gS)
    gV = None if gV is None else _c64(gV)
    gTH = None if gTH is None else _c64(gTH)
    gI = np.empty((R, T)) if want_gI else None
    outs = [np.empty(R) for _ in range(4)]
    _load().oracle_alif_backward(R, T, _p(I, ctypes.c_double), *[_p(q, ctypes.c_double) for q in pr],
                                 float(dt), _sg_kind(surrogate), float(slope), int(bool(attached)),
                                 _p(fw["S"], ctypes.c_uint8), _p(fw["V"], ctypes.c_double),
                                 _p(fw["TH"], ctypes.c_double), _p(fw["A"], ctypes.c_double),
                                 _p(fw["MASK"], ctypes.c_uint8),
                                 _p(gS, ctypes.c_double), _p(gV, ctypes.c_double),
                                 _p(gTH, ctypes.c_double), _p(gI, ctypes.c_double),
                                 *[_p(q, ctypes.c_double) for q in outs])
    return {"gI": gI, "g_tau_m": outs[0], "g_tau_a": outs[1], "g_d": outs[2],
            "g_theta0": outs[3]}


# ---------------------------------------------------------------------------
# [B][T][N] convenience layer (the GPU library's layout)
# ---------------------------------------------------------------------------

def _to_rows(x):
    B, T, N = x.shape
    return np.ascontiguousarray(np.transpose(x, (0, 2, 1))).reshape(B * N, T)


def _from_rows(r, B, N):
    T = r.shape[1]
    return np.ascontiguousarray(np.transpose(r.reshape(B, N, T), (0, 2, 1)))


def _row_params(q, B, N):
    q = np.broadcast_to(np.asarray(q, dtype=np.float64), (N,))
    return np.tile(q, B)


def alif_forward(I, tau_m, tau_a, d, theta0, dt, arp, force=None):
    """Standard ALIF on current I[B][T][N] (float32 or float64, upcast exactly).

    Returns S, V, TH, A, MASK in [B][T][N] plus the row-form record ``rows``
    used by ``alif_backward``.
    """
    I = np.asarray(I)
    B, T, N = I.shape
    TR = refractory_steps(dt, arp)
    if TR < 1:
        raise ValueError("ARP/DT is not a whole number of steps")
    prm = [_row_params(q, B, N) for q in (tau_m, tau_a, d, theta0)]
    f = None if force is None else _to_rows(np.asarray(force, np.int8))
    fw = forward_rows(_to_rows(I.astype(np.float64)), *prm, dt, TR, force=f)
    out = {k: _from_rows(v, B, N) for k, v in fw.items() if k != "I"}
    out["rows"] = fw
    out["TR"] = TR
    out["params"] = prm
    return out


def alif_forward_recurrent(Iff, W_rec, tau_m, tau_a, d, theta0, dt, arp, force=None, D=None):
    """The recurrent network (Eq. 3 with W_rec S[t - D], D = T_R unless given) on
    Iff [B][T][N] = bias + feedforward current. Returns S, V, TH, A, MASK and
    Itot (the whole current) in [B][T][N], plus ``ff``: the row-wise forward of
    the same neurons driven by Itot with the recurrent run's decisions imposed,
    which is what ``alif_backward`` differentiates (under the detached policy the
    recurrent input is a constant of the spike path)."""
    Iff = np.ascontiguousarray(Iff, np.float64)
    B, T, N = Iff.shape
    TR = refractory_steps(dt, arp)
    if TR < 1:
        raise ValueError("ARP is not a whole number of steps")
    D = TR if D is None else int(D)
    W_rec = _c64(W_rec)
    prm = [_c64(np.broadcast_to(np.asarray(q, np.float64), (N,))) for q in (tau_m, tau_a, d, theta0)]
    fc = None if force is None else np.ascontiguousarray(force, np.int8)
    S = np.empty((B, T, N), np.uint8)
    M = np.empty((B, T, N), np.uint8)
    V, TH, A, It = (np.empty((B, T, N)) for _ in range(4))
    _load().oracle_alif_forward_recurrent(B, T, N, _p(Iff, ctypes.c_double), _p(W_rec, ctypes.c_double),
                                          *[_p(q, ctypes.c_double) for q in prm], float(dt), TR, D,
                                          _p(fc, ctypes.c_int8), _p(S, ctypes.c_uint8), _p(V, ctypes.c_double),
                                          _p(TH, ctypes.c_double), _p(A, ctypes.c_double),
                                          _p(M, ctypes.c_uint8), _p(It, ctypes.c_double))
    ff = alif_forward(It, prm[0], prm[1], prm[2], prm[3], dt, arp, force=S.astype(np.int8))
    return {"S": S, "V": V, "TH": TH, "A": A, "MASK": M, "Itot": It, "ff": ff}


def recurrent_weight_grad(gI, S, D):
    """Gradient with respect to W_rec of the recurrent term of Eq. 3, with the
    spikes held constant (detached policy): dL/dW_rec[i][j] = sum over (b, t) of
    gI[b][t][i] S[b][t - D][j] (one FP64 matrix product over the shifted spikes)."""
    gI = np.asarray(gI, np.float64)
    S = np.asarray(S, np.float64)
    Ssh = np.zeros_like(S)
    Ssh[:, D:, :] = S[:, :S.shape[1] - D, :]
    return gI.reshape(-1, gI.shape[-1]).T @ Ssh.reshape(-1, S.shape[-1])


def alif_backward(fwd, dt, slope=10.0, gS=None, gV=None, gTH=None, want_gI=True,
                  surrogate="fast_sigmoid", attached=False):
    """Adjoint for ``alif_forward`` output; gradients summed over the batch.

    gS, gV, gTH are [B][T][N] (or None). Returns gI [B][T][N] (or None) and
    per-neuron g_tau_m, g_tau_a, g_d, g_theta0 [N] plus their per-row values.
    """
    B, T, N = fwd["S"].shape
    conv = lambda g: None if g is None else _to_rows(np.asarray(g, np.float64))
    bw = backward_rows(fwd["rows"], *fwd["params"], dt, slope, conv(gS), conv(gV), conv(gTH),
                       want_gI=want_gI, surrogate=surrogate, attached=attached)
    out = {"gI": None if bw["gI"] is None else _from_rows(bw["gI"], B, N)}
    for k in ("g_tau_m", "g_tau_a", "g_d", "g_theta0"):
        out[k] = bw[k].reshape(B, N).sum(axis=0)
        out[k + "_rows"] = bw[k].reshape(B, N)
    return out


def readout_forward(Ir, tau_r, dt):
    """Leaky readout, o[b][c] = sum_t Vr[b][t][c]; Ir is [B][T][C]."""
    Ir = np.asarray(Ir, np.float64)
    B, T, C = Ir.shape
    rows = _to_rows(Ir)
    tr = _row_params(tau_r, B, C)
    Vr = np.empty_like(rows)
    o = np.empty(B * C)
    _load().oracle_readout_forward(B * C, T, _p(rows, ctypes.c_double), _p(tr, ctypes.c_double),
                                   float(dt), _p(Vr, ctypes.c_double), _p(o, ctypes.c_double))
    return {"o": o.reshape(B, C), "Vr": _from_rows(Vr, B, C)}


def readout_backward(Ir, tau_r, dt, go):
    """Adjoint of ``readout_forward`` for upstream gradient go[B][C]."""
    Ir = np.asarray(Ir, np.float64)
    B, T, C = Ir.shape
    rows = _to_rows(Ir)
    tr = _row_params(tau_r, B, C)
    g = _c64(np.asarray(go, np.float64).reshape(B * C))
    gIr = np.empty_like(rows)
    gt = np.empty(B * C)
    _load().oracle_readout_backward(B * C, T, _p(rows, ctypes.c_double), _p(tr, ctypes.c_double),
                                    float(dt), _p(g, ctypes.c_double), _p(gIr, ctypes.c_double),
                                    _p(gt, ctypes.c_double))
    return {"gIr": _from_rows(gIr, B, C), "g_tau_r": gt.reshape(B, C).sum(axis=0)}


# ---------------------------------------------------------------------------
# Losses the configurations use (plain definitions, float64)
# ---------------------------------------------------------------------------

def softmax_cross_entropy(o, labels):
    """Supplementary "Supervised training loss": mean over the batch of -log softmax.

    Returns (loss, d loss / d o)."""
    o = np.asarray(o, np.float64)
    B = o.shape[0]
    z = o - o.max(axis=1, keepdims=True)
    e = np.exp(z)
    prob = e / e.sum(axis=1, keepdims=True)
    loss = -np.log(prob[np.arange(B), labels]).mean()
    g = prob.copy()
    g[np.arange(B), labels] -= 1.0
    return loss, g / B


def gaussian_kernel(sigma_steps: float, truncate: float = 4.0) -> np.ndarray:
    """Discrete Gaussian, +-truncate*sigma taps, normalised to unit sum."""
    h = int(np.ceil(truncate * sigma_steps))
    k = np.arange(-h, h + 1, dtype=np.float64)
    g = np.exp(-0.5 * (k / sigma_steps) ** 2)
    return g / g.sum()


def smooth_time(x, kernel):
    """'same' convolution with zero padding along axis 1 of [B][T][N]."""
    x = np.asarray(x, np.float64)
    B, T, N = x.shape
    out = np.empty_like(x)
    for b in range(B):
        for n in range(N):
            out[b, :, n] = np.convolve(x[b, :, n], kernel, mode="same")
    return out


def smoothed_mse(S, S_target, kernel):
    """Mean squared error between Gaussian-smoothed spike trains; returns (loss, dL/dS).

    The kernel is symmetric, so the adjoint of the 'same' convolution is the
    same convolution."""
    a = smooth_time(S, kernel)
    b = smooth_time(S_target, kernel)
    diff = a - b
    M = diff.size
    loss = float((diff ** 2).sum() / M)
    g = smooth_time(2.0 * diff / M, kernel[::-1].copy())
    return loss, g


# ---------------------------------------------------------------------------
# Neural-fit loss and optimiser (supplementary "Neural fits")
# ---------------------------------------------------------------------------

def van_rossum(x, y, dt, tau, scale=1.0):
    """Van Rossum distance of supplementary "Supervised training loss" and its gradient.

    D = sqrt((1/tau) * integral over [0, T] of (k*x - k*y)^2), k(t) = H(t) exp(-t/tau),
    put on the simulation grid: a spike (or count) at step s is an impulse of unit
    area at step s, so (k*x)[t] = sum_{s <= t} exp(-(t - s) dt / tau) x[s] (H(0) = 1),
    and the integral is dt times the sum over the T simulated steps.

    x: model spike trains [B][T][N]; y: targets [B][T][N] or [B][R][T][N] (R repeats
    compared with the same model train). Returns (D [B][R][N],
    grad [B][T][N] = scale * sum_r dD[b][r][n] / dx[b][t][n]); where D = 0 the
    gradient of that term is taken as 0 (the square root's subgradient).
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if y.ndim == 3:
        y = y[:, None]
    B, T, N = x.shape
    R = y.shape[1]
    a = np.exp(-dt / tau)
    e = np.zeros((B, R, T, N))              # k*x - k*y
    run = np.zeros((B, R, N))
    for t in range(T):
        run = a * run + (x[:, None, t, :] - y[:, :, t, :])
        e[:, :, t, :] = run
    D = np.sqrt(dt / tau * (e ** 2).sum(axis=2))
    # dD/dx[s] = (dt / (tau D)) * sum_{t >= s} exp(-(t - s) dt / tau) e[t]
    w = np.where(D > 0, dt / (tau * np.where(D > 0, D, 1.0)), 0.0)
    grad = np.zeros((B, T, N))
    run = np.zeros((B, R, N))
    for t in range(T - 1, -1, -1):
        run = a * run + e[:, :, t, :]
        grad[:, t, :] = (w * run).sum(axis=1)
    return D, scale * grad


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=-np.inf, hi=np.inf):
    """One Adam update (Kingma and Ba, Algorithm 1; the optimiser the neural fits use),
    followed by a projection of the parameter onto [lo, hi] (the paper leaves how the
    parameters are kept valid open). ``step`` counts from 1. Returns (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return np.clip(p, lo, hi), m, v
