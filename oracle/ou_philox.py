"""Counter-based Ornstein-Uhlenbeck input current -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module. It is the oracle side's own implementation
of the generator the library uses to draw a request's input current on the
device, written from the published definitions, so that a test can rebuild that
current on the host without reading it back from the GPU path:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC 2011): a 4-word counter and a 2-word key; each of the ten
  rounds multiplies counter words 0 and 2 by two fixed 32-bit constants, takes
  the high and low halves of the 64-bit products, swaps and xors them with the
  other two words and the round key; the key grows by two Weyl constants
  between rounds.
* Box-Muller: two uniforms (u1 in (0, 1], u2 in [0, 1)) give the independent
  standard normals r cos(2 pi u2) and r sin(2 pi u2), r = sqrt(-2 ln u1).
* OU: the exact discretisation of dX = -X / tau dt + sd sqrt(2 / tau) dW, whose
  stationary law is N(0, sd^2): X[0] = sd z_0, X[t] = e X[t-1] + sd sqrt(1 - e^2) z_t,
  e = exp(-dt / tau); the current is mean + X rounded to float32.

Stream layout: neuron n, step t uses counter (t // 4, n, 0, 0) under key
(seed low word, seed high word); output words (w0, w1) give steps 4q (cos) and
4q + 1 (sin), (w2, w3) give 4q + 2 (cos) and 4q + 3 (sin), u1 = (w_even + 1) / 2^32,
u2 = w_odd / 2^32, all in FP64.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
PHILOX_M = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
PHILOX_W = (np.uint64(0x9E3779B9), np.uint64(0xBB67AE85))


def philox4x32_10(ctr, key):
    """ctr: 4 uint32-valued arrays (broadcastable), key: 2 uint32 values.
    Returns the 4 output words as uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0, k1 = (np.uint64(int(k) & 0xFFFFFFFF) for k in key)
    for _ in range(10):
        p0 = PHILOX_M[0] * c0          # < 2^64: exact in uint64
        p1 = PHILOX_M[1] * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W[0]) & MASK32
        k1 = (k1 + PHILOX_W[1]) & MASK32
    return c0, c1, c2, c3


def standard_normals(T: int, N: int, seed: int) -> np.ndarray:
    """z[t, n], FP64 [T][N], from the stream layout in the module docstring."""
    seed = int(seed) & (2**64 - 1)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    Q = (T + 3) // 4
    q = np.arange(Q, dtype=np.uint64)[:, None]
    n = np.arange(N, dtype=np.uint64)[None, :]
    zero = np.zeros((1, 1), dtype=np.uint64)
    w0, w1, w2, w3 = philox4x32_10((q, n, zero, zero), key)
    w0, w1, w2, w3 = (np.broadcast_to(w, (Q, N)) for w in (w0, w1, w2, w3))
    z = np.empty((Q, 4, N), dtype=np.float64)
    for j, (we, wo) in enumerate(((w0, w1), (w2, w3))):
        u1 = (we.astype(np.float64) + 1.0) / 4294967296.0
        u2 = wo.astype(np.float64) / 4294967296.0
        r = np.sqrt(-2.0 * np.log(u1))
        z[:, 2 * j] = r * np.cos(2.0 * np.pi * u2)
        z[:, 2 * j + 1] = r * np.sin(2.0 * np.pi * u2)
    return z.reshape(Q * 4, N)[:T]


def ou_current(T: int, N: int, dt: float, tau: float, mean: float, sd: float, seed: int):
    """float32 [T][N] OU current (FP64 recurrence, one rounding at the end), and
    the FP64 values before rounding."""
    tau, mean, sd = float(np.float32(tau)), float(np.float32(mean)), float(np.float32(sd))
    z = standard_normals(T, N, seed)
    e = np.exp(-dt / tau)
    s = sd * np.sqrt(1.0 - e * e)
    x = np.empty((T, N), dtype=np.float64)
    for t in range(T):
        x[t] = sd * z[0] if t == 0 else e * x[t - 1] + s * z[t]
    i64 = mean + x
    return i64.astype(np.float32), i64
