"""Test-only CPU transcription of the paper's Block / Blocks model (Section 3).

It follows the propositions in the paper's own order and notation, in float64,
one neuron at a time, so that the oracle (the standard model, Eqs. 1-5) can be
pinned against a second, structurally different statement of the same dynamics:

  Block (Eqs. 6-9):  V~ = I * beta~ (Prop. 1, initial potential folded in as
                     I[0] = V[0] / (1 - beta)),  S~ = f(V~),  z = phi(S~),
                     S = 1[z == 1]  (Prop. 2)
  Blocks:            input of block n+1 masked by 1[z_n[t] >= max_t S_n[t]]
                     (Prop. 3); V_{n+1}[0] = V_n[T_R] or 0 (Prop. 4);
                     theta_{n+1}[t] = theta0 + d p^t a_{n+1}[0] with
                     a_{n+1}[0] = a_n[T_R] or p^m (a_s + 1/p) (Prop. 5).

The paper's threshold baseline is the constant 1; ``theta0`` generalises it.
Traces after the block's spike (reset membrane, bumped adaptation) are not
defined by the propositions; they follow from Eqs. 2 and 5 and are returned so
that traces can be compared as well.
"""
from __future__ import annotations

import numpy as np


def phi(s_tilde: np.ndarray) -> np.ndarray:
    """Prop. 2: phi(S~)[t] = sum_{k<=t} S~[k] (t - k + 1) (1-based t, k)."""
    L = len(s_tilde)
    out = np.zeros(L, dtype=np.int64)
    for t in range(1, L + 1):
        out[t - 1] = sum(int(s_tilde[k - 1]) * (t - k + 1) for k in range(1, t + 1))
    return out


def block(I_blk, V0, a0, beta, p, d, theta0):
    """One Block of length T_R = len(I_blk) (Eqs. 6-9 with Props. 1 and 5)."""
    TR = len(I_blk)
    # Prop. 1: convolution with kernel (1 - beta) beta^t, I[0] = V0 / (1 - beta)
    I_ext = np.concatenate([[V0 / (1.0 - beta)], I_blk])
    kern = (1.0 - beta) * beta ** np.arange(TR + 1)
    V_t = np.array([sum(kern[t - j] * I_ext[j] for j in range(t + 1)) for t in range(1, TR + 1)])
    # Prop. 5: theta[t] = theta0 + d p^t a[0]
    a_t = p ** np.arange(1, TR + 1) * a0
    th = theta0 + d * a_t
    s_tilde = (V_t > th).astype(np.int64)          # Eq. 7
    z = phi(s_tilde)                               # Eq. 8
    S = (z == 1).astype(np.int64)                  # Eq. 9
    return V_t, th, a_t, z, S


class _Chain:
    """One neuron's state between Blocks: V0 and a0 (Props. 4-5) and the latent
    spike timing z and spikes S of the previous block (for Prop. 3's mask)."""

    def __init__(self):
        self.V0, self.a0, self.z_prev, self.S_prev = 0.0, 0.0, None, None

    def step(self, I_blk, beta, p, d, theta0):
        """Block n + 1 of this neuron on its (unmasked) input current I_blk."""
        TR = len(I_blk)
        if self.z_prev is None:
            mask = np.ones(TR)
        else:
            mask = (self.z_prev >= self.S_prev.max()).astype(np.float64)    # Prop. 3
        V_t, th, a_t, z, S = block(I_blk * mask, self.V0, self.a0, beta, p, d, theta0)
        V = V_t.copy()
        TH = th.copy()
        if S.max() > 0:
            ts = int(np.argmax(S))                  # 0-based index of the spike
            a_s = float((a_t * S).sum())
            V[ts + 1:] = 0.0                        # reset (Eq. 2), refractory (Eq. 4)
            k = np.arange(ts + 1, TR)
            TH[ts + 1:] = theta0 + d * (p ** (k - ts - 1) * (p * a_s + 1.0))   # Eq. 5
            m = int((z > 1).sum())
            self.V0 = 0.0                           # Prop. 4
            self.a0 = p ** m * (a_s + 1.0 / p)      # Prop. 5
        else:
            self.V0 = V_t[-1]                       # Prop. 4
            self.a0 = a_t[-1]                       # Prop. 5 (a_n[T_R])
        self.z_prev, self.S_prev = z, S
        return S, V, TH


def blocks(I, beta, p, d, theta0, TR):
    """Chain ceil(T / T_R) Blocks (Props. 3-5) over one neuron's current I[T].

    Returns S, V, TH (corrected traces, truncated to T)."""
    T = len(I)
    NB = -(-T // TR)
    Ipad = np.zeros(NB * TR)
    Ipad[:T] = I                                   # zero padding (footnote to "Blocks")
    ch = _Chain()
    S_all, V_all, TH_all = [], [], []
    for n in range(NB):
        S, V, TH = ch.step(Ipad[n * TR:(n + 1) * TR], beta, p, d, theta0)
        S_all.append(S)
        V_all.append(V)
        TH_all.append(TH)
    S = np.concatenate(S_all)[:T]
    V = np.concatenate(V_all)[:T]
    TH = np.concatenate(TH_all)[:T]
    return S.astype(np.uint8), V, TH


def blocks_recurrent(I_ff, W_rec, beta, p, d, theta0, TR):
    """The recurrent network as Blocks: Prop. 3's input current of block n + 1 is
    the bias and feedforward current plus sum_j W_rec[i][j] S_{j,n}[t], the
    spikes of every neuron in block n at the same position t of the block (the
    recurrent delay equals the block length). I_ff [T][N]; per-neuron beta, p, d,
    theta0 [N]. Returns S, V, TH [T][N]."""
    T, N = I_ff.shape
    NB = -(-T // TR)
    Ipad = np.zeros((NB * TR, N))
    Ipad[:T] = I_ff
    chains = [_Chain() for _ in range(N)]
    S_out = np.zeros((NB * TR, N), np.uint8)
    V_out = np.zeros((NB * TR, N))
    TH_out = np.zeros((NB * TR, N))
    S_prev_blk = np.zeros((TR, N))
    for n in range(NB):
        sl = slice(n * TR, (n + 1) * TR)
        I_blk = Ipad[sl] + S_prev_blk @ np.asarray(W_rec, np.float64).T
        for i in range(N):
            S, V, TH = chains[i].step(I_blk[:, i], beta[i], p[i], d[i], theta0[i])
            S_out[sl, i] = S
            V_out[sl, i] = V
            TH_out[sl, i] = TH
        S_prev_blk = S_out[sl].astype(np.float64)
    return S_out[:T], V_out[:T], TH_out[:T]
