"""Pins for the oracle's recurrent network (Eq. 3 with the recurrent current
W_rec S[t - D], D = T_R), CPU only.

* With W_rec = 0 it is the feedforward oracle.
* A neuron fed only by another neuron's spikes, below its threshold, follows the
  first-order IIR filter of the other's spike train delayed by D (a library
  routine, scipy.signal.lfilter).
* It equals the paper's Blocks formulation with recurrence (Prop. 3: block n + 1
  receives W_rec times the spikes of block n), written separately in
  tests/block_reference.py, on random small networks.
* The weight gradient of the recurrent term against explicit loops.
"""
import math

import numpy as np
import pytest

import oracle
from block_reference import blocks_recurrent


def _params(g, N, d=(0.0, 1.5)):
    return (g.uniform(3.0, 25.0, N), g.uniform(30.0, 200.0, N), g.uniform(*d, N), g.uniform(0.8, 1.2, N))


def test_zero_recurrent_weights_is_feedforward():
    g = np.random.default_rng(1)
    B, T, N = 2, 300, 5
    Iff = g.uniform(0.5, 4.0, (B, T, N))
    tm, ta, d, th0 = _params(g, N, d=(0.0, 0.5))
    r = oracle.alif_forward_recurrent(Iff, np.zeros((N, N)), tm, ta, d, th0, 0.5, 2.0)
    f = oracle.alif_forward(Iff, tm, ta, d, th0, 0.5, 2.0)
    assert f["S"].sum() > 50
    np.testing.assert_array_equal(r["S"], f["S"])
    np.testing.assert_array_equal(r["V"], f["V"])
    np.testing.assert_array_equal(r["TH"], f["TH"])
    np.testing.assert_array_equal(r["Itot"], Iff)


@pytest.mark.parametrize("TR,dt,D", [(2, 1.0, 2), (5, 0.4, 5), (2, 1.0, 7), (5, 0.4, 10)])
def test_driven_by_another_neuron_is_a_delayed_iir_filter(TR, dt, D):
    """Neuron 0 fires periodically on a constant current; neuron 1 has no other
    input and W_rec[1][0] = w < theta0, so it never fires and its membrane is the
    IIR filter (1 - beta) / (1 - beta z^-1) of w S_0[t - D]."""
    from scipy.signal import lfilter
    T, N, w = 400, 2, 0.35
    Iff = np.zeros((1, T, N))
    Iff[0, :, 0] = 2.5
    W_rec = np.array([[0.0, 0.0], [w, 0.0]])
    tm = np.array([10.0, 7.0])
    r = oracle.alif_forward_recurrent(Iff, W_rec, tm, [100.0, 100.0], [0.0, 0.0], [1.0, 1.0], dt, TR * dt, D=D)
    S0 = r["S"][0, :, 0].astype(np.float64)
    assert S0.sum() > 10 and r["S"][0, :, 1].sum() == 0
    drive = np.zeros(T)
    drive[D:] = w * S0[:T - D]
    np.testing.assert_array_equal(r["Itot"][0, :, 1], drive)
    beta = math.exp(-dt / tm[1])
    np.testing.assert_allclose(r["V"][0, :, 1], lfilter([1.0 - beta], [1.0, -beta], drive), rtol=0, atol=1e-13)


@pytest.mark.parametrize("TR,dt", [(2, 1.0), (3, 2.0 / 3.0), (5, 0.4)])
def test_recurrent_equals_blocks_formulation(TR, dt):
    """Random small recurrent networks: the oracle (step by step) and the Blocks
    formulation (Props. 1-5 with Prop. 3's recurrent current) agree spike for
    spike, traces to rounding."""
    g = np.random.default_rng(20 + TR)
    fired = 0
    for trial in range(6):
        N = int(g.integers(2, 6))
        T = int(g.integers(20 * TR, 60 * TR))
        Iff = g.uniform(0.2, 3.0, (1, T, N)) + (g.random((1, T, N)) < 0.05) * 2.0
        W_rec = g.normal(0.0, 0.8, (N, N))
        tm, ta, d, th0 = _params(g, N, d=(0.0, 0.8))
        r = oracle.alif_forward_recurrent(Iff, W_rec, tm, ta, d, th0, dt, TR * dt)
        beta, p = np.exp(-dt / tm), np.exp(-dt / ta)
        S, V, TH = blocks_recurrent(Iff[0], W_rec, beta, p, d, th0, TR)
        np.testing.assert_array_equal(S, r["S"][0])
        np.testing.assert_allclose(V, r["V"][0], rtol=0, atol=1e-11)
        np.testing.assert_allclose(TH, r["TH"][0], rtol=0, atol=1e-11)
        fired += int(S.sum())
        # the feedforward record the backward differentiates is the same run
        np.testing.assert_array_equal(r["ff"]["S"], r["S"])
        np.testing.assert_allclose(r["ff"]["V"], r["V"], rtol=0, atol=0)
    assert fired > 30


def test_recurrent_weight_grad_brute_force():
    g = np.random.default_rng(5)
    B, T, N, D = 2, 9, 3, 2
    gI = g.standard_normal((B, T, N))
    S = (g.random((B, T, N)) < 0.4).astype(np.uint8)
    ref = np.zeros((N, N))
    for b in range(B):
        for t in range(D, T):
            for i in range(N):
                for j in range(N):
                    ref[i, j] += gI[b, t, i] * S[b, t - D, j]
    np.testing.assert_allclose(oracle.recurrent_weight_grad(gI, S, D), ref, rtol=0, atol=1e-12)
