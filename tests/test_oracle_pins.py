"""Pins for the FP64 oracle's forward pass (CPU only).

Each test ties the oracle to something other than itself: a closed form of
the recurrence, a library routine it reduces to, an invariant the paper states,
or the paper's second formulation of the same dynamics (the Block propositions).
"""
import math

import numpy as np
import pytest

import oracle
from block_reference import blocks, phi


def _run(I, tau_m=20.0, tau_a=200.0, d=1.8, theta0=1.0, dt=1.0, TR=2, force=None):
    I = np.atleast_2d(np.asarray(I, np.float64))
    R = I.shape[0]
    f = oracle.forward_rows(I, np.full(R, tau_m), np.full(R, tau_a), np.full(R, d),
                            np.full(R, theta0), dt, TR, force=force)
    return f


def test_refractory_steps():
    assert oracle.refractory_steps(0.05, 2.0) == 40
    assert oracle.refractory_steps(1.0, 2.0) == 2
    assert oracle.refractory_steps(0.5, 2.0) == 4
    assert oracle.refractory_steps(0.1, 2.0) == 20
    assert oracle.refractory_steps(0.3, 2.0) == -1
    assert oracle.refractory_steps(0.0, 2.0) == -1


@pytest.mark.parametrize("c", [0.3, 0.7, 0.999])
def test_charging_curve_closed_form(c):
    """Constant sub-threshold drive: V[t] = c (1 - beta^t) (unrolled Eq. 2,
    supplementary proof of Prop. 1, step 1); no spike and a == 0."""
    dt, tau = 1.0, 20.0
    beta = math.exp(-dt / tau)
    T = 400
    f = _run(np.full(T, c), tau_m=tau, dt=dt)
    t = np.arange(1, T + 1)
    np.testing.assert_allclose(f["V"][0], c * (1 - beta ** t), rtol=0, atol=1e-14)
    assert f["S"].sum() == 0
    assert np.all(f["A"] == 0) and np.all(f["TH"] == 1.0)


def test_subthreshold_equals_iir_filter():
    """No spike => the membrane is the first-order IIR filter (1-beta)/(1 - beta z^-1)."""
    from scipy.signal import lfilter
    g = np.random.default_rng(1)
    for tau, dt in [(20.0, 1.0), (13.0, 0.05), (30.0, 0.5)]:
        beta = math.exp(-dt / tau)
        I = g.uniform(-1.0, 1.0, 3000)          # max I <= theta0 = 1 -> never fires
        f = _run(I, tau_m=tau, dt=dt, TR=7)
        ref = lfilter([1 - beta], [1, -beta], I)
        assert f["S"].sum() == 0
        np.testing.assert_allclose(f["V"][0], ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("c,tau,dt", [(1.3, 20.0, 1.0), (2.0, 20.0, 1.0), (1.05, 10.0, 0.05),
                                      (1.7, 30.0, 0.1), (5.0, 20.0, 1.0)])
def test_time_to_first_spike(c, tau, dt):
    """Constant drive c > theta0: first spike at t* = floor(ln(1 - theta0/c) / ln beta) + 1."""
    beta = math.exp(-dt / tau)
    x = math.log(1 - 1.0 / c) / math.log(beta)
    assert abs(x - round(x)) > 1e-6            # keep away from exact ties
    t_star = math.floor(x) + 1
    f = _run(np.full(t_star + 50, c), tau_m=tau, dt=dt, TR=2)
    first = int(np.argmax(f["S"][0])) + 1
    assert f["S"][0].any() and first == t_star


@pytest.mark.parametrize("TR", [2, 3, 7, 40])
def test_periodic_firing_isi(TR):
    """d = 0, constant drive: spikes at t*, then every T_R - 1 + t* steps (Eq. 4 gate
    reopens T_R steps after the spike, charging restarts from V = 0)."""
    c, tau, dt = 1.4, 20.0, 1.0
    beta = math.exp(-dt / tau)
    t_star = math.floor(math.log(1 - 1.0 / c) / math.log(beta)) + 1
    T = 2000
    f = _run(np.full(T, c), tau_m=tau, dt=dt, d=0.0, TR=TR)
    times = np.flatnonzero(f["S"][0]) + 1
    assert times[0] == t_star
    assert np.all(np.diff(times) == TR - 1 + t_star)


def test_adaptation_unrolled():
    """Eq. 5 unrolled: a[t] = sum_{k<t} p^(t-1-k) S[k], theta = theta0 + d a."""
    g = np.random.default_rng(2)
    dt, tau_a, d = 1.0, 150.0, 0.6
    p = math.exp(-dt / tau_a)
    I = g.uniform(2.0, 9.0, 1500)
    f = _run(I, tau_a=tau_a, d=d, dt=dt, TR=3)
    S = f["S"][0].astype(np.float64)
    assert S.sum() > 20
    T = len(S)
    a_ref = np.array([sum(p ** (t - 1 - k) * S[k - 1] for k in range(1, t)) for t in range(1, T + 1)])
    np.testing.assert_allclose(f["A"][0], a_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f["TH"][0], 1.0 + d * a_ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("TR", [2, 4, 20, 40])
def test_invariants_random_drive(TR):
    """At most one spike per window of T_R steps (ISI >= T_R), the gate closed and
    V == 0 for the T_R - 1 steps after a spike, membrane inside the input hull."""
    g = np.random.default_rng(3 + TR)
    R, T = 16, 4000
    I = g.uniform(-0.5, 6.0, (R, T))
    f = _run(I, tau_m=5.0, tau_a=100.0, d=0.2, dt=0.1, TR=TR)
    assert f["S"].sum() > 50
    for r in range(R):
        times = np.flatnonzero(f["S"][r])
        assert np.all(np.diff(times) >= TR)
        for ts in times:
            blank = slice(ts + 1, min(T, ts + TR))
            assert np.all(f["V"][r, blank] == 0.0)
            assert np.all(f["MASK"][r, blank] == 0)
        # per aligned block [n T_R, (n+1) T_R): at most one spike (Prop. 2's premise)
        nb = T // TR
        per_block = f["S"][r, :nb * TR].reshape(nb, TR).sum(axis=1)
        assert per_block.max() <= 1
        assert f["V"][r].min() >= min(0.0, I[r].min()) - 1e-12
        assert f["V"][r].max() <= max(0.0, I[r].max()) + 1e-12


def test_no_spike_when_input_below_threshold():
    g = np.random.default_rng(4)
    I = g.uniform(-3.0, 1.0, (8, 5000))     # max I <= theta0
    f = _run(I, TR=5)
    assert f["S"].sum() == 0


def test_force_imposes_decisions():
    g = np.random.default_rng(5)
    I = g.uniform(0.0, 3.0, (2, 300))
    f = _run(I, TR=2)
    force = np.full(I.shape, -1, np.int8)
    t0 = int(np.flatnonzero(f["S"][0])[0])
    force[0, t0] = 0
    h = _run(I, TR=2, force=force)
    assert h["S"][0, t0] == 0
    np.testing.assert_array_equal(h["S"][1], f["S"][1])


def test_phi_exhaustive_prop2():
    """Prop. 2: phi = cumsum(cumsum(S~)) and it equals 1 exactly once, at the first
    spike, for every binary vector up to length 12."""
    for L in range(1, 13):
        for code in range(1 << L):
            s = np.array([(code >> i) & 1 for i in range(L)], np.int64)
            z = phi(s)
            np.testing.assert_array_equal(z, np.cumsum(np.cumsum(s)))
            ones = np.flatnonzero(z == 1)
            if s.any():
                assert list(ones) == [int(np.argmax(s))]
            else:
                assert len(ones) == 0


@pytest.mark.parametrize("TR", [2, 3, 5, 8, 40])
def test_blocks_equal_standard_model(TR):
    """Props. 1-5 (the Blocks model) reproduce Eqs. 1-5 for T_R >= 2: identical
    spikes, traces to rounding."""
    g = np.random.default_rng(10 + TR)
    mism = 0
    for trial in range(12):
        tau_m = g.uniform(8.0, 30.0)
        tau_a = g.uniform(50.0, 300.0)
        d = g.uniform(0.0, 2.0)
        dt = 1.0 if TR < 8 else 0.05
        T = int(g.integers(TR * 5, TR * 40))
        I = g.uniform(-0.5, 2.5, T) + (g.random(T) < 0.1) * 3.0
        beta, p = math.exp(-dt / tau_m), math.exp(-dt / tau_a)
        f = _run(I, tau_m=tau_m, tau_a=tau_a, d=d, dt=dt, TR=TR)
        S, V, TH = blocks(I, beta, p, d, 1.0, TR)
        if not np.array_equal(S, f["S"][0]):
            mism += 1
            continue
        np.testing.assert_allclose(V, f["V"][0], rtol=0, atol=1e-11)
        np.testing.assert_allclose(TH, f["TH"][0], rtol=0, atol=1e-11)
    assert mism == 0


def test_blocks_differ_from_standard_model_at_TR1():
    """With T_R = 1 the Block model lets a neuron fire on the step right after a
    spike, which Eq. 2's reset forbids: the two disagree (why T_R >= 2 is required)."""
    g = np.random.default_rng(99)
    mism = 0
    for trial in range(40):
        T = 60
        I = g.uniform(0.0, 30.0, T)
        f = _run(I, tau_m=2.0, tau_a=100.0, d=0.1, dt=1.0, TR=1)
        S, _, _ = blocks(I, math.exp(-0.5), math.exp(-0.01), 0.1, 1.0, 1)
        mism += int(not np.array_equal(S, f["S"][0]))
    assert mism > 0


@pytest.mark.parametrize("n_in,T,weights,bias", [
    (1, 12, [(1.2,), (2.5,), (6.0,)], 0.0),
    (2, 5, [(1.5, -0.6), (2.0, 2.0), (0.7, 4.0)], 0.2)])
def test_brute_force_all_input_patterns(n_in, T, weights, bias):
    """Every binary input pattern of a tiny spike-input layer (Eq. 3 feeding
    Eqs. 1-5), over a grid of weights and T_R in {2, 3}: the oracle (its C input
    current and standard-model recurrence) equals the Blocks model of Props. 1-5
    on the current b + W x computed here, spike for spike, traces to rounding."""
    patterns = np.array([[(k >> i) & 1 for i in range(n_in * T)] for k in range(2 ** (n_in * T))],
                        np.uint8).reshape(-1, T, n_in)
    tau_m, tau_a, d, theta0, dt = 2.0, 20.0, 0.5, 1.0, 1.0
    beta, p = math.exp(-dt / tau_m), math.exp(-dt / tau_a)
    fired = 0
    for wv in weights:
        W = np.array([wv], np.float64)
        I_here = patterns.astype(np.float64) @ W[0] + bias              # [P][T]
        I_orc = oracle.input_current(patterns, W, np.array([bias]))[..., 0]
        np.testing.assert_allclose(I_orc, I_here, rtol=0, atol=1e-15)
        for TR in (2, 3):
            f = _run(I_orc, tau_m=tau_m, tau_a=tau_a, d=d, theta0=theta0, dt=dt, TR=TR)
            for r in range(len(patterns)):
                S, V, TH = blocks(I_here[r], beta, p, d, theta0, TR)
                assert np.array_equal(S, f["S"][r]), (wv, TR, r)
                np.testing.assert_allclose(V, f["V"][r], rtol=0, atol=1e-11)
                np.testing.assert_allclose(TH, f["TH"][r], rtol=0, atol=1e-11)
            fired += int(f["S"].any(axis=1).sum())
    assert fired > len(patterns)          # the grid reaches the spiking regime


def test_input_current_matches_matmul():
    g = np.random.default_rng(6)
    x = (g.random((3, 50, 37)) < 0.2).astype(np.uint8)
    W = g.standard_normal((11, 37))
    b = g.standard_normal(11)
    out = oracle.input_current(x, W, b)
    ref = x.astype(np.float64) @ W.T + b
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)


def test_projection_gradients_brute_force_and_fd():
    """Eq. 3 gradients: weight_grad and input_grad against explicit loops over
    (b, t, n, i), and weight_grad against central differences of the C oracle's
    input current (the loss sum(gI * I) is linear in W, so differences are exact
    up to rounding)."""
    g = np.random.default_rng(8)
    B, T, n_in, N = 2, 5, 4, 3
    x = (g.random((B, T, n_in)) < 0.5).astype(np.uint8)
    W = g.standard_normal((N, n_in))
    gI = g.standard_normal((B, T, N))
    dW = np.zeros((N, n_in))
    dx = np.zeros((B, T, n_in))
    for b in range(B):
        for t in range(T):
            for n in range(N):
                for i in range(n_in):
                    dW[n, i] += gI[b, t, n] * x[b, t, i]
                    dx[b, t, i] += gI[b, t, n] * W[n, i]
    np.testing.assert_allclose(oracle.weight_grad(gI, x), dW, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.input_grad(gI, W), dx, rtol=0, atol=1e-12)
    eps = 1e-3
    fd = np.zeros_like(W)
    for n in range(N):
        for i in range(n_in):
            Wp, Wm = W.copy(), W.copy()
            Wp[n, i] += eps
            Wm[n, i] -= eps
            fd[n, i] = ((gI * oracle.input_current(x, Wp)).sum() - (gI * oracle.input_current(x, Wm)).sum()) / (2 * eps)
    np.testing.assert_allclose(oracle.weight_grad(gI, x), fd, rtol=0, atol=1e-9)


def test_bth_layout_roundtrip():
    """The [B][T][N] wrapper is the row core transposed (row = (b, n))."""
    g = np.random.default_rng(7)
    B, T, N = 3, 200, 5
    I = g.uniform(0, 3, (B, T, N)).astype(np.float32)
    tm = g.uniform(10, 30, N)
    out = oracle.alif_forward(I, tm, 200.0, 1.8, 1.0, 1.0, 2.0)
    for b in range(B):
        for n in range(N):
            r = _run(I[b, :, n].astype(np.float64), tau_m=tm[n], TR=2)
            np.testing.assert_array_equal(out["S"][b, :, n], r["S"][0])
            np.testing.assert_array_equal(out["V"][b, :, n], r["V"][0])


def test_readout_closed_form():
    """Constant input c to the leaky readout: V[t] = c (1 - beta^t), so
    o = c (T - beta (1 - beta^T) / (1 - beta))."""
    c, tau, dt, T = 0.7, 20.0, 1.0, 300
    beta = math.exp(-dt / tau)
    out = oracle.readout_forward(np.full((1, T, 1), c), np.array([tau]), dt)
    expect = c * (T - beta * (1 - beta ** T) / (1 - beta))
    assert abs(out["o"][0, 0] - expect) < 1e-10
