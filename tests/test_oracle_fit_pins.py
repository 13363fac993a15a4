"""Pins for the oracle's neural-fit pieces (supplementary "Neural fits"), CPU only.

Van Rossum distance (supplementary "Supervised training loss"):
* an explicit double sum over (t, s) of exp(-(t - s) dt / tau), on tiny inputs;
* closed forms: one spike against none gives D^2 = (dt/tau)(1 - a^(2(T - t1)))/(1 - a^2),
  two single spikes Delta steps apart the geometric-series form, and both tend to the
  continuous-time values 1/2 and 1 - exp(-Delta dt / tau) as dt -> 0;
* metric properties: D(x, x) = 0, symmetry, invariance to a common shift;
* the gradient against central finite differences of D with real-valued x, for
  one and several repeats, and zero where D = 0.
Adam: against torch.optim.Adam on the CPU in float64 (a library routine).
"""
import math

import numpy as np
import pytest

import oracle


def _brute_force(x, y, dt, tau):
    """D[b][n] by the definition with explicit kernel sums (x, y [B][T][N])."""
    B, T, N = x.shape
    D = np.zeros((B, N))
    for b in range(B):
        for n in range(N):
            acc = 0.0
            for t in range(T):
                kx = sum(math.exp(-(t - s) * dt / tau) * x[b, s, n] for s in range(t + 1))
                ky = sum(math.exp(-(t - s) * dt / tau) * y[b, s, n] for s in range(t + 1))
                acc += (kx - ky) ** 2
            D[b, n] = math.sqrt(acc * dt / tau)
    return D


def test_van_rossum_equals_explicit_kernel_sums():
    g = np.random.default_rng(0)
    x = (g.random((2, 23, 3)) < 0.3).astype(np.uint8)
    y = (g.random((2, 23, 3)) < 0.3).astype(np.uint8)
    y[0, :, 0] = x[0, :, 0]
    D, _ = oracle.van_rossum(x, y, 0.5, 4.0)
    ref = _brute_force(x.astype(float), y.astype(float), 0.5, 4.0)
    np.testing.assert_allclose(D[:, 0, :], ref, rtol=1e-13, atol=1e-15)
    assert D[0, 0, 0] == 0.0


@pytest.mark.parametrize("t1", [0, 17, 290])
def test_van_rossum_one_spike_closed_form(t1):
    T, dt, tau = 300, 0.25, 10.0
    x = np.zeros((1, T, 1))
    x[0, t1, 0] = 1
    D, _ = oracle.van_rossum(x, np.zeros_like(x), dt, tau)
    a = math.exp(-dt / tau)
    want = dt / tau * (1 - a ** (2 * (T - t1))) / (1 - a * a)
    assert D[0, 0, 0] ** 2 == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("delta", [1, 8, 120])
def test_van_rossum_two_spikes_closed_form(delta):
    T, dt, tau, t1 = 400, 0.5, 20.0, 30
    x = np.zeros((1, T, 1))
    y = np.zeros_like(x)
    x[0, t1, 0] = 1
    y[0, t1 + delta, 0] = 1
    a = math.exp(-dt / tau)
    t2 = t1 + delta
    q = 1 - a * a
    want = dt / tau * ((1 - a ** (2 * (T - t1))) / q + (1 - a ** (2 * (T - t2))) / q
                       - 2 * a ** delta * (1 - a ** (2 * (T - t2))) / q)
    for xx, yy in ((x, y), (y, x)):
        D, _ = oracle.van_rossum(xx, yy, dt, tau)
        assert D[0, 0, 0] ** 2 == pytest.approx(want, rel=1e-12)


def test_van_rossum_continuous_time_limit():
    """dt/tau = 1e-4 over 12 tau: within 2 dt/tau (relative) of the continuous values."""
    dt, tau = 0.01, 100.0
    T = int(12 * tau / dt)
    x = np.zeros((1, T, 2))
    y = np.zeros_like(x)
    x[0, 10, 0] = 1                               # one spike against none
    x[0, 10, 1] = 1
    y[0, 10 + 3000, 1] = 1                        # 30 ms apart
    D, _ = oracle.van_rossum(x, y, dt, tau)
    bound = 2 * dt / tau
    assert D[0, 0, 0] ** 2 == pytest.approx(0.5, rel=bound)
    assert D[0, 0, 1] ** 2 == pytest.approx(1 - math.exp(-30.0 / tau), rel=bound)


def test_van_rossum_metric_properties():
    g = np.random.default_rng(3)
    T = 200
    x = np.zeros((1, T + 50, 4))
    y = np.zeros_like(x)
    x[0, :T] = g.random((T, 4)) < 0.05
    y[0, :T] = g.random((T, 4)) < 0.05
    D, _ = oracle.van_rossum(x, y, 0.2, 5.0)
    Dr, _ = oracle.van_rossum(y, x, 0.2, 5.0)
    np.testing.assert_array_equal(D, Dr)
    D0, grad0 = oracle.van_rossum(x, x, 0.2, 5.0)
    assert (D0 == 0).all() and (grad0 == 0).all()
    # shifting both trains by 50 steps: the same distance up to the tail cut at T
    xs, ys = np.roll(x, 50, axis=1), np.roll(y, 50, axis=1)
    long_x = np.concatenate([x, np.zeros((1, 2000, 4))], axis=1)
    long_y = np.concatenate([y, np.zeros((1, 2000, 4))], axis=1)
    long_xs = np.concatenate([xs, np.zeros((1, 2000, 4))], axis=1)
    long_ys = np.concatenate([ys, np.zeros((1, 2000, 4))], axis=1)
    np.testing.assert_allclose(oracle.van_rossum(long_xs, long_ys, 0.2, 5.0)[0],
                               oracle.van_rossum(long_x, long_y, 0.2, 5.0)[0], rtol=1e-12)


@pytest.mark.parametrize("R", [1, 3])
def test_van_rossum_gradient_finite_differences(R):
    g = np.random.default_rng(10 + R)
    B, T, N, dt, tau, scale = 2, 40, 3, 0.5, 6.0, 0.37
    x = g.random((B, T, N))
    y = g.random((B, R, T, N)) * (g.random((B, R, T, N)) < 0.5)
    _, grad = oracle.van_rossum(x, y, dt, tau, scale)

    def loss(xx):
        return scale * oracle.van_rossum(xx, y, dt, tau)[0].sum()

    h = 1e-6
    for (b, t, n) in [(0, 0, 0), (1, 39, 2), (0, 17, 1), (1, 5, 0), (0, 33, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[b, t, n] += h
        xm[b, t, n] -= h
        fd = (loss(xp) - loss(xm)) / (2 * h)
        assert grad[b, t, n] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(7)
    p0 = g.standard_normal(11)
    grads = g.standard_normal((6, 11))
    P = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([P], lr=0.03, betas=(0.8, 0.99), eps=1e-6)
    p, m, v = p0.copy(), np.zeros(11), np.zeros(11)
    for k in range(6):
        opt.zero_grad()
        P.grad = torch.tensor(grads[k])
        opt.step()
        p, m, v = oracle.adam_step(p, grads[k], m, v, k + 1, 0.03, 0.8, 0.99, 1e-6)
        np.testing.assert_allclose(p, P.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_projection():
    p, m, v = oracle.adam_step(np.array([1.0, 5.0]), np.array([1.0, -1.0]), np.zeros(2), np.zeros(2),
                               1, 2.0, lo=0.5, hi=6.0)
    # the first bias-corrected step moves each parameter by lr against its gradient's sign
    np.testing.assert_allclose(p, [0.5, 6.0])
