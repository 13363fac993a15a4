"""Pins for the fine-DT workload's loss in the oracle (CPU only): the mean squared
error between Gaussian-smoothed spike trains, G * S against G * S_target, with G
a unit-sum discrete Gaussian of sigma 2 ms cut at +-4 sigma and the convolution
taken along time with zero padding ("same" length).

Each pin fixes the oracle to something other than itself:
* the smoothing against scipy.ndimage's Gaussian filter (a library routine with
  the same unit-sum kernel, radius and zero padding) and against an explicit
  zero-padded sum over the kernel taps, on [B][T][N] arrays whose three sizes
  differ, so a convolution along the wrong axis fails;
* one spike gives the centred kernel at its own step, cut at the train's ends;
* a 1 x 5 x 1 train worked by hand fixes the loss's 1/M normalisation and its
  gradient;
* the benchmark's FFT form of the loss gradient (the dL/dS the timed step
  consumes) equals the oracle's gradient.
"""
import numpy as np
import pytest

import oracle


def _explicit_same_conv(x, k):
    """sum_j k[j] x[t + h - j] over valid t + h - j, along axis 1 (the time axis)."""
    B, T, N = x.shape
    h = (len(k) - 1) // 2
    out = np.zeros_like(x, dtype=np.float64)
    for t in range(T):
        for j in range(len(k)):
            s = t + h - j
            if 0 <= s < T:
                out[:, t, :] += k[j] * x[:, s, :]
    return out


@pytest.mark.parametrize("sigma", [2.5, 3.0, 40.0])
def test_gaussian_kernel_matches_scipy_filter(sigma):
    ndimage = pytest.importorskip("scipy.ndimage")
    k = oracle.gaussian_kernel(sigma)
    h = (len(k) - 1) // 2
    assert h == int(np.ceil(4 * sigma)) and abs(k.sum() - 1.0) < 1e-14
    assert np.allclose(k, k[::-1], rtol=0, atol=0)          # symmetric
    assert np.argmax(k) == h                                  # centred
    # a unit impulse at the centre of a long train returns the filter's own taps
    T = 2 * h + 1
    x = np.zeros((1, T, 1))
    x[0, h, 0] = 1.0
    ref = ndimage.gaussian_filter1d(x, sigma, axis=1, mode="constant", cval=0.0, truncate=4.0)
    np.testing.assert_allclose(oracle.smooth_time(x, k)[0, :, 0], ref[0, :, 0], rtol=0, atol=1e-15)


def test_smooth_time_axis_and_padding():
    ndimage = pytest.importorskip("scipy.ndimage")
    g = np.random.default_rng(5)
    B, T, N = 3, 47, 5                      # three different sizes: a wrong axis cannot match
    x = (g.random((B, T, N)) < 0.2).astype(np.float64) * g.uniform(0.5, 2.0, (B, T, N))
    k = oracle.gaussian_kernel(2.5)          # 21 taps, several of them past each end of the train
    got = oracle.smooth_time(x, k)
    np.testing.assert_allclose(got, _explicit_same_conv(x, k), rtol=0, atol=1e-14)
    ref = ndimage.gaussian_filter1d(x, 2.5, axis=1, mode="constant", cval=0.0, truncate=4.0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
    # an asymmetric kernel fixes the orientation: out[t] = sum_j k[j] x[t + h - j]
    ka = np.array([0.1, 0.2, 0.7])
    np.testing.assert_allclose(oracle.smooth_time(x, ka), _explicit_same_conv(x, ka), rtol=0, atol=1e-15)


def test_single_spike_gives_centred_kernel_cut_at_the_ends():
    k = oracle.gaussian_kernel(3.0)          # h = 12
    h = 12
    B, T, N = 2, 30, 3
    for s in (0, 5, 14, 29):
        x = np.zeros((B, T, N))
        x[1, s, 2] = 1.0
        y = oracle.smooth_time(x, k)
        expect = np.zeros(T)
        for t in range(T):
            if abs(t - s) <= h:
                expect[t] = k[h + (t - s)]
        np.testing.assert_allclose(y[1, :, 2], expect, rtol=0, atol=1e-16)
        y[1, :, 2] = 0.0
        assert not y.any()                   # nothing leaks into other rows or neurons


def test_smoothed_mse_worked_by_hand():
    # S = [0, 1, 0, 0, 1], target silent, kernel [1/4, 1/2, 1/4]:
    # G*S = [1/4, 1/2, 1/4, 1/4, 1/2]; squares sum to 11/16 over M = 5 elements.
    S = np.array([0, 1, 0, 0, 1], np.float64).reshape(1, 5, 1)
    St = np.zeros_like(S)
    k = np.array([0.25, 0.5, 0.25])
    loss, g = oracle.smoothed_mse(S, St, k)
    assert abs(loss - (11.0 / 16.0) / 5.0) < 1e-15
    # dL/dS[t] = (2/M) sum_u diff[u] k[u - t + 1]: (2/5) [1/4, 3/8, 5/16, 5/16, 5/16]
    np.testing.assert_allclose(g[0, :, 0], 0.4 * np.array([0.25, 0.375, 0.3125, 0.3125, 0.3125]),
                               rtol=0, atol=1e-16)
    # the mean is over every element: the same trains in a [2][5][3] batch (other entries equal on
    # both sides) keep the summed error and divide it by 30
    S2 = np.zeros((2, 5, 3))
    S2[1, :, 1] = S[0, :, 0]
    loss2, g2 = oracle.smoothed_mse(S2, np.zeros_like(S2), k)
    assert abs(loss2 - (11.0 / 16.0) / 30.0) < 1e-15
    np.testing.assert_allclose(g2[1, :, 1], g[0, :, 0] * 5.0 / 30.0, rtol=0, atol=1e-16)


def test_bench_loss_gradient_equals_oracle():
    """The timed step's dL/dS comes from an FFT form of the same loss; on CPU
    tensors it must equal the oracle's gradient."""
    torch = pytest.importorskip("torch")
    import bench
    g = np.random.default_rng(8)
    B, T, N = 2, 300, 3
    sigma = 7.0
    S = (g.random((B, T, N)) < 0.03).astype(np.float32)
    St = (g.random((B, T, N)) < 0.03).astype(np.float32)
    got = bench.smoothed_mse_grad(torch.from_numpy(S), torch.from_numpy(St), sigma).numpy()
    _, ref = oracle.smoothed_mse(S, St, oracle.gaussian_kernel(sigma))
    # FP32 FFT of trains whose smoothed values are <= 1: error a few ulps of the largest gradient
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
