"""Pins for the oracle's real-valued Eq. 3 projection (input_current_values), CPU only:
a hand-computed case, agreement with the binary spike sum (the C loop of
input_current) on 0/1 inputs, and linearity in x."""
import numpy as np

import oracle


def test_hand_computed():
    x = np.array([[2.0, 0.0, 1.0]])
    W = np.array([[1.0, 2.0, 3.0], [-1.0, 0.5, 4.0]])
    b = np.array([0.5, -1.0])
    # [2*1 + 0*2 + 1*3 + 0.5, 2*(-1) + 0*0.5 + 1*4 - 1]
    np.testing.assert_array_equal(oracle.input_current_values(x, W, b), [[5.5, 1.0]])


def test_binary_inputs_equal_the_spike_sum():
    g = np.random.default_rng(5)
    x = (g.random((3, 40, 57)) < 0.2).astype(np.uint8)
    W = g.standard_normal((23, 57))
    b = g.standard_normal(23)
    np.testing.assert_allclose(oracle.input_current_values(x, W, b), oracle.input_current(x, W, b),
                               rtol=1e-12, atol=1e-12)


def test_linear_in_x():
    g = np.random.default_rng(6)
    x1 = g.standard_normal((10, 31)) * (g.random((10, 31)) < 0.3)
    x2 = g.integers(0, 4, (10, 31)).astype(np.float64)
    W = g.standard_normal((9, 31))
    b = g.standard_normal(9)
    f = lambda x: oracle.input_current_values(x, W, b) - b
    np.testing.assert_allclose(f(1.5 * x1 - x2), 1.5 * f(x1) - f(x2), rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(oracle.input_current_values(np.zeros((2, 31)), W, b), np.broadcast_to(b, (2, 9)))
