"""Pins of the oracle's counter-based OU current (oracle/ou_philox.py), the
host-side twin of the current the library draws on the device for serving
requests. Philox4x32-10 is pinned by the generator authors' published
known-answer vectors; Box-Muller and the OU recurrence by the distributions
they must produce (a dropped sqrt, a wrong decay or a swapped word shows up as
a wrong variance, autocorrelation or a correlated pair)."""
import numpy as np
import pytest
from scipy import stats

from oracle import ou_philox as op

# Philox4x32-10 known-answer vectors: (counter, key) -> output, from the
# known-answer test file distributed with Random123 by the generator's authors
# (Salmon et al., SC 2011).
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = tuple(int(w) for w in op.philox4x32_10(ctr, key))
    assert got == want


def test_philox_avalanche():
    # flipping one counter bit flips about half of the 128 output bits
    g = np.random.default_rng(1)
    base = g.integers(0, 2**32, (4, 2000), dtype=np.uint64)
    out0 = np.stack(op.philox4x32_10(tuple(base), (0x1234, 0x5678)))
    flips = []
    for word in range(4):
        for bit in (0, 13, 31):
            c = base.copy()
            c[word] ^= np.uint64(1 << bit)
            out1 = np.stack(op.philox4x32_10(tuple(c), (0x1234, 0x5678)))
            x = out0 ^ out1
            flips.append(sum(bin(int(v)).count("1") for v in x.ravel()) / base.shape[1])
    assert all(abs(f - 64.0) < 1.0 for f in flips), flips


def test_normals_are_standard_and_independent():
    z = op.standard_normals(2000, 128, seed=7)
    assert z.shape == (2000, 128)
    flat = z.ravel()
    assert abs(flat.mean()) < 0.01
    assert abs(flat.var() - 1.0) < 0.015
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    # the cos / sin halves of a Box-Muller pair, consecutive steps, neighbours
    for a, b in ((z[0::2], z[1::2]), (z[:-1], z[1:]), (z[:, :-1], z[:, 1:]), (z[0::4], z[2::4])):
        r = np.corrcoef(a.ravel(), b.ravel())[0, 1]
        assert abs(r) < 0.01, r


def test_stream_layout_is_independent_of_shape():
    big = op.standard_normals(1001, 70, seed=2**40 + 3)
    small = op.standard_normals(301, 7, seed=2**40 + 3)
    np.testing.assert_array_equal(small, big[:301, :7])
    other = op.standard_normals(301, 7, seed=2**40 + 4)
    assert not np.allclose(small, other)


def test_ou_stationary_law_and_autocorrelation():
    T, N, dt, tau, mu, sd = 1500, 4000, 0.05, 5.0, 0.8, 0.5
    I32, I = op.ou_current(T, N, dt, tau, mu, sd, seed=11)
    assert I32.dtype == np.float32 and I32.shape == (T, N)
    assert np.abs(I32 - I).max() <= np.spacing(np.float32(4.0))
    X = I - mu
    se_var = sd * sd * np.sqrt(2.0 / N)
    for t in (0, 1, 700, T - 1):
        assert abs(X[t].mean()) < 5 * sd / np.sqrt(N)
        assert abs(X[t].var() - sd * sd) < 5 * se_var, (t, X[t].var())
    e = np.exp(-dt / tau)
    for k in (1, 20, 200):
        r = np.corrcoef(X[1000], X[1000 - k])[0, 1]
        assert abs(r - e ** k) < 5 * (1 - e ** (2 * k)) / np.sqrt(N) + 1e-3, (k, r, e ** k)


def test_ou_degenerate_cases():
    I32, I = op.ou_current(50, 3, 1.0, 5.0, 0.8, 0.0, seed=3)
    assert np.all(I == np.float32(0.8).astype(np.float64))
    I32, I = op.ou_current(1, 5, 1.0, 5.0, 0.0, 1.0, seed=3)
    np.testing.assert_allclose(I[0], op.standard_normals(1, 5, 3)[0])
    I32, I = op.ou_current(0, 5, 1.0, 5.0, 0.0, 1.0, seed=3)
    assert I32.shape == (0, 5)
