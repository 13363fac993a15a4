"""GPU parity of the neural-fit pieces (supplementary "Neural fits") through the C ABI:
the van Rossum distance and its gradient, the Adam step, and one fitting epoch
(forward, loss, surrogate-gradient backward) against the oracle's chain."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import gpu_forward, log, np_, random_params
from parity import check_forward, check_grad
from paper_2311_11390_amd.synth import rng

pytestmark = pytest.mark.gpu


def _trains(seed, B, R, T, N, p=0.08, counts=False):
    g = rng(seed)
    x = (g.random((B, T, N)) < p).astype(np.uint8)
    y = (g.random((B, R, T, N)) < p).astype(np.uint8)
    if counts:
        y += (g.random((B, R, T, N)) < p / 4).astype(np.uint8)
    if B and N and R:
        y[0, 0, :, 0] = x[0, :, 0]          # one column at distance 0
    return x, y


def _grad_tol(T, g_ref):
    """FP32 recurrences over at most T steps: T * 2^-22 of the largest gradient."""
    return max(T, 64) * 2.0 ** -22 * float(np.abs(g_ref).max(initial=0.0)) + 1e-30


def _gpu_vr(x, y, dt, tau, scale, **kw):
    import torch

    from paper_2311_11390_amd import alif
    xs = torch.as_tensor(x, device="cuda").contiguous()
    ys = torch.as_tensor(y, device="cuda").contiguous()
    d, gr, _ = alif.van_rossum(xs, ys, dt, tau, scale=scale, **kw)
    torch.cuda.synchronize()
    return np_(d), np_(gr)


@pytest.mark.parametrize("B,R,T,N,dt,tau", [
    (2, 1, 300, 64, 0.5, 10.0),        # four neurons per thread
    (3, 1, 1001, 67, 0.1, 20.0),       # one neuron per thread, ragged T
    (2, 4, 777, 36, 1.0, 100.0),       # four repeats in one pass
    (1, 5, 4099, 20, 0.05, 100.0),     # two repeat groups, many chunks
    (2, 8, 513, 12, 0.25, 5.0),        # the most repeats
])
def test_van_rossum_matches_oracle(B, R, T, N, dt, tau):
    x, y = _trains(B * 1000 + T, B, R, T, N, counts=(R == 4))
    scale = 1.0 / (B * R * N)
    log(f"[vr] B={B} R={R} T={T} N={N} dt={dt} tau={tau}")
    d, gr = _gpu_vr(x, y, dt, tau, scale)
    D, G = oracle.van_rossum(x, y, dt, tau, scale)
    assert d.shape == (B, R, N) and gr.shape == (B, T, N)
    np.testing.assert_allclose(d, D, rtol=2e-6, atol=1e-7)
    assert d[0, 0, 0] == 0.0
    np.testing.assert_allclose(gr, G, rtol=0, atol=_grad_tol(T, G))
    log(f"    max |dD| {np.abs(d - D).max():.2e}  max |dgrad| / max|grad| "
        f"{np.abs(gr - G).max() / np.abs(G).max():.2e}")


@pytest.mark.parametrize("B,R,T,N", [(1, 1, 1, 4), (1, 2, 15, 5), (2, 3, 17, 8), (1, 5, 31, 3)])
def test_van_rossum_short_trains(B, R, T, N):
    """Trains shorter than one 16-step piece, or just over one, with one or four
    neurons per thread and one or two repeat groups."""
    x, y = _trains(77 + T, B, R, T, N, p=0.3)
    log(f"[vr] short B={B} R={R} T={T} N={N}")
    d, gr = _gpu_vr(x, y, 0.5, 3.0, 0.25)
    D, G = oracle.van_rossum(x, y, 0.5, 3.0, 0.25)
    np.testing.assert_allclose(d, D, rtol=2e-6, atol=1e-7)
    np.testing.assert_allclose(gr, G, rtol=0, atol=_grad_tol(T, G))


def test_van_rossum_outputs_alone_and_empty():
    import torch

    from paper_2311_11390_amd import alif
    x, y = _trains(5, 2, 2, 200, 8)
    d_both, g_both = _gpu_vr(x, y, 0.5, 10.0, 0.5)
    d_only, g_none = _gpu_vr(x, y, 0.5, 10.0, 0.5, want_grad=False)
    d_none, g_only = _gpu_vr(x, y, 0.5, 10.0, 0.5, want_dist=False)
    assert g_none is None and d_none is None
    np.testing.assert_array_equal(d_only, d_both)
    np.testing.assert_array_equal(g_only, g_both)
    # identical trains: zero distance and zero gradient
    d0, g0 = _gpu_vr(x, np.stack([x, x], axis=1), 0.5, 10.0, 1.0)
    assert (d0 == 0).all() and (g0 == 0).all()
    # T = 0: distances 0; B = 0 and N = 0: nothing to do
    log("[vr] empty shapes")
    dz, gz = _gpu_vr(np.zeros((2, 0, 8), np.uint8), np.zeros((2, 3, 0, 8), np.uint8), 0.5, 10.0, 1.0)
    assert dz.shape == (2, 3, 8) and (dz == 0).all() and gz.shape == (2, 0, 8)
    for shp in [(0, 10, 8), (2, 10, 0)]:
        xs = torch.zeros(shp, dtype=torch.uint8, device="cuda")
        ys = torch.zeros((shp[0], 1) + shp[1:], dtype=torch.uint8, device="cuda")
        d, g, _ = alif.van_rossum(xs, ys, 0.5, 10.0)
        torch.cuda.synchronize()
        assert d.numel() == 0 and g.numel() == 0


def test_van_rossum_fullsize_sampled():
    """The fit workload's size (4 stimuli x 4 repeats x 20000 steps x 2048 neurons at
    DT 0.1 ms, tau_R 100 ms): sampled columns against the oracle one by one."""
    import torch

    from paper_2311_11390_amd import alif
    B, R, T, N = 4, 4, 20000, 2048
    g = torch.Generator(device="cuda").manual_seed(3)
    log(f"[vr] full size B={B} R={R} T={T} N={N}")
    x = (torch.rand((B, T, N), device="cuda", generator=g) < 0.004).to(torch.uint8)
    y = (torch.rand((B, R, T, N), device="cuda", generator=g) < 0.004).to(torch.uint8)
    d, gr, _ = alif.van_rossum(x, y, 0.1, 100.0, scale=1.0 / (B * R * N))
    torch.cuda.synchronize()
    cols = [0, 1, 2, 3, 511, 1024, 2047]
    xs = x[:, :, cols].cpu().numpy()
    ys = y[:, :, :, cols].cpu().numpy()
    D, G = oracle.van_rossum(xs, ys, 0.1, 100.0, 1.0 / (B * R * N))
    np.testing.assert_allclose(d[:, :, cols].cpu().numpy(), D, rtol=2e-6, atol=1e-7)
    gs = gr[:, :, cols].cpu().numpy()
    np.testing.assert_allclose(gs, G, rtol=0, atol=_grad_tol(T, G))
    log(f"    max |dgrad| / max|grad| {np.abs(gs - G).max() / np.abs(G).max():.2e}")


def test_adam_matches_oracle():
    import torch

    from paper_2311_11390_amd import alif
    g = rng(11)
    n = 1000
    p = g.uniform(0.5, 30.0, n)
    ps = torch.tensor(p, dtype=torch.float32, device="cuda")
    ms = torch.zeros(n, dtype=torch.float32, device="cuda")
    vs = torch.zeros(n, dtype=torch.float32, device="cuda")
    pr, mr, vr = p.astype(np.float32).astype(np.float64), np.zeros(n), np.zeros(n)
    mabs = np.zeros(n)   # the same average of |g|: FP32 rounding of m is relative to it (terms may cancel)
    for step in range(1, 6):
        gr = (g.standard_normal(n) * 10 ** g.uniform(-3, 2, n)).astype(np.float32)
        alif.adam_step(ps, torch.tensor(gr, device="cuda"), ms, vs, step, 0.3, 0.9, 0.999, 1e-8, 1.0, 29.0)
        pr, mr, vr = oracle.adam_step(pr, gr, mr, vr, step, 0.3, 0.9, 0.999, 1e-8, 1.0, 29.0)
        mabs = 0.9 * mabs + 0.1 * np.abs(gr)
        torch.cuda.synchronize()
        np.testing.assert_allclose(ps.cpu().numpy(), pr, rtol=2e-6, atol=1e-5)
        assert (np.abs(ms.cpu().numpy() - mr) <= 4 * step * 2.0 ** -24 * mabs).all()
        np.testing.assert_allclose(vs.cpu().numpy(), vr, rtol=4 * step * 2.0 ** -24, atol=0)
    assert (ps.cpu().numpy() >= 1.0).all() and (ps.cpu().numpy() <= 29.0).all()


@pytest.mark.parametrize("TR,dt,R", [(20, 0.1, 2), (4, 0.5, 1)])
def test_fit_epoch_gradients_match_oracle(TR, dt, R):
    """forward -> van Rossum gradient -> surrogate-gradient backward: the parameter
    gradients of one fitting epoch against the oracle's chain on the same spikes."""
    import torch

    from paper_2311_11390_amd import alif
    B, N, T = 2, 40, 2000
    g = rng(70 + TR)
    I = (1.3 + 1.0 * g.standard_normal((B, T, N))).astype(np.float32)
    prm = random_params(70 + TR, N, tm=(10.0, 30.0), ta=(80.0, 200.0), d=(0.05, 0.3), bias=(-0.1, 0.1))
    y = (g.random((B, R, T, N)) < 0.01).astype(np.uint8)
    arp = TR * dt
    log(f"[fit epoch] T_R={TR} dt={dt} R={R}")
    f, It, P = gpu_forward(I, prm, dt, arp, traces=False, save=True)
    S = f["spikes"]
    _, gS, _ = alif.van_rossum(S, torch.as_tensor(y, device="cuda"), dt, 100.0, scale=1.0 / (B * R * N),
                               want_dist=False)
    out = alif.backward(f, It, P, grad_spikes=gS)
    torch.cuda.synchronize()
    Sn = np_(S)
    assert Sn.sum() > 50
    rep = check_forward(Sn, I, prm, dt, arp)
    _, Go = oracle.van_rossum(Sn, y, dt, 100.0, 1.0 / (B * R * N))
    ob = oracle.alif_backward(rep["oracle"], dt, 10.0, gS=Go)
    check_grad("grad_tau_mem", np_(out["grad_tau_mem"]), ob["g_tau_m"])
    check_grad("grad_tau_adapt", np_(out["grad_tau_adapt"]), ob["g_tau_a"])
    check_grad("grad_d", np_(out["grad_d"]), ob["g_d"])
    check_grad("grad_theta0", np_(out["grad_theta0"]), ob["g_theta0"])
    check_grad("grad_bias", np_(out["grad_bias"]), ob["gI"].sum(axis=(0, 1)))
