"""Pins for the oracle's sequential surrogate-gradient adjoint (CPU only).

* Central finite differences of smooth losses sum(wV V) + sum(wTh th), which do
  not go through the spike function, at points where no spike flips.
* float64 torch autograd through a plain transcription of Eqs. 1-5 in which the
  spike has one of the three surrogate derivatives and its uses in reset,
  adaptation and refractory gate are detached (the supplementary "Detaching
  gradients" policy). Autograd derives the adjoint mechanically, so a dropped
  term or a wrong index in the hand-written adjoint shows up as a mismatch.
* The surrogate derivatives themselves against closed-form integrals over u,
  evenness and their special values.
"""
import math

import numpy as np
import pytest
import torch

import oracle


def _setup(seed, R=3, T=240, dt=0.5, TR=4):
    g = np.random.default_rng(seed)
    I = g.uniform(0.5, 5.0, (R, T)) + (g.random((R, T)) < 0.05) * 3.0
    prm = dict(tau_m=g.uniform(8, 30, R), tau_a=g.uniform(60, 300, R),
               d=g.uniform(0.2, 1.8, R), theta0=g.uniform(0.8, 1.2, R))
    return g, I, prm, dt, TR


def _fw(I, prm, dt, TR):
    return oracle.forward_rows(I, prm["tau_m"], prm["tau_a"], prm["d"], prm["theta0"], dt, TR)


def _smooth_loss(I, prm, dt, TR, wV, wT):
    f = _fw(I, prm, dt, TR)
    return float((wV * f["V"]).sum() + (wT * f["TH"]).sum()), f["S"]


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_finite_differences(seed):
    g, I, prm, dt, TR = _setup(seed)
    R, T = I.shape
    wV = g.standard_normal((R, T))
    wT = g.standard_normal((R, T))
    f = _fw(I, prm, dt, TR)
    assert f["S"].sum() > 10
    bw = oracle.backward_rows(f, prm["tau_m"], prm["tau_a"], prm["d"], prm["theta0"], dt,
                              gV=wV, gTH=wT)
    checked = 0
    for name, key in [("tau_m", "g_tau_m"), ("tau_a", "g_tau_a"), ("d", "g_d"),
                      ("theta0", "g_theta0")]:
        for r in range(R):
            h = 1e-6 * max(1.0, abs(prm[name][r]))
            up = {k: v.copy() for k, v in prm.items()}
            dn = {k: v.copy() for k, v in prm.items()}
            up[name][r] += h
            dn[name][r] -= h
            lu, su = _smooth_loss(I, up, dt, TR, wV, wT)
            ld, sd = _smooth_loss(I, dn, dt, TR, wV, wT)
            if not (np.array_equal(su, f["S"]) and np.array_equal(sd, f["S"])):
                continue                      # a spike flipped: FD not defined here
            fd = (lu - ld) / (2 * h)
            assert abs(fd - bw[key][r]) <= 1e-5 * max(1.0, abs(fd)), (name, r, fd, bw[key][r])
            checked += 1
    # gradient w.r.t. individual input currents
    for _ in range(12):
        r, t = int(g.integers(R)), int(g.integers(T))
        h = 1e-6
        Iu, Id = I.copy(), I.copy()
        Iu[r, t] += h
        Id[r, t] -= h
        lu, su = _smooth_loss(Iu, prm, dt, TR, wV, wT)
        ld, sd = _smooth_loss(Id, prm, dt, TR, wV, wT)
        if not (np.array_equal(su, f["S"]) and np.array_equal(sd, f["S"])):
            continue
        fd = (lu - ld) / (2 * h)
        assert abs(fd - bw["gI"][r, t]) <= 1e-6 * max(1.0, abs(fd)), (r, t, fd, bw["gI"][r, t])
        checked += 1
    assert checked >= 14


def _torch_surrogate(u, kind, k):
    """The three surrogate derivatives in torch (an implementation separate from
    the oracle's C code): fast sigmoid, boxcar, multi-Gaussian."""
    if kind == "boxcar":
        return 0.5 * (u.abs() <= 0.5).to(u.dtype)
    if kind == "multi_gaussian":
        nd = lambda m, sd: torch.exp(-0.5 * ((u - m) / sd) ** 2) / (sd * math.sqrt(2 * math.pi))
        return 1.15 * nd(0.0, 0.5) - 0.15 * nd(3.0, 3.0) - 0.15 * nd(-3.0, 3.0)
    return 1.0 / (k * u.abs() + 1.0) ** 2


class _ForcedSpike(torch.autograd.Function):
    """Spike with given forward decisions and a surrogate derivative."""

    @staticmethod
    def forward(ctx, u, s, k, kind="fast_sigmoid"):
        ctx.save_for_backward(u)
        ctx.k = k
        ctx.kind = kind
        return s.clone()

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        return g * _torch_surrogate(u, ctx.kind, ctx.k), None, None, None


def _torch_standard(I, prm, dt, TR, S_forced, slope, kind="fast_sigmoid", attached=False):
    """Eqs. 1-5 in torch float64 with detached spike uses (reset, adaptation, gate),
    or with ``attached`` the reset and adaptation uses left in the graph (the gate
    is a step function of the spike history either way)."""
    R, T = I.shape
    I = torch.tensor(I, dtype=torch.float64, requires_grad=True)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in prm.items()}
    beta = torch.exp(-dt / P["tau_m"])
    p = torch.exp(-dt / P["tau_a"])
    Sf = torch.tensor(S_forced, dtype=torch.float64)
    v = torch.zeros(R, dtype=torch.float64)
    a = torch.zeros(R, dtype=torch.float64)
    s_prev = torch.zeros(R, dtype=torch.float64)
    last = np.full(R, -10 ** 9)
    Vs, THs, Ss = [], [], []
    for t in range(T):
        gate = torch.tensor(((t - last) >= TR).astype(np.float64))
        sp = s_prev if attached else s_prev.detach()
        v = (beta * v + (1 - beta) * I[:, t] * gate) * (1 - sp)
        a = p * a + sp
        th = P["theta0"] + P["d"] * a
        s = _ForcedSpike.apply(v - th, Sf[:, t], slope, kind)
        last = np.where(S_forced[:, t] > 0, t, last)
        Vs.append(v)
        THs.append(th)
        Ss.append(s)
        s_prev = s
    return I, P, torch.stack(Vs, 1), torch.stack(THs, 1), torch.stack(Ss, 1)


@pytest.mark.parametrize("attached", [False, True])
@pytest.mark.parametrize("kind", ["fast_sigmoid", "boxcar", "multi_gaussian"])
@pytest.mark.parametrize("seed,TR", [(3, 2), (4, 4), (5, 9)])
def test_adjoint_matches_torch_autograd(seed, TR, kind, attached):
    g, I, prm, dt, _ = _setup(seed, R=4, T=150, TR=TR)
    R, T = I.shape
    f = _fw(I, prm, dt, TR)
    assert f["S"].sum() > 5
    wS, wV, wT = (g.standard_normal((R, T)) for _ in range(3))
    slope = 10.0
    It, P, V, TH, S = _torch_standard(I, prm, dt, TR, f["S"], slope, kind, attached)
    np.testing.assert_allclose(V.detach().numpy(), f["V"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(TH.detach().numpy(), f["TH"], rtol=0, atol=1e-12)
    loss = (torch.tensor(wS) * S).sum() + (torch.tensor(wV) * V).sum() + (torch.tensor(wT) * TH).sum()
    loss.backward()
    bw = oracle.backward_rows(f, prm["tau_m"], prm["tau_a"], prm["d"], prm["theta0"], dt,
                              slope=slope, gS=wS, gV=wV, gTH=wT, surrogate=kind, attached=attached)
    if attached:   # the two policies must differ here, or the attached pin bites nothing
        bd = oracle.backward_rows(f, prm["tau_m"], prm["tau_a"], prm["d"], prm["theta0"], dt,
                                  slope=slope, gS=wS, gV=wV, gTH=wT, surrogate=kind)
        assert np.abs(bd["gI"] - bw["gI"]).max() > 1e-6
    if kind == "boxcar":   # some steps must sit inside the window for the pin to bite
        assert (np.abs(f["V"] - f["TH"]) <= 0.5).sum() > 20
    # rounding order differs between autograd and the oracle's loop; the attached
    # adjoint adds terms that partly cancel, so its floor is relative to max |g|
    ref = It.grad.numpy()
    floor = 1e-11 * max(1.0, float(np.abs(ref).max())) if attached else 1e-12
    np.testing.assert_allclose(bw["gI"], ref, rtol=1e-10, atol=floor)
    for name, key in [("tau_m", "g_tau_m"), ("tau_a", "g_tau_a"), ("d", "g_d"), ("theta0", "g_theta0")]:
        r = P[name].grad.numpy()
        np.testing.assert_allclose(bw[key], r, rtol=1e-10,
                                   atol=1e-11 * max(1.0, float(np.abs(r).max())) if attached else 1e-12)


def test_surrogate_integrals_and_special_values():
    """The surrogate derivatives against closed forms: the integral over u of the
    fast sigmoid on [-X, X] is (2/k)(1 - 1/(kX + 1)), of the boxcar 0.5, and of
    the multi-Gaussian 1.15 - 0.15 - 0.15 = 0.85 (unit-mass Gaussians, tails beyond
    |u| = 60 negligible); all are even in u; the boxcar window is closed."""
    X, n = 60.0, 240001
    u = np.linspace(-X, X, n)
    h = u[1] - u[0]
    k = 10.0
    for kind, ref in [("fast_sigmoid", 2.0 / k * (1.0 - 1.0 / (k * X + 1.0))), ("boxcar", 0.5),
                      ("multi_gaussian", 0.85)]:
        v = np.array([oracle.surrogate(kind, x, k) for x in u])
        integral = h * (v.sum() - 0.5 * (v[0] + v[-1]))
        tol = 2 * h * 0.5 if kind == "boxcar" else 1e-6   # the boxcar jumps at the grid edges
        assert abs(integral - ref) <= tol, (kind, integral, ref)
        w = np.array([oracle.surrogate(kind, -x, k) for x in u])
        np.testing.assert_allclose(v, w, rtol=1e-13, atol=1e-16)   # even (up to summation order)
    assert oracle.surrogate("fast_sigmoid", 0.0, k) == 1.0
    assert oracle.surrogate("fast_sigmoid", 0.1, k) == 0.25
    assert oracle.surrogate("boxcar", 0.5) == 0.5 and oracle.surrogate("boxcar", -0.5) == 0.5
    assert oracle.surrogate("boxcar", 0.5 + 1e-12) == 0.0 and oracle.surrogate("boxcar", 0.0) == 0.5
    # the multi-Gaussian peaks at 0 and dips below zero in its tails
    assert oracle.surrogate("multi_gaussian", 0.0) > oracle.surrogate("multi_gaussian", 0.3) > 0
    assert oracle.surrogate("multi_gaussian", 2.0) < 0


def test_readout_adjoint_finite_differences():
    g = np.random.default_rng(8)
    B, T, C = 2, 120, 3
    Ir = g.standard_normal((B, T, C))
    tau = g.uniform(10, 30, C)
    go = g.standard_normal((B, C))
    bw = oracle.readout_backward(Ir, tau, 1.0, go)

    def L(Ir_, tau_):
        return float((oracle.readout_forward(Ir_, tau_, 1.0)["o"] * go).sum())

    for c in range(C):
        h = 1e-6 * tau[c]
        tu, td = tau.copy(), tau.copy()
        tu[c] += h
        td[c] -= h
        fd = (L(Ir, tu) - L(Ir, td)) / (2 * h)
        assert abs(fd - bw["g_tau_r"][c]) <= 1e-6 * max(1, abs(fd))
    for _ in range(6):
        b, t, c = int(g.integers(B)), int(g.integers(T)), int(g.integers(C))
        Iu, Id = Ir.copy(), Ir.copy()
        Iu[b, t, c] += 1e-6
        Id[b, t, c] -= 1e-6
        fd = (L(Iu, tau) - L(Id, tau)) / 2e-6
        assert abs(fd - bw["gIr"][b, t, c]) <= 1e-7 * max(1, abs(fd))


def test_cross_entropy_gradient():
    g = np.random.default_rng(9)
    o = g.standard_normal((5, 7))
    y = g.integers(0, 7, 5)
    loss, go = oracle.softmax_cross_entropy(o, y)
    ref = torch.nn.functional.cross_entropy(torch.tensor(o), torch.tensor(y))
    assert abs(loss - ref.item()) < 1e-12
    ot = torch.tensor(o, requires_grad=True)
    torch.nn.functional.cross_entropy(ot, torch.tensor(y)).backward()
    np.testing.assert_allclose(go, ot.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_smoothed_mse_gradient():
    g = np.random.default_rng(10)
    k = oracle.gaussian_kernel(3.0)
    assert abs(k.sum() - 1) < 1e-15 and len(k) == 2 * 12 + 1
    S = (g.random((2, 80, 3)) < 0.1).astype(np.float64)
    St = (g.random((2, 80, 3)) < 0.1).astype(np.float64)
    loss, gS = oracle.smoothed_mse(S, St, k)
    for _ in range(8):
        b, t, n = int(g.integers(2)), int(g.integers(80)), int(g.integers(3))
        Su, Sd = S.copy(), S.copy()
        Su[b, t, n] += 1e-5
        Sd[b, t, n] -= 1e-5
        fd = (oracle.smoothed_mse(Su, St, k)[0] - oracle.smoothed_mse(Sd, St, k)[0]) / 2e-5
        assert abs(fd - gS[b, t, n]) < 1e-9
