"""GPU parity of the event-driven input current (alif_input_current_events) and
of alif_transpose, through the C ABI: Eq. 3's current against the oracle's
plain projection, within the FP32 bound of summing the active terms; a spike
layer driven through it against the GEMM path."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, np_, random_params, to_dev
from paper_2311_11390_amd.synth import bernoulli_spikes, normal_weights, rng

pytestmark = pytest.mark.gpu


def _as_torch_spikes(x, kind):
    import torch
    t = torch.as_tensor(x, device="cuda")
    if kind == "u8":
        return t.to(torch.uint8).contiguous()
    if kind == "bf16":
        return t.to(torch.bfloat16).contiguous()
    return t.to(torch.float32).contiguous()


@pytest.mark.parametrize("rows,cols", [(1, 1), (33, 70), (700, 1024), (1024, 20), (5, 0)])
def test_transpose(rows, cols):
    import torch

    from paper_2311_11390_amd import alif
    g = rng(rows * 7 + cols)
    m = g.standard_normal((rows, cols)).astype(np.float32)
    out = alif.transpose(torch.as_tensor(m, device="cuda").contiguous())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(out), m.T)


@pytest.mark.parametrize("kind", ["u8", "bf16", "f32"])
@pytest.mark.parametrize("B,T,n_in,N,p", [(2, 301, 700, 260, 0.01), (1, 500, 1024, 20, 0.05),
                                          (3, 70, 37, 19, 0.3), (2, 64, 256, 1024, 0.0),
                                          (1, 40, 300, 130, 1.0), (1, 30, 2100, 1500, 0.02),
                                          (1, 1_100_000, 8, 4, 0.2), (1, 6, 20000, 70, 0.01)])
def test_input_current_events_matches_oracle(kind, B, T, n_in, N, p):
    import torch

    from paper_2311_11390_amd import alif
    g = rng(B + T + n_in + N)
    x = bernoulli_spikes(g, (B, T, n_in), p)   # binary, as Eq. 3's spikes (the oracle's projection)
    W = normal_weights(g, N, n_in)
    b = g.standard_normal(N).astype(np.float32)
    log(f"[events] {kind} B={B} T={T} n_in={n_in} N={N} p={p}")
    WT = alif.transpose(torch.as_tensor(W, device="cuda"))
    out = alif.input_current_events(_as_torch_spikes(x, kind), WT, torch.as_tensor(b, device="cuda"))
    out_nb = alif.input_current_events(_as_torch_spikes(x, kind), WT)
    torch.cuda.synchronize()
    ref = oracle.input_current(x, W.astype(np.float64), b)
    # FP32 sums of the active terms in increasing input order: the worst case is
    # (count + 1) roundings of at most the running sum of absolute terms
    absum = x.astype(np.float64) @ np.abs(W.astype(np.float64)).T + np.abs(b)
    active = (x != 0).sum(axis=2, keepdims=True)
    bound = (active + 1) * 2.0 ** -24 * absum + 1e-30
    err = np.abs(np_(out) - ref)
    assert (err <= bound).all(), float((err / bound).max())
    ref0 = oracle.input_current(x, W.astype(np.float64), None)
    assert (np.abs(np_(out_nb) - ref0) <= bound).all()
    if p == 0.0:
        np.testing.assert_array_equal(np_(out), np.broadcast_to(b, (B, T, N)))


def test_events_layer_equals_gemm_layer_spikes():
    """A spike-input ALIF layer whose current comes from the event kernel gives the
    same spikes as the FP32 GEMM path on the same input (both within FP32 of Eq. 3,
    flips only within the near-threshold band), and the oracle's on both."""
    import torch

    from paper_2311_11390_amd import alif
    B, T, n_in, N, dt = 2, 600, 200, 96, 0.5
    g = rng(91)
    x = bernoulli_spikes(g, (B, T, n_in), 0.05)
    W = (normal_weights(g, N, n_in) * 3.0).astype(np.float32)
    prm = random_params(91, N, bias=(0.5, 1.2))
    xt, Wt = torch.as_tensor(x, device="cuda"), torch.as_tensor(W, device="cuda")
    P = to_dev(prm)
    log("[events] layer vs GEMM")
    cur = alif.input_current_events(xt, alif.transpose(Wt))          # bias added by the forward
    f_ev = alif.forward(cur, P, dt, 2.0)
    f_gm = alif.forward(xt, P, dt, 2.0, Wt)
    torch.cuda.synchronize()
    s_ev, s_gm = np_(f_ev["spikes"]), np_(f_gm["spikes"])
    assert s_gm.sum() > 100
    from parity import check_forward
    rep_ev = check_forward(s_ev, oracle.input_current(x, W.astype(np.float64), None), prm, dt, 2.0)
    rep_gm = check_forward(s_gm, oracle.input_current(x, W.astype(np.float64), None), prm, dt, 2.0)
    log(f"    spikes {int(s_ev.sum())} / {int(s_gm.sum())}, excused {rep_ev['excused']} / {rep_gm['excused']}, "
        f"differing {int((s_ev != s_gm).sum())}")


@pytest.mark.parametrize("kind,off", [("u8", 1), ("u8", 2), ("u8", 3), ("bf16", 1)])
def test_input_current_events_unaligned_rows(kind, off):
    """Input views that do not start on a 4-byte boundary (element loads instead of
    word loads) give the oracle's current within the same FP32 bound."""
    import torch

    from paper_2311_11390_amd import alif
    B, T, n_in, N, p = 2, 90, 130, 70, 0.05
    g = rng(400 + off)
    x = bernoulli_spikes(g, (B, T, n_in), p)
    W = normal_weights(g, N, n_in)
    flat = _as_torch_spikes(x, kind).reshape(-1)
    buf = torch.zeros(flat.numel() + off, dtype=flat.dtype, device="cuda")
    buf[off:] = flat
    xv = buf[off:].view(B, T, n_in)
    assert xv.data_ptr() % 4 != 0
    log(f"[events] unaligned {kind} offset {off}")
    out = alif.input_current_events(xv, alif.transpose(torch.as_tensor(W, device="cuda")))
    torch.cuda.synchronize()
    ref = oracle.input_current(x, W.astype(np.float64), None)
    absum = x.astype(np.float64) @ np.abs(W.astype(np.float64)).T
    bound = ((x != 0).sum(axis=2, keepdims=True) + 1) * 2.0 ** -24 * absum + 1e-30
    assert (np.abs(np_(out) - ref) <= bound).all()


@pytest.mark.parametrize("kind", ["u8", "bf16", "f32"])
def test_input_current_events_weights_values(kind):
    """Non-binary inputs are weighted by their value: spike counts 0-3 (u8), graded
    values exact in bfloat16, and FP32 values with -0.0 entries (skipped), against the
    oracle's real-valued projection within the FP32 bound."""
    import torch

    from paper_2311_11390_amd import alif
    B, T, n_in, N = 2, 150, 300, 200
    g = rng(500 + len(kind))
    on = g.random((B, T, n_in)) < 0.05
    if kind == "u8":
        x = (on * g.integers(1, 4, (B, T, n_in))).astype(np.uint8)
        xt = torch.as_tensor(x, device="cuda")
    elif kind == "bf16":
        x = (on * g.choice([0.5, -1.25, 3.0, 0.375], (B, T, n_in))).astype(np.float32)
        xt = torch.as_tensor(x, device="cuda").to(torch.bfloat16)
    else:
        x = (on * g.standard_normal((B, T, n_in))).astype(np.float32)
        x[~on & (g.random((B, T, n_in)) < 0.5)] = -0.0
        xt = torch.as_tensor(x, device="cuda")
    W = normal_weights(g, N, n_in)
    b = g.standard_normal(N).astype(np.float32)
    log(f"[events] values {kind}")
    out = alif.input_current_events(xt.contiguous(), alif.transpose(torch.as_tensor(W, device="cuda")),
                                    torch.as_tensor(b, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle.input_current_values(x, W, b)
    absum = np.abs(x.astype(np.float64)) @ np.abs(W.astype(np.float64)).T + np.abs(b)
    bound = ((x != 0).sum(axis=2, keepdims=True) + 1) * 2.0 ** -24 * absum + 1e-30
    assert (np.abs(np_(out) - ref) <= bound).all()
