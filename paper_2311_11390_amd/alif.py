"""Torch-facing wrappers of libblockalif.

PyTorch supplies device memory and the current stream; every step of the ALIF
path runs in the library's HIP kernels. There is no CPU fallback: if the
library is missing, importing the binding raises.

Layout: every per-step tensor is [B][T][N] (batch, step, neuron), contiguous.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Params:
    """Per-neuron ALIF parameters, float32 [N] device tensors. ``d`` is the paper's
    adaptation scalar (threshold jump per spike)."""
    tau_mem: torch.Tensor
    tau_adapt: torch.Tensor
    d: torch.Tensor
    theta0: torch.Tensor
    bias: torch.Tensor | None = None

    def c(self) -> L.AlifParams:
        for t in (self.tau_mem, self.tau_adapt, self.d, self.theta0, self.bias):
            if t is not None:
                assert t.dtype == torch.float32 and t.is_contiguous() and t.is_cuda
        return L.AlifParams(self.tau_mem.data_ptr(), self.tau_adapt.data_ptr(), self.d.data_ptr(),
                            self.theta0.data_ptr(), None if self.bias is None else self.bias.data_ptr())

    @staticmethod
    def from_numpy(lp, device="cuda"):
        f = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float32, device=device).contiguous()
        return Params(f(lp.tau_mem), f(lp.tau_adapt), f(lp.d), f(lp.theta0), f(getattr(lp, "bias", None)))


_SPIKE_TORCH = {L.SPIKES_U8: torch.uint8, L.SPIKES_BF16: torch.bfloat16, L.SPIKES_F32: torch.float32}
_INPUT_KIND = {torch.uint8: L.INPUT_SPIKES_U8, torch.bfloat16: L.INPUT_SPIKES_BF16,
               torch.float32: L.INPUT_SPIKES_F32}


def refractory_steps(dt_ms: float, arp_ms: float) -> int:
    return L.check(L.load().alif_refractory_steps(float(dt_ms), float(arp_ms)))


def make_desc(B, T, N, dt, arp, n_in=0, input_kind=L.INPUT_CURRENT_F32, gemm_precision=L.GEMM_FP32,
              spike_dtype=L.SPIKES_U8, algo=L.ALGO_BLOCKS, slope=10.0,
              surrogate=L.SG_FAST_SIGMOID, grad_policy=L.GRAD_DETACHED) -> L.AlifDesc:
    return L.AlifDesc(int(B), int(n_in), int(N), int(T), float(dt), float(arp), int(input_kind),
                      int(gemm_precision), int(spike_dtype), int(algo), int(surrogate), float(slope),
                      int(grad_policy))


def carry_bytes(desc) -> int:
    n = ctypes.c_size_t()
    L.check(L.load().alif_carry_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def backward_workspace_bytes(desc) -> int:
    n = ctypes.c_size_t()
    L.check(L.load().alif_backward_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def new_state(B, N, device="cuda"):
    return {"v": torch.zeros(B, N, dtype=torch.float64, device=device),
            "a": torch.zeros(B, N, dtype=torch.float64, device=device),
            "ts": torch.zeros(B, N, dtype=torch.int32, device=device)}


def _cstate(s):
    return None if s is None else L.AlifState(s["v"].data_ptr(), s["a"].data_ptr(), s["ts"].data_ptr())


def forward(inp: torch.Tensor, params: Params, dt: float, arp: float, W: torch.Tensor | None = None, *,
            gemm_precision=L.GEMM_FP32, spike_dtype=L.SPIKES_U8, algo=L.ALGO_BLOCKS,
            want_v=False, want_theta=False, save=False, init=None, want_final=False,
            slope=10.0, surrogate=L.SG_FAST_SIGMOID, grad_policy=L.GRAD_DETACHED, out=None) -> dict:
    """One ALIF layer over T steps (alif_forward).

    ``inp`` is the current float32 [B][T][N] when ``W`` is None, else presynaptic
    spikes [B][T][n_in] (uint8, bfloat16 or float32 0/1). Returns a dict with
    ``spikes`` (dtype from ``spike_dtype``), optional ``v``/``theta``, and what the
    backward needs (``current``, ``carries``, ``desc``) when ``save``. ``surrogate``
    (SG_FAST_SIGMOID with ``slope``, SG_BOXCAR, SG_MULTI_GAUSSIAN) selects the
    surrogate derivative the backward of this forward uses, ``grad_policy``
    (GRAD_DETACHED, GRAD_ATTACHED) its gradient policy."""
    assert inp.is_cuda and inp.is_contiguous()
    B, T = inp.shape[0], inp.shape[1]
    dev = inp.device
    if W is None:
        assert inp.dtype == torch.float32
        N, n_in, kind = inp.shape[2], 0, L.INPUT_CURRENT_F32
    else:
        assert W.dtype == torch.float32 and W.is_contiguous()
        N, n_in = W.shape
        assert inp.shape[2] == n_in
        kind = _INPUT_KIND[inp.dtype]
    desc = make_desc(B, T, N, dt, arp, n_in, kind, gemm_precision, spike_dtype, algo, slope, surrogate,
                     grad_policy)
    o = out or {}
    spikes = o.get("spikes")
    if spikes is None:
        spikes = torch.empty(B, T, N, dtype=_SPIKE_TORCH[spike_dtype], device=dev)
    v = o.get("v", torch.empty(B, T, N, dtype=torch.float32, device=dev) if want_v else None)
    th = o.get("theta", torch.empty(B, T, N, dtype=torch.float32, device=dev) if want_theta else None)
    current = None
    if W is not None:
        current = o.get("current")
        if current is None:
            current = torch.empty(B, T, N, dtype=torch.float32, device=dev)
    carries = None
    if save or algo == L.ALGO_SEQUENTIAL_STEP:
        carries = o.get("carries")
        if carries is None:
            carries = torch.empty(max(1, carry_bytes(desc)), dtype=torch.uint8, device=dev)
    final = new_state(B, N, dev) if want_final else None
    cp = params.c()
    L.check(L.load().alif_forward(ctypes.byref(desc), ctypes.byref(cp), _p(inp), _p(W), _p(current),
                                  None if init is None else ctypes.byref(_cstate(init)),
                                  None if final is None else ctypes.byref(_cstate(final)),
                                  _p(spikes), _p(v), _p(th), _p(carries), _stream(dev)))
    return {"spikes": spikes, "v": v, "theta": th, "current": current, "carries": carries,
            "final": final, "desc": desc}


def backward(fwd: dict, inp: torch.Tensor, params: Params, W: torch.Tensor | None = None, *,
             grad_spikes=None, grad_v=None, grad_theta=None, want_grad_current=False,
             want_grad_input=False, want_grad_W=False, want_param_grads=True, workspace=None,
             noalloc=False) -> dict:
    """Surrogate-gradient backward (alif_backward) of a ``forward(..., save=True)``.
    ``noalloc`` calls alif_backward_noalloc instead, whose scratch is the library's
    static device array (no workspace is allocated or passed). ``grad_current`` is
    returned when asked for, and for spike input whenever grad_W or grad_input is,
    except under BF16 GEMMs with the detached block backward and a multiple of 8
    neurons (then None)."""
    desc = fwd["desc"]
    B, T, N = desc.batch, desc.T, desc.n_neurons
    dev = inp.device
    spikes_in = W is not None
    f32 = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)
    # With BF16 GEMMs the detached block backward keeps dL/dI as bfloat16 in its
    # workspace for dW and dx when no float copy is asked for (the GEMMs round it so).
    gi16 = (spikes_in and not want_grad_current and (want_grad_W or want_grad_input) and
            desc.gemm_precision == L.GEMM_BF16 and desc.algo == L.ALGO_BLOCKS and
            desc.grad_policy != L.GRAD_ATTACHED and grad_v is None and grad_theta is None and N % 8 == 0)
    g_cur = f32(B, T, N) if (want_grad_current or want_grad_W or want_grad_input) and not gi16 else None
    g_in = f32(B, T, desc.n_in) if (spikes_in and want_grad_input) else None
    g_W = f32(N, desc.n_in) if (spikes_in and want_grad_W) else None
    pg = {k: f32(N) for k in ("bias", "tau_mem", "tau_adapt", "d", "theta0")} if want_param_grads else {}
    if workspace is None and not noalloc:
        workspace = torch.empty(max(1, backward_workspace_bytes(desc)), dtype=torch.uint8, device=dev)
    cp = params.c()
    for g in (grad_spikes, grad_v, grad_theta):
        if g is not None:
            assert g.dtype == torch.float32 and g.is_contiguous() and g.shape == (B, T, N)
    args = [ctypes.byref(desc), ctypes.byref(cp), _p(inp), _p(W), _p(fwd["current"]), _p(fwd["carries"]),
            _p(grad_spikes), _p(grad_v), _p(grad_theta), _p(g_cur), _p(g_in), _p(g_W), _p(pg.get("bias")),
            _p(pg.get("tau_mem")), _p(pg.get("tau_adapt")), _p(pg.get("d")), _p(pg.get("theta0"))]
    if noalloc:
        L.check(L.load().alif_backward_noalloc(*args, _stream(dev)))
    else:
        L.check(L.load().alif_backward(*args, _p(workspace), _stream(dev)))
    out = {"grad_current": g_cur, "grad_input": g_in if spikes_in else g_cur, "grad_W": g_W}
    out.update({"grad_" + k: v for k, v in pg.items()})
    return out


def forward_recurrent(inp: torch.Tensor, params: Params, dt: float, arp: float, W_rec: torch.Tensor,
                      W: torch.Tensor | None = None, *, gemm_precision=L.GEMM_FP32, spike_dtype=L.SPIKES_U8,
                      want_v=False, want_theta=False, save=True, slope=10.0, surrogate=L.SG_FAST_SIGMOID,
                      delay=0, workspace=None) -> dict:
    """One recurrent ALIF layer (alif_forward_recurrent): Eq. 3 with the recurrent
    current W_rec S[t - D], D = ``delay`` steps (0: T_R). ``inp`` as in ``forward``. Returns ``spikes``,
    optional ``v``/``theta``, ``current`` (the whole current, which the backward
    differentiates), ``carries``, ``desc`` and the ``workspace`` (reusable by
    ``recurrent_weight_grad``)."""
    assert inp.is_cuda and inp.is_contiguous() and W_rec.dtype == torch.float32 and W_rec.is_contiguous()
    B, T = inp.shape[0], inp.shape[1]
    dev = inp.device
    if W is None:
        assert inp.dtype == torch.float32
        N, n_in, kind = inp.shape[2], 0, L.INPUT_CURRENT_F32
    else:
        assert W.dtype == torch.float32 and W.is_contiguous()
        N, n_in = W.shape
        kind = _INPUT_KIND[inp.dtype]
    assert W_rec.shape == (N, N)
    desc = make_desc(B, T, N, dt, arp, n_in, kind, gemm_precision, spike_dtype, L.ALGO_BLOCKS, slope, surrogate)
    spikes = torch.empty(B, T, N, dtype=_SPIKE_TORCH[spike_dtype], device=dev)
    v = torch.empty(B, T, N, dtype=torch.float32, device=dev) if want_v else None
    th = torch.empty(B, T, N, dtype=torch.float32, device=dev) if want_theta else None
    current = torch.empty(B, T, N, dtype=torch.float32, device=dev)
    carries = torch.empty(max(1, carry_bytes(desc)), dtype=torch.uint8, device=dev) if save else None
    if workspace is None:
        n = ctypes.c_size_t()
        L.check(L.load().alif_recurrent_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
        workspace = torch.empty(max(1, n.value), dtype=torch.uint8, device=dev)
    cp = params.c()
    L.check(L.load().alif_forward_recurrent(ctypes.byref(desc), ctypes.byref(cp), _p(inp), _p(W), _p(W_rec),
                                            int(delay), _p(current), _p(spikes), _p(v), _p(th), _p(carries),
                                            _p(workspace), _stream(dev)))
    return {"spikes": spikes, "v": v, "theta": th, "current": current, "carries": carries, "desc": desc,
            "workspace": workspace, "recurrent": True, "current_input": W is None, "delay": int(delay)}


def recurrent_weight_grad(fwd: dict, grad_current: torch.Tensor) -> torch.Tensor:
    """grad_W_rec [N][N] = sum_{b,t} grad_current[b][t]^T S[b][t - D] (alif_recurrent_weight_grad)."""
    desc = fwd["desc"]
    N = desc.n_neurons
    out = torch.empty(N, N, dtype=torch.float32, device=grad_current.device)
    L.check(L.load().alif_recurrent_weight_grad(ctypes.byref(desc), fwd["delay"], _p(grad_current.contiguous()),
                                                _p(fwd["spikes"]), _p(out), _p(fwd["workspace"]),
                                                _stream(grad_current.device)))
    return out


def backward_recurrent(fwd: dict, inp: torch.Tensor, params: Params, W: torch.Tensor | None = None, **kw) -> dict:
    """Backward of ``forward_recurrent`` under the detached policy: the ordinary
    layer backward on the whole current (the recurrent input is a constant of the
    spike path), plus ``grad_W_rec``. Keyword arguments as ``backward``."""
    kw = dict(kw)
    kw["want_grad_current"] = True
    if fwd["current_input"]:
        f = dict(fwd, current=None)
        out = backward(f, fwd["current"], params, None, **kw)
    else:
        out = backward(fwd, inp, params, W, **kw)
    out["grad_W_rec"] = recurrent_weight_grad(fwd, out["grad_current"])
    return out


def decay_tables(params: Params, N, dt, arp):
    desc = make_desc(1, 1, N, dt, arp)
    TR = refractory_steps(dt, arp)
    bp = torch.empty(N, TR + 1, dtype=torch.float32, device=params.tau_mem.device)
    pp = torch.empty_like(bp)
    cp = params.c()
    L.check(L.load().alif_decay_tables(ctypes.byref(desc), ctypes.byref(cp), _p(bp), _p(pp),
                                       _stream(bp.device)))
    return bp, pp


def input_current(x: torch.Tensor, W: torch.Tensor, bias=None, gemm_precision=L.GEMM_FP32):
    B, T, n_in = x.shape
    N = W.shape[0]
    desc = make_desc(B, T, N, 1.0, 2.0, n_in, _INPUT_KIND[x.dtype], gemm_precision)
    out = torch.empty(B, T, N, dtype=torch.float32, device=x.device)
    L.check(L.load().alif_input_current(ctypes.byref(desc), _p(x), _p(W), _p(bias), _p(out),
                                        _stream(x.device)))
    return out


def transpose(m: torch.Tensor) -> torch.Tensor:
    """float32 [rows][cols] -> [cols][rows] on the device (alif_transpose)."""
    assert m.dtype == torch.float32 and m.is_contiguous() and m.dim() == 2
    out = torch.empty(m.shape[1], m.shape[0], dtype=torch.float32, device=m.device)
    L.check(L.load().alif_transpose(m.shape[0], m.shape[1], _p(m), _p(out), _stream(m.device)))
    return out


def input_current_events(x: torch.Tensor, WT: torch.Tensor, bias=None, out=None):
    """Eq. 3's current from the active inputs only (alif_input_current_events):
    x spikes [B][T][n_in] (uint8, bfloat16 or float32), WT = W transposed [n_in][N]."""
    assert x.is_contiguous() and WT.dtype == torch.float32 and WT.is_contiguous()
    B, T, n_in = x.shape
    N = WT.shape[1]
    assert WT.shape[0] == n_in
    desc = make_desc(B, T, N, 1.0, 2.0, n_in, _INPUT_KIND[x.dtype])
    cur = out if out is not None else torch.empty(B, T, N, dtype=torch.float32, device=x.device)
    L.check(L.load().alif_input_current_events(ctypes.byref(desc), _p(x), _p(WT), _p(bias), _p(cur),
                                               _stream(x.device)))
    return cur


def weight_grad(grad_current: torch.Tensor, x: torch.Tensor, gemm_precision=L.GEMM_FP32, workspace=None):
    """grad_W [N][n_in] = sum_{b,t} grad_current[b][t][:]^T x[b][t][:] (alif_weight_grad)."""
    B, T, n_in = x.shape
    N = grad_current.shape[2]
    desc = make_desc(B, T, N, 1.0, 2.0, n_in, _INPUT_KIND[x.dtype], gemm_precision)
    if workspace is None:
        n = ctypes.c_size_t()
        L.check(L.load().alif_weight_grad_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
        workspace = torch.empty(max(1, n.value), dtype=torch.uint8, device=x.device)
    out = torch.empty(N, n_in, dtype=torch.float32, device=x.device)
    L.check(L.load().alif_weight_grad(ctypes.byref(desc), _p(grad_current), _p(x), _p(out), _p(workspace),
                                      _stream(x.device)))
    return out


def input_grad(grad_current: torch.Tensor, W: torch.Tensor, input_kind=L.INPUT_SPIKES_U8,
               gemm_precision=L.GEMM_FP32):
    """grad_input [B][T][n_in] = grad_current[b][t][:] W (alif_input_grad)."""
    B, T, N = grad_current.shape
    n_in = W.shape[1]
    desc = make_desc(B, T, N, 1.0, 2.0, n_in, input_kind, gemm_precision)
    out = torch.empty(B, T, n_in, dtype=torch.float32, device=W.device)
    L.check(L.load().alif_input_grad(ctypes.byref(desc), _p(grad_current), _p(W), _p(out),
                                     _stream(W.device)))
    return out


def device_status(device=None) -> int:
    bits = ctypes.c_uint32()
    L.check(L.load().alif_device_status(ctypes.byref(bits), _stream(device)))
    return bits.value


# ---------------------------------------------------------------------------
# readout
# ---------------------------------------------------------------------------

def readout_workspace(B, T, H, C, device):
    n = ctypes.c_size_t()
    L.check(L.load().alif_readout_workspace_bytes(B, T, H, C, ctypes.byref(n)))
    return torch.empty(max(1, n.value), dtype=torch.uint8, device=device)


_SPIKE_CODE = {torch.uint8: L.SPIKES_U8, torch.bfloat16: L.SPIKES_BF16, torch.float32: L.SPIKES_F32}


def readout_forward(spikes, W_r, tau_r, dt, workspace=None):
    B, T, H = spikes.shape
    C = W_r.shape[0]
    ws = workspace if workspace is not None else readout_workspace(B, T, H, C, spikes.device)
    o = torch.empty(B, C, dtype=torch.float32, device=spikes.device)
    L.check(L.load().alif_readout_forward(B, T, H, C, float(dt), _SPIKE_CODE[spikes.dtype], _p(spikes),
                                          _p(W_r), _p(tau_r), _p(o), _p(ws), _stream(spikes.device)))
    return o, ws


def readout_backward(spikes, W_r, tau_r, dt, go, workspace):
    B, T, H = spikes.shape
    C = W_r.shape[0]
    dev = spikes.device
    gS = torch.empty(B, T, H, dtype=torch.float32, device=dev)
    gW = torch.empty(C, H, dtype=torch.float32, device=dev)
    gt = torch.empty(C, dtype=torch.float32, device=dev)
    L.check(L.load().alif_readout_backward(B, T, H, C, float(dt), _SPIKE_CODE[spikes.dtype], _p(spikes),
                                           _p(W_r), _p(tau_r), _p(go.contiguous()), _p(gS), _p(gW), _p(gt),
                                           _p(workspace), _stream(dev)))
    return gS, gW, gt


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

class BlockALIF(torch.autograd.Function):
    """One ALIF layer as an autograd op.

    apply(inp, W, tau_mem, tau_adapt, d, theta0, bias, cfg) -> (spikes, v, theta)
    ``inp``: current [B][T][N] (W None) or spikes [B][T][n_in]. Spikes come back in
    float32 (or bfloat16 with cfg['spike_dtype'] = SPIKES_BF16) so that they carry
    gradient; v/theta are empty tensors unless cfg['traces'] is true."""

    @staticmethod
    def forward(ctx, inp, W, tau_mem, tau_adapt, d, theta0, bias, cfg):
        prm = Params(tau_mem.contiguous(), tau_adapt.contiguous(), d.contiguous(), theta0.contiguous(),
                     None if bias is None else bias.contiguous())
        traces = cfg.get("traces", False)
        # the kernels read dense [B][T][*] rows: the forward and the backward both get the same contiguous copy
        x = inp.contiguous()
        Wc = None if W is None else W.contiguous()
        f = forward(x, prm, cfg["dt"], cfg["arp"], Wc, gemm_precision=cfg.get("gemm", L.GEMM_FP32),
                    spike_dtype=cfg.get("spike_dtype", L.SPIKES_F32), algo=cfg.get("algo", L.ALGO_BLOCKS),
                    want_v=traces, want_theta=traces, save=True, slope=cfg.get("slope", 10.0),
                    surrogate=cfg.get("surrogate", L.SG_FAST_SIGMOID))
        ctx.cfg = cfg
        ctx.fwd = {k: f[k] for k in ("current", "carries", "desc")}
        ctx.prm = prm
        ctx.has_bias = bias is not None
        ctx.save_for_backward(x, Wc)
        empty = inp.new_empty(0, dtype=torch.float32)
        return f["spikes"], (f["v"] if traces else empty), (f["theta"] if traces else empty)

    @staticmethod
    def backward(ctx, g_s, g_v, g_th):
        inp, W = ctx.saved_tensors
        cfg = ctx.cfg
        gs = None if g_s is None else g_s.float().contiguous()
        gv = g_v.contiguous() if (g_v is not None and g_v.numel() > 0) else None
        gt = g_th.contiguous() if (g_th is not None and g_th.numel() > 0) else None
        need_in = ctx.needs_input_grad[0]
        need_W = W is not None and ctx.needs_input_grad[1]
        g = backward(ctx.fwd, inp, ctx.prm, W, grad_spikes=gs, grad_v=gv, grad_theta=gt,
                     want_grad_input=need_in, want_grad_W=need_W)
        g_inp = g["grad_input"] if need_in else None
        if g_inp is not None and W is not None and inp.dtype != torch.float32:
            g_inp = g_inp.to(inp.dtype)
        return (g_inp, g["grad_W"] if need_W else None, g["grad_tau_mem"], g["grad_tau_adapt"], g["grad_d"],
                g["grad_theta0"], g["grad_bias"] if ctx.has_bias else None, None)


class Readout(torch.autograd.Function):
    """Leaky readout o[b][c] = sum_t V_r (supplementary "Readout neurons")."""

    @staticmethod
    def forward(ctx, spikes, W_r, tau_r, dt):
        s = spikes.contiguous()
        o, ws = readout_forward(s, W_r.contiguous(), tau_r.contiguous(), dt)
        ctx.save_for_backward(s, W_r, tau_r)
        ctx.ws = ws
        ctx.dt = dt
        return o

    @staticmethod
    def backward(ctx, go):
        s, W_r, tau_r = ctx.saved_tensors
        gS, gW, gt = readout_backward(s, W_r.contiguous(), tau_r.contiguous(), ctx.dt, go.float(), ctx.ws)
        return (gS.to(s.dtype) if ctx.needs_input_grad[0] else None, gW, gt, None)


def ou_current(T: int, N: int, dt: float, tau: float, mean: float, sd: float, seed: int,
               device="cuda", out: torch.Tensor | None = None) -> torch.Tensor:
    """float32 [T][N] Ornstein-Uhlenbeck current drawn on the device by the library
    (Philox4x32-10 + Box-Muller, FP64 recurrence; the definition is in the header)."""
    lib = L.load()
    ws_b = ctypes.c_size_t()
    L.check(lib.alif_ou_workspace_bytes(T, N, ctypes.byref(ws_b)))
    if out is None:
        out = torch.empty((T, N), dtype=torch.float32, device=device)
    assert out.shape == (T, N) and out.dtype == torch.float32 and out.is_contiguous()
    ws = torch.empty(max(ws_b.value, 1), dtype=torch.uint8, device=out.device)
    L.check(lib.alif_ou_current(T, N, dt, tau, mean, sd, seed, _p(out), _p(ws), ws_b.value,
                                _stream(out.device)))
    return out


# ---------------------------------------------------------------------------
# neural fits: van Rossum loss and Adam
# ---------------------------------------------------------------------------

def van_rossum_workspace(B, R, T, N, device):
    n = ctypes.c_size_t()
    L.check(L.load().alif_van_rossum_workspace_bytes(B, R, T, N, ctypes.byref(n)))
    return torch.empty(max(1, n.value), dtype=torch.uint8, device=device)


def van_rossum(spikes: torch.Tensor, targets: torch.Tensor, dt: float, tau: float = 100.0, *,
               scale: float = 1.0, want_dist: bool = True, want_grad: bool = True,
               dist=None, grad=None, workspace=None):
    """Van Rossum distance of uint8 spikes [B][T][N] against uint8 targets [B][R][T][N]
    (or [B][T][N] for R = 1). Returns (dist [B][R][N] or None,
    grad [B][T][N] = scale * sum_r dD/dspikes or None, workspace)."""
    if targets.dim() == 3:
        targets = targets.unsqueeze(1)
    B, T, N = spikes.shape
    R = targets.shape[1]
    assert spikes.dtype == torch.uint8 and targets.dtype == torch.uint8
    assert targets.shape == (B, R, T, N) and spikes.is_contiguous() and targets.is_contiguous()
    dev = spikes.device
    ws = workspace if workspace is not None else van_rossum_workspace(B, R, T, N, dev)
    if want_dist and dist is None:
        dist = torch.empty(B, R, N, dtype=torch.float32, device=dev)
    if want_grad and grad is None:
        grad = torch.empty(B, T, N, dtype=torch.float32, device=dev)
    L.check(L.load().alif_van_rossum(B, R, T, N, float(dt), float(tau), _p(spikes), _p(targets), float(scale),
                                     _p(dist) if want_dist else None, _p(grad) if want_grad else None,
                                     _p(ws), _stream(dev)))
    return (dist if want_dist else None), (grad if want_grad else None), ws


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
              beta1=0.9, beta2=0.999, eps=1e-8, lo=float("-inf"), hi=float("inf")):
    """One in-place Adam step on float32 ``param`` (Kingma and Ba), clamped to [lo, hi]."""
    for t in (param, grad, m, v):
        assert t.dtype == torch.float32 and t.is_contiguous() and t.numel() == param.numel()
    L.check(L.load().alif_adam_step(param.numel(), _p(param), _p(grad), _p(m), _p(v), int(step), float(lr),
                                    float(beta1), float(beta2), float(eps), float(lo), float(hi),
                                    _stream(param.device)))
