"""Python binding of the library's serving calls (alif_server_create, alif_submit,
alif_poll, alif_server_destroy): continuous batching of independent single-layer
ALIF forward simulations. Argument marshalling only; scheduling, admission and
all compute run in the library."""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass

import numpy as np

from . import _lib as L


@dataclass
class Request:
    """One simulation: per-neuron float parameters (numpy [N]) and either a host
    current [T][N] (float32) or an on-device Ornstein-Uhlenbeck current."""
    T: int
    dt: float
    arp: float
    tau_mem: np.ndarray
    tau_adapt: np.ndarray
    d: np.ndarray
    theta0: np.ndarray
    bias: np.ndarray | None = None
    current: np.ndarray | None = None      # host [T][N] float32; None -> OU
    ou_tau: float = 5.0
    ou_mean: float = 0.8
    ou_sd: float = 0.5
    seed: int = 0
    want_spikes: bool = True        # dense uint8 [T][N] raster
    events_capacity: int = 0        # > 0: also the spikes as flat indices t * N + n

    @property
    def N(self) -> int:
        return int(np.asarray(self.tau_mem).shape[0])


@dataclass
class Result:
    status: int
    n_spikes: int
    spikes: np.ndarray | None     # uint8 [T][N]
    events: np.ndarray | None     # uint32 flat indices t * N + n, ascending
    events_truncated: bool
    t_submit: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def c_request(r: Request):
    """The C struct for ``r`` and the host arrays it points to (keep them alive)."""
    N = r.N
    arrs = {k: _f32(getattr(r, k)) for k in ("tau_mem", "tau_adapt", "d", "theta0", "bias")}
    for k, a in arrs.items():
        if a is not None and a.shape != (N,):
            raise ValueError(f"{k} must have shape ({N},)")
    cur = None
    if r.current is not None:
        cur = _f32(r.current)
        if cur.shape != (r.T, N):
            raise ValueError(f"current must have shape ({r.T}, {N})")
    spk = np.empty((r.T, N), dtype=np.uint8) if r.want_spikes else None
    ev = np.empty(int(r.events_capacity), dtype=np.uint32) if r.events_capacity > 0 else None

    def ptr(a):
        return None if a is None else a.ctypes.data

    c = L.AlifRequest(n_neurons=N, T=r.T, dt_ms=r.dt, arp_ms=r.arp,
                      tau_mem_ms=ptr(arrs["tau_mem"]), tau_adapt_ms=ptr(arrs["tau_adapt"]),
                      d=ptr(arrs["d"]), theta0=ptr(arrs["theta0"]), bias=ptr(arrs["bias"]),
                      input=L.REQ_HOST_CURRENT if cur is not None else L.REQ_OU,
                      host_current=ptr(cur), ou_tau_ms=r.ou_tau, ou_mean=r.ou_mean,
                      ou_sd=r.ou_sd, seed=r.seed & (2**64 - 1), host_spikes=ptr(spk),
                      host_events=ptr(ev), events_capacity=int(r.events_capacity))
    return c, (arrs, cur, spk, ev)


def footprint(r: Request) -> int:
    """Device bytes the request holds while admitted (no device needed)."""
    c, _ = c_request(r)
    b = ctypes.c_size_t()
    L.check(L.load().alif_request_footprint(ctypes.byref(c), ctypes.byref(b)))
    return b.value


class Server:
    """A serving instance on one device. ``budget_bytes`` bounds the device memory
    of the admitted requests; ``max_slots`` bounds how many run at once."""

    def __init__(self, budget_bytes: int, max_slots: int = 8, device: int = 0):
        self._lib = L.load()
        h = ctypes.c_void_p()
        L.check(self._lib.alif_server_create(budget_bytes, max_slots, device, ctypes.byref(h)))
        self._h = h
        self._keep = {}   # ticket -> host arrays the library still reads or writes

    def submit(self, r: Request) -> int:
        c, keep = c_request(r)
        t = ctypes.c_uint64()
        L.check(self._lib.alif_submit(self._h, ctypes.byref(c), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def poll(self, ticket: int) -> Result | None:
        res = L.AlifResult()
        rc = L.check(self._lib.alif_poll(self._h, ticket, ctypes.byref(res)))
        if rc == L.ALIF_PENDING:
            return None
        keep = self._keep.pop(ticket, None)
        spk, ev = (keep[2], keep[3]) if keep is not None else (None, None)
        if ev is not None:
            ev = ev[:min(res.n_spikes, ev.shape[0])]
        return Result(res.status, res.n_spikes, spk, ev, bool(res.events_truncated), res.t_submit_s,
                      res.t_admit_s, res.t_done_s)

    def wait(self, ticket: int, timeout: float = 60.0, interval: float = 1e-4) -> Result:
        end = time.monotonic() + timeout
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() > end:
                raise TimeoutError(f"request {ticket} not done after {timeout} s")
            time.sleep(interval)

    def close(self):
        if self._h is not None:
            L.check(self._lib.alif_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
