"""Parity helpers: compare GPU results with the FP64 oracle.

Spike trains must be identical except at crossings whose oracle margin
|V - theta| is below MARGIN (1e-6). Such a flip is "excused": the oracle is
re-run with that decision imposed (teacher forcing), so the trajectories stay
comparable afterwards, and the excused flips are counted. Any other mismatch
fails. Traces are then compared on the teacher-forced oracle run.
"""
from __future__ import annotations

import numpy as np

import oracle

MARGIN = 1e-6      # crossings this close to threshold may differ (FP32 vs FP64)
TRACE_TOL = 1e-4   # |V_gpu - V_oracle|, |theta_gpu - theta_oracle|
GRAD_TOL = 1e-4    # relative L2 and elementwise (scaled by max |g|) gradient error


class ParityError(AssertionError):
    pass


def teacher_forced_forward(gpu_S, I, tau_m, tau_a, d, theta0, dt, arp, max_iter=200):
    """Run the oracle on current I[B][T][N]; impose the GPU's decision at each first
    mismatch of a row whose oracle margin is below MARGIN; raise on any other.

    Returns (oracle result dict, number of excused flips)."""
    gpu_S = np.asarray(gpu_S).astype(np.uint8)
    B, T, N = gpu_S.shape
    force = np.full((B, T, N), -1, np.int8)
    excused = 0
    for _ in range(max_iter):
        orc = oracle.alif_forward(I, tau_m, tau_a, d, theta0, dt, arp, force=force)
        mism = gpu_S != orc["S"]
        if not mism.any():
            return orc, excused
        # first mismatch per (b, n) row
        b_idx, n_idx = np.nonzero(mism.any(axis=1))
        first_t = np.argmax(mism[b_idx, :, n_idx], axis=1)
        margin = orc["V"][b_idx, first_t, n_idx] - orc["TH"][b_idx, first_t, n_idx]
        bad = np.abs(margin) >= MARGIN
        if bad.any():
            k = int(np.flatnonzero(bad)[0])
            raise ParityError(
                f"spike mismatch at b={b_idx[k]} t={first_t[k]} n={n_idx[k]}: gpu={gpu_S[b_idx[k], first_t[k], n_idx[k]]} "
                f"oracle={orc['S'][b_idx[k], first_t[k], n_idx[k]]} margin={margin[k]:.3e} "
                f"({int(bad.sum())} rows with a non-excusable first mismatch)")
        force[b_idx, first_t, n_idx] = gpu_S[b_idx, first_t, n_idx]
        excused += len(b_idx)
    raise ParityError("teacher forcing did not converge")


def teacher_forced_recurrent(gpu_S, Iff, W_rec, tau_m, tau_a, d, theta0, dt, arp, max_iter=200, D=None):
    """The recurrent oracle on Iff[B][T][N] (bias + feedforward current), with the
    GPU's decisions imposed where they differ from the oracle's within MARGIN of
    threshold. Neurons of one batch element are coupled through W_rec, so each
    round imposes the mismatches at the earliest differing step of every batch
    element and re-runs; a mismatch there with a larger margin fails.

    Returns (oracle result dict, number of excused flips)."""
    gpu_S = np.asarray(gpu_S).astype(np.uint8)
    B, T, N = gpu_S.shape
    force = np.full((B, T, N), -1, np.int8)
    excused = 0
    for _ in range(max_iter):
        orc = oracle.alif_forward_recurrent(Iff, W_rec, tau_m, tau_a, d, theta0, dt, arp, force=force, D=D)
        mism = gpu_S != orc["S"]
        if not mism.any():
            return orc, excused
        for b in np.flatnonzero(mism.any(axis=(1, 2))):
            t = int(np.argmax(mism[b].any(axis=1)))
            ns = np.flatnonzero(mism[b, t])
            margin = orc["V"][b, t, ns] - orc["TH"][b, t, ns]
            if (np.abs(margin) >= MARGIN).any():
                k = int(ns[np.argmax(np.abs(margin) >= MARGIN)])
                raise ParityError(f"recurrent spike mismatch at b={b} t={t} n={k}: gpu={gpu_S[b, t, k]} "
                                  f"oracle={orc['S'][b, t, k]} margin={orc['V'][b, t, k] - orc['TH'][b, t, k]:.3e}")
            force[b, t, ns] = gpu_S[b, t, ns]
            excused += len(ns)
    raise ParityError("teacher forcing did not converge")


def check_forward(gpu, I, prm, dt, arp, v_gpu=None, th_gpu=None):
    """Full forward parity. ``prm`` has numpy tau_mem, tau_adapt, d, theta0 (and bias)
    [N]; I is the current before bias. Returns a report dict."""
    I64 = np.asarray(I, np.float64)
    if getattr(prm, "bias", None) is not None:
        I64 = I64 + np.asarray(prm.bias, np.float64)[None, None, :]
    orc, excused = teacher_forced_forward(gpu, I64, prm.tau_mem, prm.tau_adapt, prm.d, prm.theta0, dt, arp)
    rep = {"excused": excused, "n_spikes": int(orc["S"].sum()), "oracle": orc}
    if v_gpu is not None:
        dv = np.abs(np.asarray(v_gpu, np.float64) - orc["V"])
        rep["max_dV"] = float(dv.max()) if dv.size else 0.0
        if rep["max_dV"] > TRACE_TOL:
            raise ParityError(f"membrane trace error {rep['max_dV']:.3e} > {TRACE_TOL}")
    if th_gpu is not None:
        dt_ = np.abs(np.asarray(th_gpu, np.float64) - orc["TH"])
        rep["max_dTH"] = float(dt_.max()) if dt_.size else 0.0
        if rep["max_dTH"] > TRACE_TOL:
            raise ParityError(f"threshold trace error {rep['max_dTH']:.3e} > {TRACE_TOL}")
    return rep


def check_grad(name, g_gpu, g_orc, tol=GRAD_TOL):
    g_gpu = np.asarray(g_gpu, np.float64)
    g_orc = np.asarray(g_orc, np.float64)
    assert g_gpu.shape == g_orc.shape, (name, g_gpu.shape, g_orc.shape)
    scale = float(np.abs(g_orc).max()) if g_orc.size else 0.0
    if scale == 0.0:
        err = float(np.abs(g_gpu).max()) if g_gpu.size else 0.0
        if err > 1e-12:
            raise ParityError(f"{name}: oracle gradient is zero, gpu max |g| = {err:.3e}")
        return {"rel_l2": 0.0, "max_rel": 0.0}
    rel_l2 = float(np.linalg.norm(g_gpu - g_orc) / np.linalg.norm(g_orc))
    max_rel = float(np.abs(g_gpu - g_orc).max() / scale)
    if rel_l2 > tol or max_rel > tol:
        raise ParityError(f"{name}: rel L2 {rel_l2:.3e}, max elementwise {max_rel:.3e} (tol {tol})")
    return {"rel_l2": rel_l2, "max_rel": max_rel}


def coincidence(S_a, S_b, window=1):
    """Greedy one-to-one matching of spikes within +-window steps, per (b, n) row;
    returns 2 * matches / (n_a + n_b) (1.0 when both are empty)."""
    S_a = np.asarray(S_a).astype(bool)
    S_b = np.asarray(S_b).astype(bool)
    B, T, N = S_a.shape
    match = 0
    na, nb = int(S_a.sum()), int(S_b.sum())
    if na + nb == 0:
        return 1.0
    for b in range(B):
        for n in range(N):
            ta = np.flatnonzero(S_a[b, :, n])
            tb = np.flatnonzero(S_b[b, :, n])
            i = j = 0
            while i < len(ta) and j < len(tb):
                if abs(int(ta[i]) - int(tb[j])) <= window:
                    match += 1
                    i += 1
                    j += 1
                elif ta[i] < tb[j]:
                    i += 1
                else:
                    j += 1
    return 2.0 * match / (na + nb)
