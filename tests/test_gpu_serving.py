"""Serving (continuous batching) on the GPU: the on-device OU current against the
oracle's own generator, served results against alif_forward and the FP64 oracle,
each result the same alone and in a mix of concurrent requests, admission within
the HBM budget, and the ticket / budget errors."""
import time

import numpy as np
import pytest

from oracle import ou_philox
from paper_2311_11390_amd import _lib as L
from paper_2311_11390_amd.synth import REQUEST_OU, request_params, request_stream
from gpu_helpers import driven_current, log, random_params
from parity import check_forward

pytestmark = pytest.mark.gpu


def _ulp_diff(a32, b32):
    a = np.asarray(a32, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b32, np.float32).view(np.int32).astype(np.int64)
    a = np.where(a < 0, -(a & 0x7FFFFFFF), a)
    b = np.where(b < 0, -(b & 0x7FFFFFFF), b)
    return np.abs(a - b)


@pytest.mark.parametrize("T,N", [(1, 1), (3, 5), (257, 64), (1000, 100), (2050, 130)])
def test_ou_current_matches_oracle_generator(T, N):
    import torch

    from paper_2311_11390_amd import alif
    log(f"ou_current T={T} N={N}")
    seed = 0x1234_5678_9ABC + T
    dev = alif.ou_current(T, N, 0.05, 5.0, 0.8, 0.5, seed)
    torch.cuda.synchronize()
    got = dev.cpu().numpy()
    want, want64 = ou_philox.ou_current(T, N, 0.05, 5.0, 0.8, 0.5, seed)
    ulp = _ulp_diff(got, want)
    # the device evaluates the same FP64 recurrence in chunks with fused
    # multiply-adds and its own libm: the float results may differ by one ulp
    # where the FP64 value sits next to a rounding boundary
    assert ulp.max() <= 1, ulp.max()
    assert (ulp > 0).mean() < 1e-3
    assert np.abs(got - want64).max() < 1e-6


def _params(N, seed):
    return random_params(seed, N, tm=(10.0, 30.0), ta=(100.0, 300.0), d=(0.0, 1.8), th=(0.9, 1.1))


def _req(prm, T, dt, arp=2.0, current=None, seed=0, events=0, raster=True):
    from paper_2311_11390_amd.serving import Request
    return Request(T=T, dt=dt, arp=arp, tau_mem=prm.tau_mem, tau_adapt=prm.tau_adapt, d=prm.d,
                   theta0=prm.theta0, bias=prm.bias, current=current, seed=seed, want_spikes=raster,
                   events_capacity=events, **{"ou_" + k: v for k, v in REQUEST_OU.items()})


def _forward_spikes(I, prm, dt, arp=2.0):
    import torch

    from gpu_helpers import gpu_forward
    f, _, _ = gpu_forward(I[None], prm, dt, arp, traces=False)
    torch.cuda.synchronize()
    return f["spikes"][0].cpu().numpy()


def test_served_host_current_matches_forward_and_oracle():
    from paper_2311_11390_amd.serving import Server
    T, N, dt = 1203, 150, 0.1
    prm = _params(N, 5)
    I = driven_current(5, 1, T, N)[0]
    log(f"serve host current T={T} N={N} dt={dt}")
    with Server(1 << 30, max_slots=2) as srv:
        r = srv.wait(srv.submit(_req(prm, T, dt, current=I)))
    assert r.status == L.ALIF_OK
    np.testing.assert_array_equal(r.spikes, _forward_spikes(I, prm, dt))
    assert r.n_spikes == int(r.spikes.sum()) > 0
    rep = check_forward(r.spikes[None], I[None], prm, dt, 2.0)
    log(f"  spikes={rep['n_spikes']} excused={rep['excused']}")
    assert r.t_submit <= r.t_admit <= r.t_done


def test_served_ou_matches_forward_and_oracle():
    from paper_2311_11390_amd import alif
    from paper_2311_11390_amd.serving import Server
    T, N, dt, seed = 3001, 96, 0.05, 987654321
    prm = _params(N, 6)
    log(f"serve OU T={T} N={N} dt={dt}")
    with Server(1 << 30, max_slots=2) as srv:
        r = srv.wait(srv.submit(_req(prm, T, dt, seed=seed)))
    assert r.status == L.ALIF_OK
    Idev = alif.ou_current(T, N, dt, REQUEST_OU["tau"], REQUEST_OU["mean"], REQUEST_OU["sd"], seed)
    np.testing.assert_array_equal(r.spikes, _forward_spikes(Idev.cpu().numpy(), prm, dt))
    # the oracle on the oracle's own OU current (float32 as the device rounds it)
    I_or, _ = ou_philox.ou_current(T, N, dt, REQUEST_OU["tau"], REQUEST_OU["mean"], REQUEST_OU["sd"], seed)
    rep = check_forward(r.spikes[None], I_or[None], prm, dt, 2.0)
    log(f"  spikes={rep['n_spikes']} excused={rep['excused']}")
    assert rep["n_spikes"] > 0


def _mix(n=14, seed=3):
    reqs = request_stream(seed=seed, n=n, n_range=(40, 700), t_range=(1, 6000))
    return [(q, request_params(q)) for q in reqs]


def _run(srv, mix, stagger=0.0, events=0):
    tickets = []
    for q, prm in mix:
        tickets.append(srv.submit(_req(prm, q.T, q.dt, seed=q.seed, events=events)))
        if stagger:
            time.sleep(stagger)
    return [srv.wait(t, timeout=120) for t in tickets]


def test_each_result_is_the_same_alone_and_in_the_mix():
    from paper_2311_11390_amd import serving
    from paper_2311_11390_amd.serving import Server
    mix = _mix()
    log(f"mix of {len(mix)}: " + ", ".join(f"N={q.N} T={q.T} dt={q.dt}" for q, _ in mix))
    fps = [serving.footprint(_req(prm, q.T, q.dt, seed=q.seed)) for q, prm in mix]
    budget = int(sum(sorted(fps)[-3:]) * 1.01)      # about three of the largest at once
    # all submitted at once: the budget admits about three at a time, the rest
    # are admitted as earlier requests complete
    with Server(budget, max_slots=6) as srv:
        mixed = _run(srv, mix, events=1 << 20)
    alone = []
    for (q, prm) in mix:
        with Server(1 << 31, max_slots=1) as srv:
            alone.append(_run(srv, [(q, prm)])[0])
    for (q, _), a, m in zip(mix, alone, mixed):
        assert a.status == m.status == L.ALIF_OK
        np.testing.assert_array_equal(a.spikes, m.spikes)
        assert a.n_spikes == m.n_spikes == int(a.spikes.sum())
        # the event list is the raster's nonzeros in ascending flat order
        assert not m.events_truncated
        np.testing.assert_array_equal(m.events, np.flatnonzero(a.spikes.ravel()).astype(np.uint32))
    # admission in arrival order, never more than the budget resident, and the
    # work of different requests overlapped
    admits = [m.t_admit for m in mixed]
    assert admits == sorted(admits)
    for i, m in enumerate(mixed):
        resident = sum(fps[j] for j, o in enumerate(mixed) if o.t_admit <= m.t_admit < o.t_done)
        assert resident <= budget
    overlap = sum(1 for i, a in enumerate(mixed) for b in mixed[i + 1:]
                  if a.t_admit < b.t_done and b.t_admit < a.t_done)
    late = sum(1 for m in mixed if m.t_admit > min(o.t_done for o in mixed))
    log(f"  overlapping pairs: {overlap}, admitted after a completion: {late}")
    assert overlap > 0 and late > 0


def test_served_mix_matches_the_oracle():
    from paper_2311_11390_amd.serving import Server
    mix = _mix(n=5, seed=8)
    with Server(1 << 31, max_slots=4) as srv:
        res = _run(srv, mix)
    for (q, prm), r in zip(mix, res):
        log(f"oracle check N={q.N} T={q.T} dt={q.dt}")
        I_or, _ = ou_philox.ou_current(q.T, q.N, q.dt, REQUEST_OU["tau"], REQUEST_OU["mean"],
                                       REQUEST_OU["sd"], q.seed)
        check_forward(r.spikes[None], I_or[None], prm, q.dt, q.arp)


def test_tickets_budget_and_empty_requests():
    from paper_2311_11390_amd import serving
    from paper_2311_11390_amd.serving import Server
    prm = _params(64, 9)
    small = _req(prm, 500, 1.0, seed=1)
    fp = serving.footprint(small)
    with Server(fp, max_slots=2) as srv:
        with pytest.raises(L.AlifError) as ei:
            srv.submit(_req(prm, 5000, 1.0, seed=1))
        assert ei.value.code == L.ALIF_EBUDGET
        with pytest.raises(L.AlifError) as ei:
            srv.poll(12345)
        assert ei.value.code == L.ALIF_ENOTFOUND
        # a budget that holds one request at a time serialises them
        ts = [srv.submit(small) for _ in range(3)]
        res = [srv.wait(t) for t in ts]
        assert all(r.status == L.ALIF_OK for r in res)
        for a, b in zip(res, res[1:]):
            assert b.t_admit >= a.t_done
            np.testing.assert_array_equal(a.spikes, b.spikes)
        with pytest.raises(L.AlifError) as ei:
            srv.poll(ts[0])                        # already collected
        assert ei.value.code == L.ALIF_ENOTFOUND
        r0 = srv.wait(srv.submit(_req(prm, 0, 1.0, seed=1)))
        assert r0.status == L.ALIF_OK and r0.n_spikes == 0 and r0.spikes.shape == (0, 64)
    # destroy waits for everything still queued or running
    srv = Server(1 << 30, max_slots=2)
    ts = [srv.submit(_req(prm, 4000, 0.1, seed=s)) for s in range(6)]
    srv.close()


def test_spike_events_and_truncation():
    from paper_2311_11390_amd.serving import Server
    T, N, dt = 20011, 333, 0.1
    prm = _params(N, 12)
    log(f"serve events T={T} N={N}")
    with Server(1 << 30, max_slots=3) as srv:
        full = srv.wait(srv.submit(_req(prm, T, dt, seed=5)))
        only = srv.wait(srv.submit(_req(prm, T, dt, seed=5, events=10 ** 7, raster=False)))
        cut = srv.wait(srv.submit(_req(prm, T, dt, seed=5, events=100, raster=False)))
    idx = np.flatnonzero(full.spikes.ravel()).astype(np.uint32)
    assert full.n_spikes == idx.size > 100 and full.events is None
    assert only.spikes is None and not only.events_truncated
    np.testing.assert_array_equal(only.events, idx)
    assert cut.events_truncated and cut.n_spikes == idx.size
    np.testing.assert_array_equal(cut.events, idx[:100])
    t, n = np.divmod(only.events, N)
    assert np.all(full.spikes[t, n] == 1)
