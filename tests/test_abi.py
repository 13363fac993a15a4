"""C-ABI checks that need no GPU: the library loads, exports every function the
public header declares, the ctypes struct layouts match the C compiler's, and
host-side validation rejects bad descriptors before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2311_11390_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blockalif.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*(alif_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.exported_symbols())


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "blockalif.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(alif_desc), sizeof(alif_params), sizeof(alif_state),
         sizeof(alif_request), sizeof(alif_result));
  printf("%zu %zu %zu %zu\\n", offsetof(alif_desc, dt_ms), offsetof(alif_desc, sg_slope),
         offsetof(alif_request, seed), offsetof(alif_request, host_spikes));
  printf("%zu %zu %zu\\n", offsetof(alif_request, host_events), offsetof(alif_request, events_capacity),
         offsetof(alif_result, n_spikes));
  return 0;
}""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    c = [int(x) for x in out]
    py = [ctypes.sizeof(L.AlifDesc), ctypes.sizeof(L.AlifParams), ctypes.sizeof(L.AlifState),
          ctypes.sizeof(L.AlifRequest), ctypes.sizeof(L.AlifResult),
          L.AlifDesc.dt_ms.offset, L.AlifDesc.sg_slope.offset, L.AlifRequest.seed.offset,
          L.AlifRequest.host_spikes.offset, L.AlifRequest.host_events.offset,
          L.AlifRequest.events_capacity.offset, L.AlifResult.n_spikes.offset]
    assert c == py


def test_refractory_steps_rules():
    lib = L.load()
    assert lib.alif_refractory_steps(0.05, 2.0) == 40
    assert lib.alif_refractory_steps(1.0, 2.0) == 2
    assert lib.alif_refractory_steps(1.0, 1.0) == L.ALIF_EINVAL       # T_R = 1
    assert b"T_R" in lib.alif_last_error()
    assert lib.alif_refractory_steps(0.3, 2.0) == L.ALIF_EINVAL       # not whole
    assert lib.alif_refractory_steps(0.01, 2.0) == L.ALIF_EUNSUPPORTED  # 200 > 128


def _desc(**kw):
    d = dict(batch=2, n_in=0, n_neurons=8, T=100, dt_ms=0.5, arp_ms=2.0, input_kind=0,
             gemm_precision=0, spike_dtype=0, algo=0, surrogate=0, sg_slope=10.0)
    d.update(kw)
    return L.AlifDesc(**d)


def test_sizes_and_validation_host_side():
    lib = L.load()
    n = ctypes.c_size_t()
    assert lib.alif_carry_bytes(ctypes.byref(_desc()), ctypes.byref(n)) == 0
    nb = 25
    assert n.value >= 2 * 8 * nb * 4 * 2 + 2 * 8 * nb
    assert lib.alif_carry_bytes(ctypes.byref(_desc(batch=-1)), ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_carry_bytes(ctypes.byref(_desc(input_kind=7)), ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_carry_bytes(ctypes.byref(_desc(input_kind=1, n_in=0)), ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_carry_bytes(ctypes.byref(_desc(algo=9)), ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_carry_bytes(ctypes.byref(_desc(T=2 ** 28, n_neurons=16)), ctypes.byref(n)) == L.ALIF_EUNSUPPORTED
    assert lib.alif_carry_bytes(None, ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_backward_workspace_bytes(ctypes.byref(_desc()), ctypes.byref(n)) == 0
    assert n.value >= 5 * 2 * 8 * 8
    # forward rejects a bad descriptor before any device call
    p = L.AlifParams(None, None, None, None, None)
    assert lib.alif_forward(ctypes.byref(_desc(dt_ms=1.0, arp_ms=1.0)), ctypes.byref(p), None, None, None,
                            None, None, None, None, None, None, None) == L.ALIF_EINVAL
    assert lib.alif_forward(ctypes.byref(_desc()), ctypes.byref(p), None, None, None,
                            None, None, None, None, None, None, None) == L.ALIF_EINVAL
    assert b"required" in lib.alif_last_error()


def test_projection_and_recurrent_validation_host_side():
    """The dW / dx and recurrent entry points reject bad arguments before any
    device call."""
    lib = L.load()
    n = ctypes.c_size_t()
    by = ctypes.byref
    spk = _desc(input_kind=1, n_in=16)
    assert lib.alif_weight_grad_workspace_bytes(by(spk), by(n)) == 0
    assert lib.alif_weight_grad(by(_desc()), None, None, None, None, None) == L.ALIF_EINVAL
    assert b"spike input_kind" in lib.alif_last_error()
    assert lib.alif_weight_grad(by(spk), None, None, None, None, None) == L.ALIF_EINVAL
    assert lib.alif_input_grad(by(_desc()), None, None, None, None) == L.ALIF_EINVAL
    assert lib.alif_input_grad(by(spk), None, None, None, None) == L.ALIF_EINVAL
    assert b"required" in lib.alif_last_error()
    # recurrent layer
    assert lib.alif_recurrent_workspace_bytes(by(_desc()), by(n)) == 0 and n.value > 0
    none_p = L.AlifParams(None, None, None, None, None)
    fake_p = L.AlifParams(16, 16, 16, 16, None)   # never dereferenced: validation fails first
    args = [None] * 7
    assert lib.alif_forward_recurrent(by(_desc()), by(none_p), None, None, None, 0, *args) == L.ALIF_EINVAL
    assert lib.alif_forward_recurrent(by(_desc()), by(fake_p), None, None, None, 0, *args) == L.ALIF_EINVAL
    assert b"required" in lib.alif_last_error()
    assert lib.alif_forward_recurrent(by(_desc()), by(fake_p), None, None, None, 1, *args) == L.ALIF_EINVAL
    assert b"delay" in lib.alif_last_error()
    assert lib.alif_forward_recurrent(by(_desc(algo=1)), by(fake_p), None, None, None, 0, *args) == \
        L.ALIF_EUNSUPPORTED
    assert lib.alif_recurrent_weight_grad(by(_desc()), 1, None, None, None, None, None) == L.ALIF_EINVAL
    assert lib.alif_recurrent_weight_grad(by(_desc()), 0, None, None, None, None, None) == L.ALIF_EINVAL
    assert b"required" in lib.alif_last_error()
    # the event count and masks sit at the workspace's start: it must be 256-byte aligned
    assert lib.alif_recurrent_weight_grad(by(_desc()), 0, 256, 256, 256, 256 + 16, None) == L.ALIF_EINVAL
    assert b"aligned" in lib.alif_last_error()


def _request(N=100, T=1000, dt=0.05, arp=2.0, **kw):
    import numpy as np

    from paper_2311_11390_amd.serving import Request
    base = dict(T=T, dt=dt, arp=arp, tau_mem=np.full(N, 20.0), tau_adapt=np.full(N, 200.0),
                d=np.full(N, 1.8), theta0=np.ones(N))
    base.update(kw)
    return Request(**base)


def test_serving_footprint_and_validation_host_side():
    import numpy as np

    from paper_2311_11390_amd import serving
    N, T = 100, 1000
    fp = serving.footprint(_request(N, T))
    nc = -(-T // 256)                    # OU chunks of 256 steps
    g = -(-(T * N) // 8192)              # raster compaction workgroups
    want = sum(-(-x // 256) * 256 for x in (5 * N * 4, T * N * 4, T * N, nc * N * 8, g * 4, g * 4)) + 256
    assert fp == want
    fp_host = serving.footprint(_request(N, T, current=np.zeros((T, N), np.float32)))
    assert fp_host == want - (-(-nc * N * 8 // 256) * 256)
    bad = [
        dict(dt=1.0, arp=1.0),                                   # T_R = 1
        dict(dt=0.3, arp=2.0),                                   # not whole
        dict(tau_mem=np.full(N, -1.0)),
        dict(tau_adapt=np.zeros(N)),
        dict(d=np.full(N, -0.1)),
        dict(theta0=np.zeros(N)),
        dict(theta0=np.full(N, np.nan)),
        dict(ou_tau=0.0),
        dict(ou_sd=-1.0),
        dict(events_capacity=-1),
    ]
    for kw in bad:
        with pytest.raises(L.AlifError) as ei:
            serving.footprint(_request(N, T, **kw))
        assert ei.value.code == L.ALIF_EINVAL, kw
    with pytest.raises(L.AlifError) as ei:
        serving.footprint(_request(N, T, dt=0.01))              # T_R = 200 > ALIF_MAX_TR
    assert ei.value.code == L.ALIF_EUNSUPPORTED
    with pytest.raises(L.AlifError) as ei:
        serving.footprint(_request(4096, 2 ** 17))              # T * N * 4 >= 2^31
    assert ei.value.code == L.ALIF_EUNSUPPORTED
    lib = L.load()
    c, _ = serving.c_request(_request(N, T))
    c.input = 5
    n = ctypes.c_size_t()
    assert lib.alif_request_footprint(ctypes.byref(c), ctypes.byref(n)) == L.ALIF_EINVAL
    c.input = L.REQ_HOST_CURRENT
    c.host_current = None
    assert lib.alif_request_footprint(ctypes.byref(c), ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_request_footprint(None, ctypes.byref(n)) == L.ALIF_EINVAL
    t = ctypes.c_uint64()
    assert lib.alif_submit(None, ctypes.byref(c), ctypes.byref(t)) == L.ALIF_EINVAL
    assert lib.alif_poll(None, 1, None) == L.ALIF_EINVAL
    assert lib.alif_server_destroy(None) == L.ALIF_OK
    h = ctypes.c_void_p()
    assert lib.alif_server_create(1 << 30, 0, 0, ctypes.byref(h)) == L.ALIF_EINVAL
    assert lib.alif_server_create(0, 4, 0, ctypes.byref(h)) == L.ALIF_EINVAL


def test_ou_current_sizes_and_validation_host_side():
    lib = L.load()
    n = ctypes.c_size_t()
    assert lib.alif_ou_workspace_bytes(1000, 100, ctypes.byref(n)) == 0
    assert n.value == -(-(4 * 100 * 8) // 256) * 256
    assert lib.alif_ou_workspace_bytes(-1, 100, ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_ou_current(10, 10, 0.05, 0.0, 0.8, 0.5, 1, None, None, 0, None) == L.ALIF_EINVAL
    assert lib.alif_ou_current(10, 10, 0.05, 5.0, 0.8, -0.5, 1, None, None, 0, None) == L.ALIF_EINVAL
    assert lib.alif_ou_current(10, 10, 0.0, 5.0, 0.8, 0.5, 1, None, None, 0, None) == L.ALIF_EINVAL
    assert lib.alif_ou_current(10, 10, 0.05, 5.0, 0.8, 0.5, 1, None, None, 0, None) == L.ALIF_EINVAL
    assert lib.alif_ou_current(0, 10, 0.05, 5.0, 0.8, 0.5, 1, None, None, 0, None) == L.ALIF_OK


def test_van_rossum_and_adam_validation_host_side():
    lib = L.load()
    n = ctypes.c_size_t()
    assert lib.alif_van_rossum_workspace_bytes(4, 4, 20000, 2048, ctypes.byref(n)) == L.ALIF_OK
    assert n.value > 0
    assert lib.alif_van_rossum_workspace_bytes(4, 9, 100, 8, ctypes.byref(n)) == L.ALIF_EUNSUPPORTED
    assert lib.alif_van_rossum_workspace_bytes(4, 0, 100, 8, ctypes.byref(n)) == L.ALIF_EINVAL
    assert lib.alif_van_rossum_workspace_bytes(-1, 1, 100, 8, ctypes.byref(n)) == L.ALIF_EINVAL
    vr = lib.alif_van_rossum
    dummy = ctypes.c_void_p(256)
    assert vr(2, 1, 10, 8, 0.0, 100.0, dummy, dummy, 1.0, dummy, dummy, dummy, None) == L.ALIF_EINVAL
    assert vr(2, 1, 10, 8, 0.1, -1.0, dummy, dummy, 1.0, dummy, dummy, dummy, None) == L.ALIF_EINVAL
    assert vr(2, 1, 10, 8, 0.1, float("inf"), dummy, dummy, 1.0, dummy, dummy, dummy, None) == L.ALIF_EINVAL
    assert vr(2, 1, 10, 8, 0.1, 100.0, dummy, dummy, float("nan"), dummy, dummy, dummy, None) == L.ALIF_EINVAL
    assert vr(2, 9, 10, 8, 0.1, 100.0, dummy, dummy, 1.0, dummy, dummy, dummy, None) == L.ALIF_EUNSUPPORTED
    assert vr(2, 1, 10, 8, 0.1, 100.0, None, dummy, 1.0, dummy, dummy, dummy, None) == L.ALIF_EINVAL
    assert vr(2, 1, 10, 8, 0.1, 100.0, dummy, dummy, 1.0, dummy, dummy, None, None) == L.ALIF_EINVAL
    odd = ctypes.c_void_p(258)
    assert vr(2, 1, 10, 8, 0.1, 100.0, odd, dummy, 1.0, dummy, dummy, dummy, None) == L.ALIF_EINVAL
    assert vr(2, 1, 10, 8, 0.1, 100.0, dummy, dummy, 1.0, dummy, ctypes.c_void_p(264), dummy, None) == L.ALIF_EINVAL
    # neither output requested: nothing to do
    assert vr(2, 1, 10, 8, 0.1, 100.0, None, None, 1.0, None, None, None, None) == L.ALIF_OK
    adam = lib.alif_adam_step
    assert adam(10, dummy, dummy, dummy, dummy, 0, 0.1, 0.9, 0.999, 1e-8, 0.0, 1.0, None) == L.ALIF_EINVAL
    assert adam(10, dummy, dummy, dummy, dummy, 1, 0.1, 1.0, 0.999, 1e-8, 0.0, 1.0, None) == L.ALIF_EINVAL
    assert adam(10, dummy, dummy, dummy, dummy, 1, 0.1, 0.9, 0.999, 0.0, 0.0, 1.0, None) == L.ALIF_EINVAL
    assert adam(10, dummy, dummy, dummy, dummy, 1, 0.1, 0.9, 0.999, 1e-8, 2.0, 1.0, None) == L.ALIF_EINVAL
    assert adam(10, None, dummy, dummy, dummy, 1, 0.1, 0.9, 0.999, 1e-8, 0.0, 1.0, None) == L.ALIF_EINVAL
    assert adam(0, None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8, 0.0, 1.0, None) == L.ALIF_OK


def test_event_current_and_transpose_validation_host_side():
    """alif_input_current_events and alif_transpose reject bad arguments before any
    device call."""
    lib = L.load()
    by = ctypes.byref
    dummy = ctypes.c_void_p(256)
    ev = lib.alif_input_current_events
    assert ev(None, dummy, dummy, None, dummy, None) == L.ALIF_EINVAL
    assert ev(by(_desc()), dummy, dummy, None, dummy, None) == L.ALIF_EINVAL          # current input kind
    assert b"spike input_kind" in lib.alif_last_error()
    assert ev(by(_desc(input_kind=1, n_in=-1)), dummy, dummy, None, dummy, None) == L.ALIF_EINVAL
    assert ev(by(_desc(input_kind=1, n_in=16)), None, dummy, None, dummy, None) == L.ALIF_EINVAL
    bf16 = _desc(input_kind=L.INPUT_SPIKES_BF16, n_in=16)
    assert ev(by(bf16), ctypes.c_void_p(257), dummy, None, dummy, None) == L.ALIF_EINVAL   # odd bf16 address
    assert b"aligned" in lib.alif_last_error()
    assert ev(by(_desc(input_kind=1, n_in=16)), dummy, ctypes.c_void_p(258), None, dummy, None) == L.ALIF_EINVAL
    assert ev(by(_desc(input_kind=1, n_in=16, batch=0)), None, None, None, None, None) == L.ALIF_OK
    tr = lib.alif_transpose
    assert tr(-1, 4, dummy, dummy, None) == L.ALIF_EINVAL
    assert tr(4, 4, dummy, dummy, None) == L.ALIF_EINVAL                                  # aliasing
    assert tr(0, 4, None, None, None) == L.ALIF_OK
