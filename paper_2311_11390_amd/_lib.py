"""ctypes binding of libblockalif (include/blockalif.h): structs, constants and the
exported functions under their C names. Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_double, c_float, c_int, c_int32, c_int64, c_size_t,
                    c_uint8, c_uint32, c_uint64, c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblockalif.so")

# status codes
ALIF_OK = 0
ALIF_PENDING = 1
ALIF_EINVAL = -1
ALIF_ENOMEM = -2
ALIF_EHIP = -3
ALIF_EBUDGET = -4
ALIF_ENOTFOUND = -5
ALIF_EUNSUPPORTED = -6
ALIF_ESHUTDOWN = -7
ALIF_MAX_TR = 128
ALIF_STATUS_BAD_PARAM = 1

# enums
INPUT_CURRENT_F32, INPUT_SPIKES_U8, INPUT_SPIKES_BF16, INPUT_SPIKES_F32 = 0, 1, 2, 3
GEMM_FP32, GEMM_BF16 = 0, 1
SPIKES_U8, SPIKES_BF16, SPIKES_F32 = 0, 1, 2
ALGO_BLOCKS, ALGO_SEQUENTIAL, ALGO_SEQUENTIAL_STEP = 0, 1, 2
SG_FAST_SIGMOID, SG_BOXCAR, SG_MULTI_GAUSSIAN = 0, 1, 2
GRAD_DETACHED, GRAD_ATTACHED = 0, 1
REQ_HOST_CURRENT, REQ_OU = 0, 1


class AlifDesc(Structure):
    _fields_ = [("batch", c_int32), ("n_in", c_int32), ("n_neurons", c_int32), ("T", c_int32),
                ("dt_ms", c_double), ("arp_ms", c_double), ("input_kind", c_int32),
                ("gemm_precision", c_int32), ("spike_dtype", c_int32), ("algo", c_int32),
                ("surrogate", c_int32), ("sg_slope", c_float), ("grad_policy", c_int32)]


class AlifParams(Structure):
    _fields_ = [("tau_mem_ms", c_void_p), ("tau_adapt_ms", c_void_p), ("d", c_void_p),
                ("theta0", c_void_p), ("bias", c_void_p)]


class AlifState(Structure):
    _fields_ = [("v", c_void_p), ("a", c_void_p), ("ts", c_void_p)]


class AlifRequest(Structure):
    _fields_ = [("n_neurons", c_int32), ("T", c_int32), ("dt_ms", c_double), ("arp_ms", c_double),
                ("tau_mem_ms", c_void_p), ("tau_adapt_ms", c_void_p), ("d", c_void_p),
                ("theta0", c_void_p), ("bias", c_void_p), ("input", c_int32),
                ("host_current", c_void_p), ("ou_tau_ms", c_float), ("ou_mean", c_float),
                ("ou_sd", c_float), ("seed", c_uint64), ("host_spikes", c_void_p),
                ("host_events", c_void_p), ("events_capacity", c_int64)]


class AlifResult(Structure):
    _fields_ = [("status", c_int32), ("events_truncated", c_int32), ("n_spikes", c_int64),
                ("t_submit_s", c_double), ("t_admit_s", c_double), ("t_done_s", c_double)]


_P = c_void_p
_SIGNATURES = {
    "alif_refractory_steps": (c_int, [c_double, c_double]),
    "alif_carry_bytes": (c_int, [POINTER(AlifDesc), POINTER(c_size_t)]),
    "alif_backward_workspace_bytes": (c_int, [POINTER(AlifDesc), POINTER(c_size_t)]),
    "alif_decay_tables": (c_int, [POINTER(AlifDesc), POINTER(AlifParams), _P, _P, _P]),
    "alif_input_current": (c_int, [POINTER(AlifDesc), _P, _P, _P, _P, _P]),
    "alif_recurrent_workspace_bytes": (c_int, [POINTER(AlifDesc), POINTER(c_size_t)]),
    "alif_forward_recurrent": (c_int, [POINTER(AlifDesc), POINTER(AlifParams), _P, _P, _P, c_int32, _P, _P, _P,
                                       _P, _P, _P, _P]),
    "alif_recurrent_weight_grad": (c_int, [POINTER(AlifDesc), c_int32, _P, _P, _P, _P, _P]),
    "alif_weight_grad_workspace_bytes": (c_int, [POINTER(AlifDesc), POINTER(c_size_t)]),
    "alif_weight_grad": (c_int, [POINTER(AlifDesc), _P, _P, _P, _P, _P]),
    "alif_input_grad": (c_int, [POINTER(AlifDesc), _P, _P, _P, _P]),
    "alif_forward": (c_int, [POINTER(AlifDesc), POINTER(AlifParams), _P, _P, _P,
                             POINTER(AlifState), POINTER(AlifState), _P, _P, _P, _P, _P]),
    "alif_backward": (c_int, [POINTER(AlifDesc), POINTER(AlifParams), _P, _P, _P, _P,
                              _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "alif_backward_noalloc": (c_int, [POINTER(AlifDesc), POINTER(AlifParams), _P, _P, _P, _P,
                                      _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "alif_readout_workspace_bytes": (c_int, [c_int32, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "alif_readout_forward": (c_int, [c_int32, c_int32, c_int32, c_int32, c_double, c_int32,
                                     _P, _P, _P, _P, _P, _P]),
    "alif_readout_backward": (c_int, [c_int32, c_int32, c_int32, c_int32, c_double, c_int32,
                                      _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "alif_van_rossum_workspace_bytes": (c_int, [c_int32, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "alif_van_rossum": (c_int, [c_int32, c_int32, c_int32, c_int32, c_double, c_double, _P, _P, c_float,
                                _P, _P, _P, _P]),
    "alif_adam_step": (c_int, [c_int32, _P, _P, _P, _P, c_int32, c_double, c_double, c_double, c_double,
                               c_float, c_float, _P]),
    "alif_transpose": (c_int, [c_int32, c_int32, _P, _P, _P]),
    "alif_input_current_events": (c_int, [POINTER(AlifDesc), _P, _P, _P, _P, _P]),
    "alif_device_status": (c_int, [POINTER(c_uint32), _P]),
    "alif_last_error": (ctypes.c_char_p, []),
    "alif_ou_workspace_bytes": (c_int, [c_int32, c_int32, POINTER(c_size_t)]),
    "alif_ou_current": (c_int, [c_int32, c_int32, c_double, c_float, c_float, c_float, c_uint64,
                                _P, _P, c_size_t, _P]),
    "alif_server_create": (c_int, [c_size_t, c_int32, c_int32, POINTER(c_void_p)]),
    "alif_request_footprint": (c_int, [POINTER(AlifRequest), POINTER(c_size_t)]),
    "alif_submit": (c_int, [c_void_p, POINTER(AlifRequest), POINTER(c_uint64)]),
    "alif_poll": (c_int, [c_void_p, c_uint64, POINTER(AlifResult)]),
    "alif_server_destroy": (c_int, [c_void_p]),
}

_lib = None


class AlifError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libblockalif error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load the in-tree library; fail loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2311_11390_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> int:
    if rc < 0:
        raise AlifError(rc, load().alif_last_error().decode())
    return rc


def exported_symbols():
    return list(_SIGNATURES)
