"""ctypes loader of libpospopcnt.so (the C ABI of include/pospopcnt.h).

There is no fallback: if the library is missing the import of any entry point
raises, naming the build command.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
# PPC_LIB names another build of the same sources (the sanitizer run uses it).
LIB_PATH = os.environ.get("PPC_LIB") or os.path.join(PKG, "libpospopcnt.so")

PPC_OK = 0
STATUS_NAMES = {
    0: "PPC_OK", 1: "PPC_ERR_NULL", 2: "PPC_ERR_ALIGN", 3: "PPC_ERR_WIDTH",
    4: "PPC_ERR_RANGE", 5: "PPC_ERR_HIP", 6: "PPC_ERR_BUDGET", 7: "PPC_ERR_ARG",
    8: "PPC_ERR_OVERLAP", 9: "PPC_ERR_STATE", 10: "PPC_ERR_CAPACITY", 11: "PPC_ERR_TIMEOUT",
    12: "PPC_ERR_CANCELLED",
}
VARIANT_CSA, VARIANT_BALLOT, VARIANT_HYBRID = 0, 1, 2


class PpcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        lib = _lib_or_none()
        msg = lib.ppc_status_string(status).decode() if lib else STATUS_NAMES.get(status, "?")
        if status == 5 and lib:
            msg += f" (hipError_t {lib.ppc_last_hip_error()})"
        super().__init__(f"{what}: {msg}" if what else msg)


class LaunchConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("grid", ctypes.c_int64)]


class DeviceInfo(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("compute_units", ctypes.c_int32),
                ("clock_khz", ctypes.c_int32), ("l2_bytes", ctypes.c_int32),
                ("global_mem_bytes", ctypes.c_int64), ("name", ctypes.c_char * 64),
                ("arch", ctypes.c_char * 64)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("stream_weight", ctypes.c_int32)]


class WorkloadHint(ctypes.Structure):
    _fields_ = [("max_streams", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


PLAN_GRAPH = 1
STATIC_MAX_STREAMS = 65536  # PPC_STATIC_MAX_STREAMS

_vp, _u64, _i32, _i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
_u32 = ctypes.c_uint32

# name -> (restype, argtypes); every entry point the binding uses.
MAX_PLANES = 32  # PPC_MAX_PLANES

SIGNATURES = {
    "ppc_status_string": (ctypes.c_char_p, [_i32]),
    "ppc_last_hip_error": (_i32, []),
    "pospopcnt_u8": (_i32, [_vp, _u64, _vp, _vp]),
    "pospopcnt_u16": (_i32, [_vp, _u64, _vp, _vp]),
    "pospopcnt_u32": (_i32, [_vp, _u64, _vp, _vp]),
    "pospopcnt_u64": (_i32, [_vp, _u64, _vp, _vp]),
    "pospopcnt_planes16": (_i32, [ctypes.POINTER(_vp), _u32, _u64, _vp, _vp]),
    "pospopcnt_planes16_ex": (_i32, [ctypes.POINTER(_vp), _u32, _u64, _vp, _vp,
                                     ctypes.POINTER(LaunchConfig)]),
    "pospopcnt": (_i32, [_vp, _u64, _i32, _vp, _vp]),
    "pospopcnt_ex": (_i32, [_vp, _u64, _i32, _vp, _vp, ctypes.POINTER(LaunchConfig)]),
    "ppc_read_ceiling": (_i32, [_vp, _u64, _vp, _vp, ctypes.POINTER(LaunchConfig)]),
    "ppc_get_device_info": (_i32, [ctypes.POINTER(DeviceInfo)]),
    "ppc_plan_create": (_i32, [ctypes.POINTER(WorkloadHint), ctypes.POINTER(_vp)]),
    "ppc_plan_destroy": (_i32, [_vp]),
    "pospopcnt_batch": (_i32, [_vp, _vp, _u32, _vp]),
    "ppc_plan_autotune": (_i32, [_vp, _vp, _u32, _vp, ctypes.POINTER(ctypes.c_float)]),
    "ppc_plan_get_config": (_i32, [_vp, ctypes.POINTER(BatchConfig)]),
    "ppc_plan_set_config": (_i32, [_vp, ctypes.POINTER(BatchConfig)]),
    "ppc_plan_save": (_i32, [_vp, ctypes.c_char_p]),
    "ppc_plan_load": (_i32, [_vp, ctypes.c_char_p]),
    "ppc_plan_cache_put": (_i32, [_vp, ctypes.c_char_p, ctypes.c_uint32, ctypes.c_uint64]),
    "ppc_plan_cache_get": (_i32, [_vp, ctypes.c_char_p, ctypes.c_uint32, ctypes.c_uint64]),
    "ppc_plan_rejected": (_i32, [_vp, _vp, ctypes.POINTER(_u32)]),
    "pospopcnt_each": (_i32, [_vp, _u32, _vp]),
    "pospopcnt_batch_static": (_i32, [_vp, _u32, ctypes.POINTER(BatchConfig), _vp]),
    "ppc_histogram_u8": (_i32, [_vp, _u64, _u32, _vp, _vp]),
    "ppc_histogram_u16": (_i32, [_vp, _u64, _u32, _vp, _vp]),
    "ppc_histogram_ex": (_i32, [_vp, _u64, _i32, _u32, _vp, _vp, ctypes.POINTER(LaunchConfig)]),
}

_lock = threading.Lock()
_lib = None


def _lib_or_none():
    return _lib


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_1911_02696_amd.build` (hipcc, gfx950)")
            handle = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(handle, name)
                fn.restype = res
                fn.argtypes = args
            _extend(handle)
            _lib = handle
    return _lib


_extensions = []


def register_signatures(table: dict):
    """Add signatures of further entry points (used by the batch and serving modules)."""
    _extensions.append(table)
    if _lib is not None:
        _apply(_lib, table)


def _apply(handle, table):
    for name, (res, args) in table.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args


def _extend(handle):
    for table in _extensions:
        _apply(handle, table)


def check(status: int, what: str = ""):
    if status != PPC_OK:
        raise PpcError(status, what)
