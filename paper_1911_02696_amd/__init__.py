"""MI355X-native positional population count (pospopcnt).

Every count runs in hand-written HIP kernels for gfx950 inside
``libpospopcnt.so`` (C ABI: include/pospopcnt.h); this package is the thin
Python binding.  The library must be built (``python -m
paper_1911_02696_amd.build``); there is no CPU fallback.
"""
from ._lib import LIB_PATH, LaunchConfig, PpcError  # noqa: F401

_API = {"pospopcnt", "pospopcnt_u8", "pospopcnt_u16", "pospopcnt_u32", "pospopcnt_ptr",
        "read_ceiling", "histogram", "device_info", "launch_config", "stream_handle"}


def __getattr__(name):
    # The torch-facing API is imported on first use, so that the input generator
    # and the C-ABI loader can be used without importing torch.
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
