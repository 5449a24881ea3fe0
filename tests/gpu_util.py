"""Helpers for the GPU tests: seeded host bytes, placement in device memory at a
chosen byte offset, and the oracle on the same host bytes."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_1911_02696_amd import inputs as I


def say(*args):
    """Name the case before a GPU step, flushed, so a failing run shows it."""
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def host_bytes(nbytes: int, dist: I.Dist, seed: int) -> np.ndarray:
    return I.generate(nbytes, dist, seed)


def to_device(host: np.ndarray, offset: int = 0, pad: int = 64) -> tuple[torch.Tensor, int]:
    """Copy host bytes into a fresh device buffer so that they start `offset` bytes
    past a 256-byte aligned address.  Returns (buffer, offset).  The buffer is
    padded on both sides with 0xA5 bytes, which a correct kernel never counts."""
    n = host.size
    buf = torch.full((offset + n + pad,), 0xA5, dtype=torch.uint8, device="cuda")
    assert buf.data_ptr() % 256 == 0
    if n:
        buf[offset:offset + n].copy_(torch.from_numpy(host))
    return buf, offset


def oracle_counts(host: np.ndarray, n: int, k: int, threads: int | None = None) -> np.ndarray:
    th = threads if threads is not None else (1 if n * k // 8 < (1 << 22) else I.default_threads())
    return oracle.count(host, n, k, threads=th).astype(np.int64)


def counts_np(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.int64)


_HIP = None


def hip():
    """The HIP runtime torch has loaded (same soname as the library's), for raw
    device memory the tests did not allocate through torch (a server's arena)."""
    global _HIP
    if _HIP is None:
        import ctypes
        torch.cuda.init()
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipDeviceSynchronize.argtypes = []
        _HIP = h
    return _HIP


def device_fill(ptr: int, value: int, nbytes: int):
    assert hip().hipMemset(ptr, value, nbytes) == 0
    assert hip().hipDeviceSynchronize() == 0


def device_read(ptr: int, nbytes: int) -> np.ndarray:
    out = np.empty(nbytes, np.uint8)
    assert hip().hipDeviceSynchronize() == 0
    assert hip().hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0  # device to host
    return out
