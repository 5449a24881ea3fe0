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
