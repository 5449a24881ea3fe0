"""Python binding of the batched entry points (argument marshalling only).

A descriptor is four little-endian 64-bit words: [ptr, n, k | reserved << 32,
counts] (the ppc_desc layout of include/pospopcnt.h).  ``descriptors`` builds
such a table with numpy; upload it to the device (``to_device``) and pass it to
``Plan.run``.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import BatchConfig, check
from .api import stream_handle

DESC_BYTES = 32


def descriptors(ptrs, ns, ks, counts_ptrs, reserved=None) -> np.ndarray:
    """(m, 4) uint64 table of ppc_desc records."""
    m = len(ptrs)
    d = np.zeros((m, 4), dtype=np.uint64)
    d[:, 0] = np.asarray(ptrs, dtype=np.uint64)
    d[:, 1] = np.asarray(ns, dtype=np.uint64)
    k = np.asarray(ks, dtype=np.uint64)
    r = np.zeros(m, dtype=np.uint64) if reserved is None else np.asarray(reserved, np.uint64)
    d[:, 2] = k | (r << np.uint64(32))
    d[:, 3] = np.asarray(counts_ptrs, dtype=np.uint64)
    return d


def to_device(desc: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(desc).view(np.int64)).to(device)


class Plan:
    """A batched-count plan: device scratch for up to max_streams descriptors, a
    launch configuration, and (graph=True) a captured HIP graph per workload."""

    def __init__(self, max_streams: int, graph: bool = False):
        hint = L.WorkloadHint(max_streams, L.PLAN_GRAPH if graph else 0)
        h = ctypes.c_void_p()
        check(L.lib().ppc_plan_create(ctypes.byref(hint), ctypes.byref(h)), "ppc_plan_create")
        self._h = h
        self.max_streams = max_streams
        self.graph = graph

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().ppc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _descs(descs: torch.Tensor, m):
        if not descs.is_cuda or not descs.is_contiguous():
            raise ValueError("descriptors must be a contiguous device tensor")
        cap = descs.numel() * descs.element_size() // DESC_BYTES
        m = cap if m is None else m
        if m > cap:
            raise ValueError(f"{m} descriptors requested, the tensor holds {cap}")
        return descs.data_ptr(), m

    @staticmethod
    def _keep(descs: torch.Tensor, stream):
        # The kernels read the descriptors when they run: on a stream other than
        # the one their memory belongs to, keep that memory from being reused first.
        if isinstance(stream, torch.cuda.Stream) and stream != torch.cuda.current_stream():
            descs.record_stream(stream)

    def run(self, descs: torch.Tensor, m: int | None = None, stream=None) -> None:
        ptr, m = self._descs(descs, m)
        self._keep(descs, stream)
        check(L.lib().pospopcnt_batch(self.handle, ptr, m, stream_handle(stream)),
              "pospopcnt_batch")

    def autotune(self, descs: torch.Tensor, m: int | None = None, stream=None) -> float:
        ptr, m = self._descs(descs, m)
        self._keep(descs, stream)
        best = ctypes.c_float(0.0)
        check(L.lib().ppc_plan_autotune(self.handle, ptr, m, stream_handle(stream),
                                        ctypes.byref(best)), "ppc_plan_autotune")
        return best.value

    @property
    def config(self) -> dict:
        c = BatchConfig()
        check(L.lib().ppc_plan_get_config(self.handle, ctypes.byref(c)))
        return {"depth": c.depth, "block_threads": c.block_threads,
                "blocks_per_cu": c.blocks_per_cu, "stream_weight": c.stream_weight}

    @config.setter
    def config(self, cfg: dict):
        cur = self.config
        cur.update(cfg)
        c = BatchConfig(cur["depth"], cur["block_threads"], cur["blocks_per_cu"],
                        cur["stream_weight"])
        check(L.lib().ppc_plan_set_config(self.handle, ctypes.byref(c)), "ppc_plan_set_config")

    def save(self, path: str):
        check(L.lib().ppc_plan_save(self.handle, path.encode()), "ppc_plan_save")

    def load(self, path: str):
        check(L.lib().ppc_plan_load(self.handle, path.encode()), "ppc_plan_load")

    def cache_put(self, path: str, m: int, nbytes: int):
        """Store the configuration in a cache file under the key of (m streams, nbytes)."""
        check(L.lib().ppc_plan_cache_put(self.handle, path.encode(), m, nbytes),
              "ppc_plan_cache_put")

    def cache_get(self, path: str, m: int, nbytes: int) -> bool:
        """Take the configuration stored for (m, nbytes); False if the cache has none."""
        st = L.lib().ppc_plan_cache_get(self.handle, path.encode(), m, nbytes)
        if st == 9:  # PPC_ERR_STATE: no entry for this key
            return False
        check(st, "ppc_plan_cache_get")
        return True

    def rejected(self, stream=None) -> int:
        out = ctypes.c_uint32()
        check(L.lib().ppc_plan_rejected(self.handle, stream_handle(stream), ctypes.byref(out)))
        return out.value


def batch_static(descs: torch.Tensor, m: int | None = None, config: dict | None = None,
                 stream=None) -> None:
    """The batched count without a plan (pospopcnt_batch_static): scratch in the
    library's file-scope device array, nothing allocated.  At most
    STATIC_MAX_STREAMS descriptors; calls on one device must not overlap in time.
    config: a dict of the plan configuration's fields, or None for the default."""
    ptr, m = Plan._descs(descs, m)
    Plan._keep(descs, stream)
    cfg = None
    if config is not None:
        c = dict(depth=16, block_threads=64, blocks_per_cu=4, stream_weight=2048)
        c.update(config)
        cfg = ctypes.byref(BatchConfig(c["depth"], c["block_threads"], c["blocks_per_cu"],
                                       c["stream_weight"]))
    check(L.lib().pospopcnt_batch_static(ptr, m, cfg, stream_handle(stream)),
          "pospopcnt_batch_static")


STATIC_MAX_STREAMS = L.STATIC_MAX_STREAMS


def pospopcnt_each(host_descs: np.ndarray, stream=None) -> None:
    """One single-stream launch per descriptor of a host table."""
    d = np.ascontiguousarray(host_descs, dtype=np.uint64)
    check(L.lib().pospopcnt_each(d.ctypes.data if d.size else None, d.shape[0],
                                 stream_handle(stream)), "pospopcnt_each")
