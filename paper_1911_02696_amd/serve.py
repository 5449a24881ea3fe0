"""Python binding of the serving entry points (argument marshalling only), and the
synthetic serving workload.

Requests and completions cross the C ABI as numpy record arrays laid out like
ppc_request / ppc_completion, so a whole trace is one call.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib as L
from ._lib import check

REQUEST_DTYPE = np.dtype([("src", "<u8"), ("n", "<u8"), ("k", "<u4"), ("reserved", "<u4"),
                          ("arrival", "<f8"), ("tag", "<u8"), ("timeout", "<f8")])
COMPLETION_DTYPE = np.dtype([("tag", "<u8"), ("status", "<i4"), ("batch", "<u4"),
                             ("arrival", "<f8"), ("admitted", "<f8"), ("launched", "<f8"),
                             ("completed", "<f8"), ("counts", "<u8", (32,)),
                             ("arena_offset", "<u8")])
EXEC_ITEM_DTYPE = np.dtype([("src", "<u8"), ("n", "<u8"), ("k", "<u4"), ("reserved", "<u4"),
                            ("arena_offset", "<u8"), ("tag", "<u8")])
STATS_FIELDS = ("submitted", "admitted", "completed", "rejected", "launches", "queued_now",
                "inflight_now", "max_queued", "max_inflight", "arena_used_now", "arena_peak",
                "bytes_counted", "expired", "cancelled")

IN_PLACE, FIFO_BYPASS = 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_requests", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STATS_FIELDS]


_vp, _u32, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
LAUNCH_FN = ctypes.CFUNCTYPE(_i32, _vp, _vp, _u32, ctypes.POINTER(ctypes.c_uint64))
POLL_FN = ctypes.CFUNCTYPE(_i32, _vp, ctypes.c_uint64, ctypes.POINTER(_i32))
RESULTS_FN = ctypes.CFUNCTYPE(_i32, _vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64))
RELEASE_FN = ctypes.CFUNCTYPE(_i32, _vp, ctypes.c_uint64)


class ExecutorOps(ctypes.Structure):
    _fields_ = [("launch", LAUNCH_FN), ("poll", POLL_FN), ("results", RESULTS_FN),
                ("release", RELEASE_FN)]


L.register_signatures({
    "ppc_server_create": (_i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    "ppc_server_create_with_executor": (_i32, [ctypes.POINTER(ServerConfig),
                                               ctypes.POINTER(ExecutorOps), _vp,
                                               ctypes.POINTER(_vp)]),
    "ppc_server_destroy": (_i32, [_vp]),
    "ppc_server_now": (ctypes.c_double, [_vp]),
    "ppc_server_submit": (_i32, [_vp, _vp, _u32]),
    "ppc_server_progress": (_i32, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    "ppc_server_take_completions": (_i32, [_vp, _vp, _u32, ctypes.POINTER(_u32)]),
    "ppc_server_get_stats": (_i32, [_vp, ctypes.POINTER(ServerStats)]),
    "ppc_server_run_trace": (_i32, [_vp, _vp, _u32, _vp]),
    "ppc_server_cancel": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(_u32)]),
    "ppc_server_arena": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64)]),
})


def requests(srcs, ns, ks, arrivals=None, tags=None, timeouts=None) -> np.ndarray:
    m = len(ns)
    r = np.zeros(m, REQUEST_DTYPE)
    r["src"] = np.asarray(srcs, dtype=np.uint64)
    r["n"] = np.asarray(ns, dtype=np.uint64)
    r["k"] = np.asarray(ks, dtype=np.uint32)
    r["arrival"] = 0.0 if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    r["tag"] = np.arange(m, dtype=np.uint64) if tags is None else np.asarray(tags, np.uint64)
    r["timeout"] = 0.0 if timeouts is None else np.asarray(timeouts, dtype=np.float64)
    return r


class Server:
    """A serving loop over the batched count (GPU), or over caller executor callbacks."""

    def __init__(self, arena_bytes: int, max_requests: int = 4096, max_batch: int = 1024,
                 streams: int = 4, in_place: bool = False, fifo_bypass: bool = False,
                 executor: "ExecutorOps | None" = None, user=None):
        cfg = ServerConfig(arena_bytes, max_requests, max_batch, streams,
                           (IN_PLACE if in_place else 0) | (FIFO_BYPASS if fifo_bypass else 0))
        h = ctypes.c_void_p()
        lib = L.lib()
        if executor is None:
            check(lib.ppc_server_create(ctypes.byref(cfg), ctypes.byref(h)), "ppc_server_create")
        else:
            self._ops = executor  # keep the callbacks alive
            check(lib.ppc_server_create_with_executor(ctypes.byref(cfg), ctypes.byref(executor),
                                                      user, ctypes.byref(h)),
                  "ppc_server_create_with_executor")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("server is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().ppc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def now(self) -> float:
        return L.lib().ppc_server_now(self.handle)

    def submit(self, reqs: np.ndarray):
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        check(L.lib().ppc_server_submit(self.handle, reqs.ctypes.data if len(reqs) else None,
                                        len(reqs)), "ppc_server_submit")

    def progress(self):
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        check(L.lib().ppc_server_progress(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def take_completions(self, cap: int = 4096) -> np.ndarray:
        out = np.zeros(cap, COMPLETION_DTYPE)
        n = ctypes.c_uint32()
        check(L.lib().ppc_server_take_completions(self.handle, out.ctypes.data, cap,
                                                  ctypes.byref(n)))
        return out[:n.value]

    def cancel(self, tag: int) -> int:
        n = ctypes.c_uint32()
        check(L.lib().ppc_server_cancel(self.handle, tag, ctypes.byref(n)), "ppc_server_cancel")
        return n.value

    def arena(self) -> tuple[int, int]:
        """(device address, bytes) of the server's arena; address 0 in place."""
        base, size = ctypes.c_void_p(), ctypes.c_uint64()
        check(L.lib().ppc_server_arena(self.handle, ctypes.byref(base), ctypes.byref(size)),
              "ppc_server_arena")
        return base.value or 0, size.value

    def stats(self) -> dict:
        s = ServerStats()
        check(L.lib().ppc_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f in STATS_FIELDS}

    def run_trace(self, reqs: np.ndarray) -> np.ndarray:
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        out = np.zeros(len(reqs), COMPLETION_DTYPE)
        check(L.lib().ppc_server_run_trace(self.handle, reqs.ctypes.data, len(reqs),
                                           out.ctypes.data), "ppc_server_run_trace")
        return out


def latency_summary(c: np.ndarray) -> dict:
    """p50/p90/p99/max of completion - arrival over the successful completions (ms)."""
    ok = c[c["status"] == 0]
    lat = (ok["completed"] - ok["arrival"]) * 1e3
    q = lambda x: float(np.percentile(lat, x)) if len(lat) else math.nan  # noqa: E731
    return {"requests": int(len(c)), "ok": int(len(ok)), "p50_ms": round(q(50), 4),
            "p90_ms": round(q(90), 4), "p99_ms": round(q(99), 4),
            "max_ms": round(float(lat.max()) if len(lat) else math.nan, 4),
            "mean_batch": round(float(ok["batch"].mean()) if len(ok) else math.nan, 2)}


class Pools:
    """The device-resident source pools of a serving trace (and their host copies,
    kept for checking), generated from the trace's seeded distributions."""

    def __init__(self, trace, pool_bytes: int, seed: int, keep_host: bool = True):
        import torch
        from . import inputs as I
        self.host = []
        self.dev = []
        for i, (k, dist) in enumerate(trace.pools):
            h = I.generate(pool_bytes, dist, seed, stream=i)
            self.dev.append(torch.from_numpy(h).cuda())
            self.host.append(h if keep_host else None)

    def requests(self, trace) -> np.ndarray:
        base = np.array([d.data_ptr() for d in self.dev], dtype=np.uint64)
        return requests(base[trace.pool] + trace.offset, trace.lengths, trace.ks,
                        arrivals=trace.arrival)

    def host_bytes(self, trace, i) -> np.ndarray:
        p, o, b = int(trace.pool[i]), int(trace.offset[i]), int(trace.nbytes[i])
        return self.host[p][o:o + b]
