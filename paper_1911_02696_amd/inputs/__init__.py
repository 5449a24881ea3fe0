"""Seeded synthetic inputs for the positional population count.

A module of its own: it draws bytes and workload shapes and computes nothing
of the counting method.  The tests, the benchmark and the serving demo all take
their inputs from here, so the GPU path and the oracle see the same bytes.

Bytes come from ``libppc_gen.so`` (counter-based SplitMix64, see ppc_gen.c), so
any byte range of a stream can be produced on its own, in parallel, into any
writable buffer (e.g. pinned host memory before an upload).  Workload shapes
(stream lengths, widths, densities, arrival times) are drawn with numpy's PCG64
from the same seeds.

Distributions follow the paper's workloads: random words (Sec. 5) as uniform
bytes or per-bit Bernoulli(p), and one-hot words (Sec. 1, Table 1) with uniform
or Zipf(s) category frequencies, category c on bit c.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PPC_GEN_LIB names another build of the same source (the sanitizer run uses it).
LIB_PATH = os.environ.get("PPC_GEN_LIB") or os.path.join(_HERE, "libppc_gen.so")

UNIFORM, BERNOULLI, ONEHOT, IDS = 0, 1, 2, 3

# Base seed of the synthetic workloads: seed of config c is BASE_SEED + c.
BASE_SEED = 0x19110269600


class _Spec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("key", ctypes.c_uint64),
                ("threshold", ctypes.c_uint64), ("cdf", ctypes.c_uint64 * 65),
                ("ncat", ctypes.c_int32), ("unused", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is not built; run `python -m paper_1911_02696_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        lib.ppcgen_fill.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.POINTER(_Spec), ctypes.c_int]
        lib.ppcgen_fill.restype = ctypes.c_int
        lib.ppcgen_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.ppcgen_key.restype = ctypes.c_uint64
        lib.ppcgen_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.ppcgen_draw.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def stream_key(seed: int, stream: int = 0) -> int:
    return _load().ppcgen_key(seed & (2**64 - 1), stream)


def draw(key: int, i: int) -> int:
    """Output i of the SplitMix64 stream with the given key."""
    return _load().ppcgen_draw(key, i)


def zipf_cdf(k: int, s: float) -> np.ndarray:
    """Integer thresholds for category frequencies P(c) proportional to (c+1)^-s, c < k."""
    w = np.array([(c + 1.0) ** (-s) for c in range(k)], dtype=np.float64)
    cum = np.cumsum(w) / w.sum()
    cdf = np.zeros(k + 1, dtype=np.uint64)
    cdf[1:] = np.floor(cum * 2.0**32).astype(np.uint64)
    cdf[k] = 2**32
    return np.maximum.accumulate(cdf)


def uniform_cdf(k: int) -> np.ndarray:
    cdf = np.array([(c * 2**32) // k for c in range(k + 1)], dtype=np.uint64)
    return cdf


@dataclass(frozen=True)
class Dist:
    """A byte distribution: kind UNIFORM, BERNOULLI (p) or ONEHOT (k, cdf)."""

    kind: int
    p: float = 0.5
    k: int = 8
    zipf_s: float | None = None  # ONEHOT, IDS: None means uniform categories
    ncat: int = 0                # IDS: number of categories
    p_invalid: float = 0.0       # IDS: share of ids >= ncat

    @staticmethod
    def uniform() -> "Dist":
        return Dist(UNIFORM)

    @staticmethod
    def bernoulli(p: float) -> "Dist":
        if not 0.0 <= p <= 1.0:
            raise ValueError("p must lie in [0, 1]")
        return Dist(BERNOULLI, p=p)

    @staticmethod
    def onehot(k: int, zipf_s: float | None = None) -> "Dist":
        return Dist(ONEHOT, k=k, zipf_s=zipf_s)

    @staticmethod
    def ids(bits: int, ncat: int, zipf_s: float | None = None, p_invalid: float = 0.0) -> "Dist":
        """Category indices (u8 or u16 words) over ncat categories; a p_invalid share
        of the words are ids >= ncat."""
        return Dist(IDS, k=bits, zipf_s=zipf_s, ncat=ncat, p_invalid=p_invalid)

    def spec(self, key: int) -> _Spec:
        s = _Spec()
        s.kind = self.kind
        s.k = self.k
        s.key = key
        p = self.p_invalid if self.kind == IDS else self.p
        s.threshold = min(2**32, int(math.floor(p * 2.0**32)))
        if self.kind in (ONEHOT, IDS):
            n = self.k if self.kind == ONEHOT else self.ncat
            cdf = zipf_cdf(n, self.zipf_s) if self.zipf_s is not None else uniform_cdf(n)
            for i, v in enumerate(cdf):
                s.cdf[i] = int(v)
            s.ncat = n
        return s


def fill(out, dist: Dist, seed: int, stream: int = 0, first_byte: int = 0,
         threads: int | None = None):
    """Write bytes [first_byte, first_byte + len(out)) of stream `stream` of `seed` into out.

    ``out`` is a writable C-contiguous numpy array (any dtype; it is filled as bytes)."""
    a = np.asarray(out)
    if not a.flags.c_contiguous or not a.flags.writeable:
        raise ValueError("out must be a writable C-contiguous array")
    nbytes = a.nbytes
    if nbytes == 0:
        return out
    spec = dist.spec(stream_key(seed, stream))
    rc = _load().ppcgen_fill(a.ctypes.data, first_byte, nbytes, ctypes.byref(spec),
                             threads or default_threads())
    if rc != 0:
        raise ValueError("bad generator spec")
    return out


def generate(nbytes: int, dist: Dist, seed: int, stream: int = 0, first_byte: int = 0,
             threads: int | None = None) -> np.ndarray:
    out = np.empty(nbytes, dtype=np.uint8)
    return fill(out, dist, seed, stream, first_byte, threads)


# ---------------------------------------------------------------- workload shapes

@dataclass
class StreamSet:
    """Shapes of a batch of independent streams (lengths in words, widths, densities)."""

    lengths: np.ndarray  # uint64 words
    ks: np.ndarray       # int32 in {8, 16, 32}
    ps: np.ndarray       # float64 Bernoulli densities

    @property
    def nbytes(self) -> np.ndarray:
        return self.lengths * (self.ks.astype(np.uint64) // 8)


def loguniform_streams(m: int, max_log2: int, seed: int, min_len: int = 1) -> StreamSet:
    """m streams: L = clamp(round(exp(u * ln 2^max_log2)), min_len, 2^max_log2), u ~ U(0,1);
    k uniform over {8, 16, 32}; density p ~ U(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(m)
    lengths = np.clip(np.rint(np.exp(u * max_log2 * math.log(2.0))), min_len,
                      2.0**max_log2).astype(np.uint64)
    ks = rng.choice(np.array([8, 16, 32], dtype=np.int32), size=m)
    ps = rng.random(m)
    return StreamSet(lengths, ks, ps)


def poisson_arrivals(rate: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate on [0, duration)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_est = int(rate * duration_s * 1.2 + 100)
    gaps = rng.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate, size=n_est)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def batch_layout(lengths_bytes: np.ndarray, seed: int, align: int = 256,
                 max_offset: int = 16) -> tuple[np.ndarray, int]:
    """Place streams one after another in one arena: each starts at an `align`-byte
    boundary plus a seeded start offset in [0, max_offset).  Returns (start byte of
    every stream, arena size)."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5A5A))
    offs = rng.integers(0, max_offset, size=len(lengths_bytes)) if max_offset > 1 else \
        np.zeros(len(lengths_bytes), dtype=np.int64)
    slot = ((np.asarray(lengths_bytes, dtype=np.int64) + offs + align - 1) // align) * align
    slot = np.maximum(slot, align)
    starts = np.concatenate([[0], np.cumsum(slot)[:-1]]) + offs
    return starts.astype(np.int64), int(slot.sum())


def fill_streams(arena: np.ndarray, streams: StreamSet, starts: np.ndarray, seed: int,
                 threads: int | None = None):
    """Stream i: Bernoulli(ps[i]) bits of sub-stream i of `seed`, at arena[starts[i]:]."""
    nb = streams.nbytes
    for i in range(len(nb)):
        b = int(nb[i])
        if b:
            s = int(starts[i])
            fill(arena[s:s + b], Dist.bernoulli(float(streams.ps[i])), seed, stream=i,
                 threads=threads if b > (1 << 22) else 1)
    return arena


@dataclass
class RequestTrace:
    """A serving trace: arrival times (s), lengths (words), widths, the source pool
    of every request (pool index into `pools`) and its byte offset there."""

    arrival: np.ndarray
    lengths: np.ndarray
    ks: np.ndarray
    pool: np.ndarray
    offset: np.ndarray
    pools: list  # [(k, Dist)] in pool-index order

    @property
    def nbytes(self) -> np.ndarray:
        return self.lengths * (self.ks.astype(np.uint64) // 8)


def serving_trace(rate: float, duration_s: float, seed: int, min_log2: int = 10,
                  max_log2: int = 26, pool_bytes: int = 1 << 29,
                  zipf_s: float = 1.1) -> RequestTrace:
    """Poisson arrivals at `rate`; lengths log-uniform in [2^min_log2, 2^max_log2]
    words; k uniform over {8, 16, 32}; input one-hot Zipf(zipf_s) or Bernoulli(1/2)
    by a fair coin; each request reads a 256-byte aligned window of a pool of its
    (k, distribution), pool_bytes long."""
    t = poisson_arrivals(rate, duration_s, seed)
    m = len(t)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    u = rng.random(m)
    lengths = np.rint(np.exp((min_log2 + u * (max_log2 - min_log2)) * math.log(2.0)))
    lengths = lengths.astype(np.uint64)
    ks = rng.choice(np.array([8, 16, 32], dtype=np.int32), size=m)
    onehot = rng.random(m) < 0.5
    pools = [(k, Dist.onehot(k, zipf_s)) for k in (8, 16, 32)] + \
            [(k, Dist.uniform()) for k in (8, 16, 32)]
    pool = np.where(onehot, 0, 3) + np.searchsorted([8, 16, 32], ks)
    nb = lengths * (ks.astype(np.uint64) // 8)
    if int(nb.max(initial=0)) > pool_bytes:
        raise ValueError("pool smaller than the largest request")
    room = (pool_bytes - nb) // 256
    offset = (rng.integers(0, np.iinfo(np.int64).max, size=m) % (room + 1)) * 256
    return RequestTrace(t, lengths, ks, pool.astype(np.int32), offset.astype(np.uint64), pools)
