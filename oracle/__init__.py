"""CPU oracle for the positional population count -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product (``paper_1911_02696_amd``) never does, and the
two share no code.

The oracle is the plain definition of the paper (Sec. 1 and Sec. 4, Fig. 3):
counts[p] = number of words whose bit p is set, for k-bit little-endian words at
any byte address, accumulated into 64-bit counters.  It also carries a model of
the Sec. 4.1 Harley-Seal algorithm (``hs16``) and the Sec. 2 carry-save adder
(``csa``), pinned by the tests against the paper's Table 2 and the plain
definition.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PPC_ORACLE_LIB names another build of the same source (the sanitizer run uses it).
LIB_PATH = os.environ.get("PPC_ORACLE_LIB") or os.path.join(_HERE, "libppc_oracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class Oracle:
    """ctypes view of one build of ppc_oracle.c (the normal one, or a planted variant)."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise FileNotFoundError(
                f"oracle library {path} is not built; run `python oracle/build.py`")
        lib = ctypes.CDLL(path)
        lib.ppc_oracle_count.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_int, _u64p]
        lib.ppc_oracle_count.restype = ctypes.c_int
        lib.ppc_oracle_count_mt.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_int, _u64p,
                                            ctypes.c_int]
        lib.ppc_oracle_count_mt.restype = ctypes.c_int
        lib.ppc_oracle_csa.argtypes = [ctypes.c_uint64] * 3 + [_u64p, _u64p]
        lib.ppc_oracle_csa.restype = None
        lib.ppc_oracle_hs16.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_int, _u64p, _u64p]
        lib.ppc_oracle_hs16.restype = ctypes.c_int
        lib.ppc_oracle_histogram.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                             _u64p]
        lib.ppc_oracle_histogram.restype = ctypes.c_int
        lib.ppc_oracle_count_planes.argtypes = [ctypes.POINTER(_u8p), ctypes.c_int,
                                                ctypes.c_uint64, _u64p]
        lib.ppc_oracle_count_planes.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    @staticmethod
    def _bytes(buf, n, k, offset):
        a = np.ascontiguousarray(np.frombuffer(buf, dtype=np.uint8) if not isinstance(
            buf, np.ndarray) else buf.view(np.uint8).reshape(-1))
        need = offset + n * (k // 8)
        if need > a.size:
            raise ValueError(f"buffer holds {a.size} bytes, {need} needed")
        return a, a.ctypes.data_as(_u8p) if a.size else ctypes.cast(0, _u8p)

    def count(self, buf, n: int, k: int, offset: int = 0, threads: int = 1,
              counts: np.ndarray = None) -> np.ndarray:
        """counts[p] += #{j < n : bit p of word j set}; word j = k/8 bytes at offset + j*k/8."""
        a, _ = self._bytes(buf, n, k, offset)
        out = np.zeros(k, dtype=np.uint64) if counts is None else counts
        if out.dtype != np.uint64 or out.size != k or not out.flags.c_contiguous:
            raise ValueError("counts must be a contiguous uint64 array of k entries")
        ptr = ctypes.cast(a.ctypes.data + offset, _u8p)
        cp = out.ctypes.data_as(_u64p)
        if threads == 1:
            rc = self.lib.ppc_oracle_count(ptr, n, k, cp)
        else:
            rc = self.lib.ppc_oracle_count_mt(ptr, n, k, cp, threads)
        if rc < 0:
            raise ValueError(f"oracle rejected k={k}")
        self.threads_used = 1 if threads == 1 else rc
        return out

    def csa(self, a: int, b: int, c: int):
        h, l = ctypes.c_uint64(), ctypes.c_uint64()
        self.lib.ppc_oracle_csa(a, b, c, ctypes.byref(h), ctypes.byref(l))
        return h.value, l.value

    def hs16(self, buf, n: int, N: int):
        """Sec. 4.1 model over n uint16 words with a 2^N-register circuit.

        Returns (counts[16], number of CSA evaluations)."""
        a, ptr = self._bytes(buf, n, 16, 0)
        out = np.zeros(16, dtype=np.uint64)
        calls = ctypes.c_uint64()
        rc = self.lib.ppc_oracle_hs16(ptr, n, N, out.ctypes.data_as(_u64p), ctypes.byref(calls))
        if rc < 0:
            raise ValueError(f"bad circuit size N={N}")
        return out, calls.value


    def histogram(self, buf, n: int, id_bytes: int, bins: int, offset: int = 0,
                  counts: np.ndarray = None) -> np.ndarray:
        """counts[c] += #{ids == c} (c < bins); counts[bins] += #{ids >= bins}."""
        a = np.ascontiguousarray(np.asarray(buf).view(np.uint8).reshape(-1))
        if offset + n * id_bytes > a.size:
            raise ValueError("ids outside the buffer")
        out = np.zeros(bins + 1, dtype=np.uint64) if counts is None else counts
        ptr = ctypes.cast(a.ctypes.data + offset, _u8p)
        if self.lib.ppc_oracle_histogram(ptr, n, id_bytes, bins, out.ctypes.data_as(_u64p)) < 0:
            raise ValueError("bad id width or bin count")
        return out

    def count_planes(self, planes, n: int, offsets=None, counts: np.ndarray = None) -> np.ndarray:
        """Words of 16*m bits held as m planes of n uint16 limbs (plane j = limb j):
        counts[16j + p] += #{words whose limb j has bit p set}.  planes: m byte buffers;
        plane j starts offsets[j] bytes into planes[j]."""
        m = len(planes)
        offsets = [0] * m if offsets is None else list(offsets)
        bufs = [np.ascontiguousarray(np.asarray(b).view(np.uint8).reshape(-1)) for b in planes]
        for b, o in zip(bufs, offsets):
            if o + 2 * n > b.size:
                raise ValueError("plane shorter than n limbs")
        ptrs = (_u8p * max(m, 1))(*[ctypes.cast(b.ctypes.data + o, _u8p)
                                    for b, o in zip(bufs, offsets)])
        out = np.zeros(16 * m, dtype=np.uint64) if counts is None else counts
        if self.lib.ppc_oracle_count_planes(ptrs, m, n, out.ctypes.data_as(_u64p)) < 0:
            raise ValueError("plane count must be 1..64")
        return out


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def count(buf, n, k, offset=0, threads=1, counts=None):
    return get().count(buf, n, k, offset=offset, threads=threads, counts=counts)
