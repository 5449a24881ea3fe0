"""Python binding of the single-stream entry points (argument marshalling only).

torch supplies device memory and the stream; every step of the count runs in
the library's HIP kernels.  Counts are returned in int64 storage, which holds
the same bits as the library's uint64 counters for any total below 2^63.

`stream` is torch's current stream when None, else a torch.cuda.Stream or a raw
hipStream_t handle.  The caller orders the producers of the inputs (and of a
supplied `out`) before that stream, as for any asynchronous launch; an output
the binding allocates itself is ordered by the binding.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from ._lib import LaunchConfig, PpcError, check

VARIANTS = {"csa": L.VARIANT_CSA, "ballot": L.VARIANT_BALLOT, "hybrid": L.VARIANT_HYBRID}


def stream_handle(stream=None) -> int:
    """A hipStream_t as an int: torch's current stream when stream is None."""
    if stream is None:
        return torch._C._cuda_getCurrentRawStream(torch.cuda.current_device())
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _launch_on(stream, fresh, device: int | None = None) -> int:
    """The stream handle to launch on, on the current device (`device`: its index,
    when the caller already has it).  `fresh` is a tensor this binding has just
    filled on torch's current stream (None if the caller supplied the output): a
    launch on another stream first waits for that fill, and the tensor is marked as
    used by that stream, so that its memory is not handed out again before the
    launch ends."""
    if stream is None:
        # torch's current stream as a raw handle, without building a Stream object
        return torch._C._cuda_getCurrentRawStream(
            torch.cuda.current_device() if device is None else device)
    cur = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        if fresh is not None and stream != cur:
            stream.wait_stream(cur)
            fresh.record_stream(stream)
        return stream.cuda_stream
    handle = int(stream)
    if fresh is not None and handle != cur.cuda_stream:
        cur.synchronize()  # a raw handle: finish the fill before launching there
    return handle


def launch_config(variant="csa", depth=0, block_threads=0, blocks_per_cu=0, grid=0):
    if isinstance(variant, str):
        if variant not in VARIANTS:
            raise ValueError(f"variant must be one of {sorted(VARIANTS)}")
        variant = VARIANTS[variant]
    return LaunchConfig(variant, depth, block_threads, blocks_per_cu, grid)


def _device_bytes(x: torch.Tensor, byte_offset: int) -> int:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("input must be a tensor in GPU memory")
    if not x.is_contiguous():
        raise ValueError("input must be contiguous")
    avail = x.numel() * x.element_size() - byte_offset
    if byte_offset < 0 or avail < 0:
        raise ValueError("byte_offset outside the tensor")
    return avail


def _counts_tensor(out, k, device):
    """`device`: a torch.device or a CUDA device index."""
    if out is None:
        return torch.zeros(k, dtype=torch.int64, device=device)
    if out.dtype not in (torch.int64, torch.uint64) or out.numel() != k:
        raise ValueError(f"out must hold {k} int64 counters")
    index = device if isinstance(device, int) else device.index
    if not out.is_contiguous() or not out.is_cuda or out.get_device() != index:
        raise ValueError("out must be contiguous and on the input's device")
    return out


def pospopcnt_ptr(ptr: int, n: int, k: int, counts_ptr: int, stream=None, config=None) -> None:
    """Raw call: counts_ptr[p] += count of bit p over n k-bit words at device address ptr."""
    cfg = ctypes.byref(config) if config is not None else None
    st = L.lib().pospopcnt_ex(ptr or None, n, k, counts_ptr or None, stream_handle(stream), cfg)
    if st:
        raise PpcError(st, f"pospopcnt(k={k}, n={n})")


def pospopcnt(x: torch.Tensor, k: int, n: int | None = None, byte_offset: int = 0,
              out: torch.Tensor | None = None, stream=None, **config) -> torch.Tensor:
    """Positional population count of n k-bit little-endian words that start
    byte_offset bytes into x's memory (x: any dtype, read as bytes).

    Adds into `out` (k int64 counters on x's device; zeros when None) and returns it.
    Keyword arguments select a launch configuration (variant='csa'|'ballot'|'hybrid', depth,
    block_threads, blocks_per_cu, grid); every configuration gives the same counts."""
    if k not in (8, 16, 32, 64):
        raise ValueError("k must be 8, 16, 32 or 64")
    avail = _device_bytes(x, byte_offset)
    if n is None:
        n = avail // (k // 8)
    if n < 0 or n * (k // 8) > avail:
        raise ValueError(f"{n} words of {k} bits do not fit in {avail} bytes")
    dev = x.get_device()
    fresh = out is None
    out = _counts_tensor(out, k, dev)
    cfg = ctypes.byref(launch_config(**config)) if config else None
    cur = torch.cuda.current_device()
    if dev == cur:  # no device switch needed
        st = L.lib().pospopcnt_ex(x.data_ptr() + byte_offset, n, k, out.data_ptr(),
                                  _launch_on(stream, out if fresh else None, cur), cfg)
    else:
        with torch.cuda.device(dev):
            st = L.lib().pospopcnt_ex(x.data_ptr() + byte_offset, n, k, out.data_ptr(),
                                      _launch_on(stream, out if fresh else None), cfg)
    if st:
        raise PpcError(st, f"pospopcnt(k={k}, n={n})")
    return out


def pospopcnt_u8(x, n=None, byte_offset=0, out=None, stream=None):
    return pospopcnt(x, 8, n, byte_offset, out, stream)


def pospopcnt_u16(x, n=None, byte_offset=0, out=None, stream=None):
    return pospopcnt(x, 16, n, byte_offset, out, stream)


def pospopcnt_u32(x, n=None, byte_offset=0, out=None, stream=None):
    return pospopcnt(x, 32, n, byte_offset, out, stream)


def pospopcnt_u64(x, n=None, byte_offset=0, out=None, stream=None):
    return pospopcnt(x, 64, n, byte_offset, out, stream)


def pospopcnt_planes(planes, n: int | None = None, byte_offsets=None,
                     out: torch.Tensor | None = None, stream=None, **config) -> torch.Tensor:
    """Positional population count of words of 16*m bits held as m planes of 16-bit
    limbs (plane j holds every word's bits 16j .. 16j+15; the encoding of wider words
    as several 16-bit streams, Sec. 4).

    planes: a sequence of m GPU tensors (any dtype, read as bytes from byte_offsets[j])
    or a 2-D tensor whose m rows are the planes.  n defaults to the shortest plane's
    limb count.  Adds into `out` (16*m int64 counters) and returns it; out[16j + p]
    counts the words whose bit 16j + p is set."""
    if isinstance(planes, torch.Tensor):
        if planes.dim() != 2:
            raise ValueError("a tensor of planes must be 2-D (m rows)")
        planes = list(planes.unbind(0))
    planes = list(planes)
    m = len(planes)
    if not 1 <= m <= L.MAX_PLANES:
        raise ValueError(f"1 to {L.MAX_PLANES} planes")
    offs = [0] * m if byte_offsets is None else list(byte_offsets)
    avail = [_device_bytes(p, o) for p, o in zip(planes, offs)]
    if n is None:
        n = min(avail) // 2
    if n < 0 or any(2 * n > a for a in avail):
        raise ValueError(f"{n} limbs do not fit in every plane")
    dev = planes[0].device
    if any(p.device != dev for p in planes):
        raise ValueError("planes must be on one device")
    fresh = out is None
    out = _counts_tensor(out, 16 * m, dev)
    ptrs = (ctypes.c_void_p * m)(*[p.data_ptr() + o for p, o in zip(planes, offs)])
    cfg = launch_config(**config) if config else None
    with torch.cuda.device(dev):
        s = _launch_on(stream, out if fresh else None)
        check(L.lib().pospopcnt_planes16_ex(ptrs, m, n, out.data_ptr(), s,
                                            ctypes.byref(cfg) if cfg is not None else None),
              f"pospopcnt_planes16(m={m}, n={n})")
    return out


def read_ceiling(x: torch.Tensor, nbytes: int | None = None, byte_offset: int = 0,
                 sink: torch.Tensor | None = None, stream=None, **config) -> torch.Tensor:
    """Read-only bandwidth reference: XOR of all (zero-padded, aligned) dwords of the
    byte range, XORed into sink[0] (an int64 on the device)."""
    avail = _device_bytes(x, byte_offset)
    nbytes = avail if nbytes is None else nbytes
    if nbytes > avail:
        raise ValueError("range outside the tensor")
    fresh = sink is None
    if fresh:
        sink = torch.zeros(1, dtype=torch.int64, device=x.device)
    cfg = launch_config(**config) if config else None
    with torch.cuda.device(x.device):
        s = _launch_on(stream, sink if fresh else None)
        check(L.lib().ppc_read_ceiling(x.data_ptr() + byte_offset, nbytes, sink.data_ptr(), s,
                                       ctypes.byref(cfg) if cfg is not None else None),
              "ppc_read_ceiling")
    return sink


def histogram(ids: torch.Tensor, bins: int, id_bytes: int | None = None, n: int | None = None,
              byte_offset: int = 0, out: torch.Tensor | None = None, stream=None,
              **config) -> torch.Tensor:
    """Histogram of n categorical ids (u8 or u16, little-endian) starting byte_offset
    bytes into ids' memory, counted as the positional population count of their
    one-hot codes.  Adds into `out` (bins + 1 int64 counters: one per category and a
    last one for ids >= bins) and returns it.  id_bytes defaults to the tensor's
    element size (1 or 2)."""
    if not 1 <= bins <= 32:
        raise ValueError("bins must be 1 .. 32")
    id_bytes = id_bytes or ids.element_size()
    if id_bytes not in (1, 2):
        raise ValueError("ids are 1 or 2 bytes")
    avail = _device_bytes(ids, byte_offset)
    if n is None:
        n = avail // id_bytes
    if n < 0 or n * id_bytes > avail:
        raise ValueError(f"{n} ids of {id_bytes} bytes do not fit in {avail} bytes")
    fresh = out is None
    out = _counts_tensor(out, bins + 1, ids.device)
    cfg = launch_config(**config) if config else None
    with torch.cuda.device(ids.device):
        s = _launch_on(stream, out if fresh else None)
        check(L.lib().ppc_histogram_ex(ids.data_ptr() + byte_offset, n, id_bytes, bins,
                                       out.data_ptr(), s,
                                       ctypes.byref(cfg) if cfg is not None else None),
              f"ppc_histogram(bins={bins}, n={n})")
    return out


def device_info() -> dict:
    info = L.DeviceInfo()
    check(L.lib().ppc_get_device_info(ctypes.byref(info)), "ppc_get_device_info")
    return {"device": info.device, "compute_units": info.compute_units,
            "clock_khz": info.clock_khz, "l2_bytes": info.l2_bytes,
            "global_mem_bytes": info.global_mem_bytes, "name": info.name.decode(),
            "arch": info.arch.decode()}


__all__ = ["pospopcnt", "pospopcnt_u8", "pospopcnt_u16", "pospopcnt_u32", "pospopcnt_u64",
           "pospopcnt_planes", "pospopcnt_ptr",
           "read_ceiling", "histogram", "device_info", "launch_config", "stream_handle", "PpcError",
           "LaunchConfig"]
