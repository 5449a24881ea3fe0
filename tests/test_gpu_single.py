"""GPU parity of the single-stream path against the CPU oracle (tolerance 0).

Inputs are seeded synthetic bytes (paper_1911_02696_amd.inputs); expected values
come only from the oracle run on the same host bytes.  Every start offset 0..15
is reached by placing the same bytes at that offset in device memory, so one
oracle run serves all offsets (the oracle's own alignment invariant is pinned
in test_oracle_pins.py).
"""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import api
from paper_1911_02696_amd import inputs as I

from gpu_util import counts_np, host_bytes, oracle_counts, say, to_device

pytestmark = pytest.mark.gpu

KS = (8, 16, 32)
SEED = I.BASE_SEED


def _lengths(k):
    wb = k // 8
    small = [0, 1, 2, 3, 5, 7, 8, 15, 16, 17, 31, 33, 63, 64, 65, 255, 256, 257]
    tiles = [b // wb + d for b in (4096, 8192, 16384, 65536, 1 << 20) for d in (-1, 0, 1)]
    return sorted(set(small + tiles + [12345, 100003]))


@pytest.mark.parametrize("k", KS)
def test_lengths_and_offsets(k):
    """n = 0, 1, 2, ..., tile - 1, tile, tile + 1, ... at every start offset 0..15."""
    wb = k // 8
    lengths = _lengths(k)
    host = host_bytes(max(lengths) * wb, I.Dist.uniform(), SEED + k)
    expect = {n: oracle_counts(host, n, k) for n in lengths}
    for off in range(16):
        say(f"single k={k} offset={off} lengths={lengths[0]}..{lengths[-1]}")
        buf, o = to_device(host, off)
        for n in lengths:
            got = counts_np(api.pospopcnt(buf, k, n=n, byte_offset=o))
            assert (got == expect[n]).all(), f"k={k} offset={off} n={n}"


@pytest.mark.parametrize("k", KS)
@pytest.mark.parametrize("cfg", [
    dict(variant="csa", depth=4), dict(variant="csa", depth=8), dict(variant="csa", depth=16),
    dict(variant="csa", depth=32), dict(variant="csa", depth=4, block_threads=64, grid=5),
    dict(variant="ballot"), dict(variant="hybrid", depth=4), dict(variant="hybrid", depth=8),
    dict(variant="hybrid", depth=16),
    dict(variant="hybrid", depth=32, block_threads=64), dict(block_threads=64),
    dict(block_threads=128),
    dict(grid=1), dict(grid=7), dict(blocks_per_cu=1), dict(depth=32, grid=3, block_threads=64),
], ids=lambda c: "-".join(f"{a}{b}" for a, b in c.items()))
def test_launch_configs_agree(k, cfg):
    """Every variant, circuit depth, block size and grid gives the oracle's counts."""
    wb = k // 8
    n = 3_000_017 // wb
    host = host_bytes(n * wb, I.Dist.bernoulli(0.3), SEED + 100 + k)
    expect = oracle_counts(host, n, k)
    for off in (0, 3, 13):
        say(f"config {cfg} k={k} offset={off} n={n}")
        buf, o = to_device(host, off)
        got = counts_np(api.pospopcnt(buf, k, n=n, byte_offset=o, **cfg))
        assert (got == expect).all(), f"{cfg} k={k} offset={off}"
        for m in (1, 5, 4095, 65537):  # short inputs take the edge and partial-tile paths
            got = counts_np(api.pospopcnt(buf, k, n=m, byte_offset=o, **cfg))
            assert (got == oracle_counts(host, m, k)).all(), f"{cfg} k={k} off={off} n={m}"


def test_c1_worked_size():
    """2^20 uint16 words: Bernoulli(0.5) bits and one-hot words (16 categories, uniform)."""
    n = 1 << 20
    for dist in (I.Dist.uniform(), I.Dist.onehot(16)):
        host = host_bytes(2 * n, dist, SEED + 0)
        say(f"C1 dist={dist}")
        buf, o = to_device(host, 0)
        got = counts_np(api.pospopcnt_u16(buf, n=n))
        assert (got == oracle_counts(host, n, 16)).all()
        if dist.kind == I.ONEHOT:
            assert got.sum() == n


def test_country_example_on_gpu():
    stream = np.array([0x10, 0x10, 0x04, 0x10, 0x01, 0x04, 0x01, 0x01, 0x01, 0x20], np.uint8)
    buf, _ = to_device(stream, 5)
    got = counts_np(api.pospopcnt_u8(buf, n=10, byte_offset=5))
    assert got.tolist() == [4, 0, 2, 0, 3, 1, 0, 0]


def test_accumulate_and_split():
    """Counts are added into; counting two pieces into one vector = counting the whole."""
    k, n = 16, 777_777
    host = host_bytes(2 * n, I.Dist.uniform(), SEED + 7)
    expect = oracle_counts(host, n, 16)
    buf, _ = to_device(host, 1)
    seeded = torch.arange(16, dtype=torch.int64, device="cuda") * 1_000_000
    out = api.pospopcnt(buf, k, n=n, byte_offset=1, out=seeded.clone())
    assert (counts_np(out) == expect + np.arange(16) * 1_000_000).all()
    for split in (0, 1, 2047, 2048, 2049, 300_001, n):
        out = torch.zeros(16, dtype=torch.int64, device="cuda")
        api.pospopcnt(buf, k, n=split, byte_offset=1, out=out)
        api.pospopcnt(buf, k, n=n - split, byte_offset=1 + 2 * split, out=out)
        assert (counts_np(out) == expect).all(), f"split {split}"


def test_run_to_run_identical_and_concurrent_streams():
    k, n = 32, 5_000_001
    host = host_bytes(4 * n, I.Dist.bernoulli(0.7), SEED + 9)
    expect = oracle_counts(host, n, k)
    buf, _ = to_device(host, 2)
    runs = [counts_np(api.pospopcnt(buf, k, n=n, byte_offset=2)) for _ in range(5)]
    for r in runs:
        assert (r == expect).all()
    # two streams adding into the same counters at once
    out = torch.zeros(k, dtype=torch.int64, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        api.pospopcnt(buf, k, n=n, byte_offset=2, out=out, stream=s1)
        api.pospopcnt(buf, k, n=n, byte_offset=2, out=out, stream=s2)
    torch.cuda.synchronize()
    assert (counts_np(out) == 6 * expect).all()


def test_side_stream_without_out():
    """A launch on another stream without `out`: the zeroed counters the binding
    allocates on the current stream are ready before the count adds into them,
    also while the current stream is still busy."""
    k, n = 16, 4_000_037
    host = host_bytes(2 * n, I.Dist.bernoulli(0.6), SEED + 12)
    expect = oracle_counts(host, n, k)
    buf, o = to_device(host, 3)
    side = torch.cuda.Stream()
    busy = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for _ in range(3):
        busy.fill_(1)  # keeps the current stream occupied while the side launch is queued
        got = api.pospopcnt(buf, k, n=n, byte_offset=o, stream=side)
        side.synchronize()
        assert (counts_np(got) == expect).all()
        got = api.pospopcnt(buf, k, n=n, byte_offset=o, stream=side.cuda_stream)
        side.synchronize()
        assert (counts_np(got) == expect).all()
    torch.cuda.synchronize()


def test_zero_length_launches_nothing():
    out = torch.full((16,), 5, dtype=torch.int64, device="cuda")
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    api.pospopcnt(buf, 16, n=0, out=out)
    assert (counts_np(out) == 5).all()


def test_read_ceiling_xor():
    """The bandwidth-reference kernel XORs every (zero-padded, aligned) dword."""
    for nbytes, off in ((1 << 20, 0), ((1 << 20) + 13, 3), (7, 9), (100_000, 15)):
        host = host_bytes(nbytes, I.Dist.uniform(), SEED + 11)
        buf, o = to_device(host, off)
        padded = np.zeros(((off + nbytes + 3) // 4) * 4, np.uint8)
        padded[off:off + nbytes] = host
        expect = int(np.bitwise_xor.reduce(padded.view(np.uint32)))
        got = int(api.read_ceiling(buf, nbytes=nbytes, byte_offset=o).cpu()[0]) & 0xFFFFFFFF
        assert got == expect, (nbytes, off)


@pytest.mark.parametrize("k", KS)
def test_c2_full_size(k):
    """n = 2^28 - 1237 words (odd, not a multiple of 4096) of each width, in the three
    bit distributions, at start offsets 0, 1, 2, 3, 7 and 15."""
    n = (1 << 28) - 1237
    wb = k // 8
    dists = [I.Dist.uniform(), I.Dist.bernoulli(0.02), I.Dist.onehot(k, 1.1)]
    for d_i, dist in enumerate(dists):
        say(f"C2 k={k} dist={dist} n={n}: generating")
        host = host_bytes(n * wb, dist, SEED + 1 + 10 * d_i + k)
        expect = oracle_counts(host, n, k)
        if dist.kind == I.ONEHOT:
            assert expect.sum() == n
        master = torch.from_numpy(host).cuda()
        buf = torch.empty(n * wb + 64, dtype=torch.uint8, device="cuda")
        for off in (0, 1, 2, 3, 7, 15):
            say(f"C2 k={k} dist={dist} offset={off}")
            buf[off:off + n * wb].copy_(master)
            got = counts_np(api.pospopcnt(buf, k, n=n, byte_offset=off))
            assert (got == expect).all(), f"k={k} {dist} offset={off}"
        del master, buf
        torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_c3_full_size_roofline_config():
    """2^33 uint16 words (16 GiB) at offset 0 in the launch configuration the
    benchmark times, against the oracle over all 16 GiB."""
    n = 1 << 33
    nbytes = 2 * n
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (1 << 30):
        pytest.skip(f"needs {nbytes >> 30} GiB of free device memory")
    say("C3 n=2^33 u16: generating")
    host = np.empty(nbytes, np.uint8)
    chunk = 1 << 30
    dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    pinned = torch.empty(chunk, dtype=torch.uint8).pin_memory()
    for first in range(0, nbytes, chunk):
        I.fill(host[first:first + chunk], I.Dist.uniform(), SEED + 2, first_byte=first)
        pinned.numpy()[:] = host[first:first + chunk]
        dev[first:first + chunk].copy_(pinned, non_blocking=False)
    say("C3: kernel")
    got = counts_np(api.pospopcnt_u16(dev, n=n))
    say("C3: oracle")
    expect = oracle_counts(host, n, 16)
    assert (got == expect).all()
    assert got.sum() == int(np.bitwise_count(host.view(np.uint64)).sum())
