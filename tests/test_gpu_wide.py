"""GPU parity of the wide-word paths against the CPU oracle (tolerance 0): 64-bit
words in one stream, and words of 16*m bits held as m planes of 16-bit limbs
(Sec. 4).  Expected values come only from the oracle on the same host bytes."""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import api
from paper_1911_02696_amd import inputs as I

import oracle
from gpu_util import counts_np, host_bytes, oracle_counts, say, to_device

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 7


def _lengths64():
    # a k = 64 tile is 64 lanes x 16 dwords = 4096 bytes = 512 words at depth 16
    small = [0, 1, 2, 3, 5, 7, 8, 15, 16, 17, 31, 33, 63, 64, 65, 255, 256, 257]
    tiles = [b // 8 + d for b in (4096, 8192, 16384, 65536, 1 << 20) for d in (-1, 0, 1)]
    return sorted(set(small + tiles + [12345, 100003]))


def test_k64_lengths_and_offsets():
    lengths = _lengths64()
    host = host_bytes(max(lengths) * 8, I.Dist.uniform(), SEED)
    expect = {n: oracle_counts(host, n, 64) for n in lengths}
    for off in range(16):
        say(f"k=64 offset={off} lengths={lengths[0]}..{lengths[-1]}")
        buf, o = to_device(host, off)
        for n in lengths:
            got = counts_np(api.pospopcnt(buf, 64, n=n, byte_offset=o))
            assert (got == expect[n]).all(), f"offset={off} n={n}"


@pytest.mark.parametrize("cfg", [
    dict(depth=4), dict(depth=8), dict(depth=16), dict(depth=32), dict(block_threads=64),
    dict(block_threads=128), dict(grid=1), dict(grid=7), dict(blocks_per_cu=3),
    dict(depth=4, grid=3, block_threads=64),
    dict(depth=32, grid=3, block_threads=64),
], ids=lambda c: "-".join(f"{a}{b}" for a, b in c.items()))
def test_k64_launch_configs_agree(cfg):
    n = 3_000_017 // 8
    host = host_bytes(n * 8, I.Dist.bernoulli(0.3), SEED + 1)
    expect = oracle_counts(host, n, 64)
    for off in (0, 3, 12):
        say(f"k=64 config {cfg} offset={off} n={n}")
        buf, o = to_device(host, off)
        got = counts_np(api.pospopcnt(buf, 64, n=n, byte_offset=o, **cfg))
        assert (got == expect).all(), (cfg, off)


def test_k64_one_hot_and_constants():
    """One-hot 64-bit words over every bit and all-ones words: closed forms."""
    n = 64 * 40_003
    words = (np.uint64(1) << (np.arange(n, dtype=np.uint64) % np.uint64(64))).astype(np.uint64)
    for off in (0, 1, 4, 9):
        say(f"k=64 one-hot offset={off}")
        buf, o = to_device(words.view(np.uint8), off)
        got = counts_np(api.pospopcnt_u64(buf, n=n, byte_offset=o))
        assert (got == n // 64).all(), off
    ones = torch.full((8 * 123_457 + 5,), 255, dtype=torch.uint8, device="cuda")
    got = counts_np(api.pospopcnt(ones, 64, n=123_457, byte_offset=5))
    assert (got == 123_457).all()


def test_k64_folds_to_k32_and_accumulates():
    """Bits p and p + 32 of the 64-bit words are bit p of the 32-bit words of the
    same bytes; and counting two pieces into one vector equals counting the whole."""
    n = 1_000_003
    host = host_bytes(n * 8, I.Dist.bernoulli(0.7), SEED + 2)
    buf, o = to_device(host, 8)
    c64 = counts_np(api.pospopcnt(buf, 64, n=n, byte_offset=o))
    c32 = counts_np(api.pospopcnt(buf, 32, n=2 * n, byte_offset=o))
    assert (c64[:32] + c64[32:] == c32).all()
    out = torch.zeros(64, dtype=torch.int64, device="cuda")
    api.pospopcnt(buf, 64, n=400_001, byte_offset=o, out=out)
    api.pospopcnt(buf, 64, n=n - 400_001, byte_offset=o + 8 * 400_001, out=out)
    assert (counts_np(out) == c64).all()


def test_k64_large_sampled():
    """2^29 + 12,345 words (4 GiB) at offsets 0 and 5, against the oracle in full."""
    n = (1 << 29) + 12_345
    host = host_bytes(n * 8, I.Dist.uniform(), SEED + 3)
    expect = oracle_counts(host, n, 64, threads=I.default_threads())
    for off in (0, 5):
        say(f"k=64 large n={n} offset={off}")
        buf, o = to_device(host, off, pad=16)
        got = counts_np(api.pospopcnt_u64(buf, n=n, byte_offset=o))
        assert (got == expect).all(), off
        del buf
        torch.cuda.empty_cache()


# ---------------------------------------------------------------- 16-bit planes

def _planes_host(m, n, seed):
    return [host_bytes(2 * n, I.Dist.bernoulli(0.1 + 0.8 * j / max(m - 1, 1)), seed + j)
            for j in range(m)]


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 8, 32])
def test_planes_against_oracle(m):
    lengths = [0, 1, 7, 8, 9, 2047, 2048, 2049, 100_003]
    hosts = _planes_host(m, max(lengths), SEED + 10 * m)
    for n in lengths:
        exp = oracle.get().count_planes(hosts, n).astype(np.int64)
        # each plane at its own start offset (0..15)
        offs = [(3 * j + n) % 16 for j in range(m)]
        say(f"planes m={m} n={n} offsets={offs[:4]}...")
        bufs = [to_device(h, o) for h, o in zip(hosts, offs)]
        got = counts_np(api.pospopcnt_planes([b for b, _ in bufs], n=n,
                                             byte_offsets=[o for _, o in bufs]))
        assert (got == exp).all(), (m, n)


def test_planes_equal_interleaved_words():
    """The limbs of 64-bit words as 4 planes count exactly like the words."""
    n = 777_777
    host = host_bytes(8 * n, I.Dist.uniform(), SEED + 20)
    limbs = host.view(np.uint16).reshape(n, 4)
    planes = torch.from_numpy(np.ascontiguousarray(limbs.T)).cuda()  # 4 rows
    words, o = to_device(host, 0)
    say(f"planes vs words n={n}")
    got = counts_np(api.pospopcnt_planes(planes))
    assert (got == counts_np(api.pospopcnt_u64(words, n=n, byte_offset=o))).all()
    assert (got == oracle_counts(host, n, 64)).all()


@pytest.mark.parametrize("cfg", [dict(depth=4), dict(depth=8), dict(depth=32),
                                 dict(block_threads=64),
                                 dict(grid=1), dict(grid=5), dict(blocks_per_cu=4)],
                         ids=lambda c: "-".join(f"{a}{b}" for a, b in c.items()))
def test_planes_launch_configs_agree(cfg):
    m, n = 6, 500_009
    hosts = _planes_host(m, n, SEED + 30)
    exp = oracle.get().count_planes(hosts, n).astype(np.int64)
    bufs = [to_device(h, 2 * j + 1) for j, h in enumerate(hosts)]
    say(f"planes config {cfg}")
    got = counts_np(api.pospopcnt_planes([b for b, _ in bufs], n=n,
                                         byte_offsets=[o for _, o in bufs], **cfg))
    assert (got == exp).all(), cfg


def test_planes_large():
    """4 planes of 2^28 + 3 limbs (2 GiB in all); expected from the plain definition
    per plane (the oracle's count, threaded), which is what a plane means."""
    m, n = 4, (1 << 28) + 3
    hosts = _planes_host(m, n, SEED + 40)
    exp = np.concatenate([oracle_counts(h, n, 16, threads=I.default_threads()) for h in hosts])
    bufs = [to_device(h, 2 * j, pad=16) for j, h in enumerate(hosts)]
    say(f"planes large m={m} n={n}")
    got = counts_np(api.pospopcnt_planes([b for b, _ in bufs], n=n,
                                         byte_offsets=[o for _, o in bufs]))
    assert (got == exp).all()


@pytest.mark.timeout(900)
def test_full_size_benchmark_workloads():
    """The benchmark's wide cases at full size in their default launch shapes, against
    the oracle over all 16 GiB: one stream of 2^31 64-bit words, then the same bytes
    as 4 planes of 2^31 16-bit limbs (4 GiB each; plane j counted by the plain
    definition into counters 16j .. 16j+15)."""
    nbytes = 1 << 34
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (1 << 30):
        pytest.skip(f"needs {nbytes >> 30} GiB of free device memory")
    say("wide 16 GiB: generating")
    host = np.empty(nbytes, np.uint8)
    chunk = 1 << 30
    dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    pinned = torch.empty(chunk, dtype=torch.uint8).pin_memory()
    for first in range(0, nbytes, chunk):
        I.fill(host[first:first + chunk], I.Dist.uniform(), SEED + 50, first_byte=first)
        pinned.numpy()[:] = host[first:first + chunk]
        dev[first:first + chunk].copy_(pinned, non_blocking=False)
    n = nbytes // 8
    say("wide 16 GiB: k = 64")
    got = counts_np(api.pospopcnt_u64(dev, n=n))
    assert (got == oracle_counts(host, n, 64, threads=I.default_threads())).all()
    m, per = 4, nbytes // 4
    say("wide 16 GiB: 4 planes")
    got = counts_np(api.pospopcnt_planes([dev[j * per:(j + 1) * per] for j in range(m)]))
    exp = np.concatenate([oracle_counts(host[j * per:(j + 1) * per], per // 2, 16,
                                        threads=I.default_threads()) for j in range(m)])
    assert (got == exp).all()
    del dev
    torch.cuda.empty_cache()
