"""GPU parity of the one-hot histogram: counts of u8/u16 category ids equal the
oracle's histogram (tolerance 0), and equal encoding the ids as one-hot words and
counting those with pospopcnt."""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import api
from paper_1911_02696_amd import inputs as I

import oracle
from gpu_util import counts_np, say, to_device

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 6


def expected(host, n, id_bytes, bins, offset=0):
    return oracle.get().histogram(host, n, id_bytes, bins, offset=offset).astype(np.int64)


@pytest.mark.parametrize("id_bytes", [1, 2])
@pytest.mark.parametrize("bins", [8, 16, 32])
def test_histogram_lengths_offsets(id_bytes, bins):
    lengths = [0, 1, 2, 3, 7, 8, 15, 16, 17, 31, 33, 63, 64, 65, 1023, 1024, 1025,
               4095, 4096, 4097, 16383, 16385, 100003]
    host = I.generate(max(lengths) * id_bytes, I.Dist.ids(8 * id_bytes, bins, 1.1, 0.03), SEED)
    for off in range(0, 16, id_bytes):
        say(f"histogram id_bytes={id_bytes} bins={bins} offset={off}")
        buf, o = to_device(host, off)
        for n in lengths:
            got = counts_np(api.histogram(buf, bins, id_bytes=id_bytes, n=n, byte_offset=o))
            assert (got == expected(host, n, id_bytes, bins)).all(), (id_bytes, bins, off, n)


@pytest.mark.parametrize("id_bytes", [1, 2])
def test_histogram_equals_encode_then_count(id_bytes):
    """The fused path equals writing the one-hot words and counting them."""
    n = 1_000_003
    for bins, k in ((8, 8), (16, 16), (32, 32)):
        host = I.generate(n * id_bytes, I.Dist.ids(8 * id_bytes, bins), SEED + bins)
        ids = torch.from_numpy(host).cuda()
        hist = counts_np(api.histogram(ids, bins, id_bytes=id_bytes))
        idv = host.view(np.uint8 if id_bytes == 1 else np.uint16).astype(np.uint64)
        words = (np.uint64(1) << idv).astype({8: np.uint8, 16: np.uint16, 32: np.uint32}[k])
        enc = counts_np(api.pospopcnt(torch.from_numpy(words.view(np.uint8)).cuda(), k))
        assert (hist[:bins] == enc[:bins]).all() and hist[bins] == 0


def test_histogram_all_invalid_and_configs():
    n = 300_007
    host = I.generate(n, I.Dist.ids(8, 8, None, 1.0), SEED + 1)  # every id >= 8
    got = counts_np(api.histogram(torch.from_numpy(host).cuda(), 8))
    assert (got[:8] == 0).all() and got[8] == n
    host = I.generate(2 * n, I.Dist.ids(16, 32, 1.1, 0.1), SEED + 2)
    exp = expected(host, n, 2, 32)
    buf, o = to_device(host, 2)
    for cfg in (dict(block_threads=64), dict(blocks_per_cu=1), dict(grid=3), dict(grid=1)):
        got = counts_np(api.histogram(buf, 32, id_bytes=2, n=n, byte_offset=o, **cfg))
        assert (got == exp).all(), cfg


def test_country_example_as_ids():
    ids = np.array([4, 4, 2, 4, 0, 2, 0, 0, 0, 5], np.uint8)  # France, ..., China
    buf, o = to_device(ids, 3)
    got = counts_np(api.histogram(buf, 8, n=10, byte_offset=o))
    assert got.tolist() == [4, 0, 2, 0, 3, 1, 0, 0, 0]


@pytest.mark.parametrize("id_bytes", [1, 2])
@pytest.mark.parametrize("bins", [8, 16, 32])
def test_histogram_rare_wide_invalid(id_bytes, bins):
    """Rare ids drawn over the whole id range (every high bit pattern, 0xFF and 0xFFFF
    included) among valid ones: some tiles hold none, some one or a few, so tiles take
    both the all-valid and the masked code paths within one launch."""
    n = 2_000_003
    dt = np.uint8 if id_bytes == 1 else np.uint16
    ids = I.generate(n * id_bytes, I.Dist.ids(8 * id_bytes, bins, 1.1), SEED + 10 + bins).view(dt)
    wide = I.generate(n * id_bytes, I.Dist.uniform(), SEED + 20 + bins).view(dt)
    pick = I.generate(2 * n, I.Dist.uniform(), SEED + 30 + bins).view(np.uint16) < 3
    ids = np.where(pick, wide, ids).astype(dt)
    ids[[5, n // 2, n - 1]] = np.array([0xFF, 0x80, bins], np.uint64).astype(dt)
    if id_bytes == 2:
        ids[[7, n // 3]] = [0xFFFF, 0x8000 | 3]
    host = ids.view(np.uint8)
    say(f"histogram rare wide invalid id_bytes={id_bytes} bins={bins} invalid={int((ids >= bins).sum())}")
    exp = expected(host, n, id_bytes, bins)
    assert 0 < exp[bins] < n // 1000
    for off in (0, 2, 6):
        buf, o = to_device(host, off)
        got = counts_np(api.histogram(buf, bins, id_bytes=id_bytes, n=n, byte_offset=o))
        assert (got == exp).all(), (id_bytes, bins, off)


@pytest.mark.parametrize("bins", [8, 16, 32])
def test_constant_ids_closed_form(bins):
    """Every u8 id value, and u16 values around each boundary, as a constant stream
    with a ragged length and an unaligned start.  Closed form: all n ids fall in the
    one class of the id, or all outside the categories.  For u8 ids and 8 categories
    this covers every byte-table form an id >= 8 takes (no code, or a code in every
    class that is taken back)."""
    n = 70_001
    buf = torch.empty(2 * n + 16, dtype=torch.uint8, device="cuda")
    for v in range(256):
        buf.fill_(v)
        got = counts_np(api.histogram(buf, bins, n=n, byte_offset=3))
        exp = np.zeros(bins + 1, np.int64)
        exp[min(v, bins)] = n
        assert (got == exp).all(), ("u8", bins, v, got)
    say(f"constant u8 ids bins={bins}: 256 values")
    # around each boundary, plus high bytes 8..12 over valid low bytes (for 8
    # categories a high byte of 12 is the selector the mask table must not meet)
    extra = [11, 12, 13, 255, 256, 257, 0x0800 | 2, 0x0B00 | 1, 0x0C00, 0x0C00 | 5, 0x0D00,
             0x7FFF, 0x8000, 0x8000 | 3, 0xFFFF]
    for v in list(range(bins + 2)) + extra:
        buf.view(torch.int16)[: n + 8].fill_(v - 65536 if v >= 32768 else v)
        got = counts_np(api.histogram(buf, bins, id_bytes=2, n=n, byte_offset=2))
        exp = np.zeros(bins + 1, np.int64)
        exp[min(v, bins)] = n
        assert (got == exp).all(), ("u16", bins, v, got)


@pytest.fixture(scope="module")
def ids_16gib():
    buf = torch.empty(1 << 34, dtype=torch.uint8, device="cuda")
    yield buf
    del buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("id_bytes,bins,p_invalid", [
    (1, 8, 0.0), (1, 16, 0.0), (1, 32, 0.0), (2, 8, 0.0), (2, 16, 0.0), (2, 32, 0.0),
    (1, 8, 0.01), (2, 16, 0.01)])
def test_full_size_benchmark_workload(ids_16gib, id_bytes, bins, p_invalid):
    """The benchmark's 16 GiB cases in its launch configuration (the defaults): one
    GiB of Zipf(1.1) ids generated and repeated 16 times, so the exact histogram is
    16 times the oracle's histogram of that GiB."""
    gen = 1 << 30
    host = I.generate(gen, I.Dist.ids(8 * id_bytes, bins, 1.1, p_invalid), SEED + 40 + bins)
    exp = 16 * expected(host, gen // id_bytes, id_bytes, bins)
    say(f"histogram 16 GiB id_bytes={id_bytes} bins={bins} p_invalid={p_invalid}")
    ids_16gib[:gen].copy_(torch.from_numpy(host))
    for c in range(1, 16):
        ids_16gib[c * gen:(c + 1) * gen].copy_(ids_16gib[:gen])
    got = counts_np(api.histogram(ids_16gib, bins, id_bytes=id_bytes))
    assert (got == exp).all(), (id_bytes, bins, p_invalid)
    assert got.sum() == (1 << 34) // id_bytes


@pytest.mark.parametrize("id_bytes", [1, 2])
@pytest.mark.parametrize("bins", [1, 3, 7, 9, 13, 17, 24, 31])
def test_histogram_any_bin_count(id_bytes, bins):
    """Category counts that are not a code width: the ids in [bins, code bits) have a
    code but no category and must be counted as outside (the generator draws ids
    outside the categories as bins .. bins + 6, exactly that range)."""
    lengths = [1, 15, 16, 17, 4097, 100_003]
    host = I.generate(max(lengths) * id_bytes, I.Dist.ids(8 * id_bytes, bins, 1.1, 0.1),
                      SEED + 60 + bins)
    for off in (0, 2, 5) if id_bytes == 1 else (0, 2, 6):
        say(f"histogram any bins id_bytes={id_bytes} bins={bins} offset={off}")
        buf, o = to_device(host, off)
        for n in lengths:
            got = counts_np(api.histogram(buf, bins, id_bytes=id_bytes, n=n, byte_offset=o))
            assert (got == expected(host, n, id_bytes, bins)).all(), (id_bytes, bins, off, n)


@pytest.mark.parametrize("bins", [1, 5, 12, 20])
def test_constant_ids_any_bin_count(bins):
    """Closed form for bin counts that are not a code width: a constant stream of id v
    falls in class v when v < bins and outside otherwise, also for v between bins and
    the code width."""
    n = 70_001
    buf = torch.empty(n + 16, dtype=torch.uint8, device="cuda")
    for v in list(range(40)) + [127, 255]:
        buf.fill_(v)
        got = counts_np(api.histogram(buf, bins, n=n, byte_offset=3))
        exp = np.zeros(bins + 1, np.int64)
        exp[min(v, bins)] = n
        assert (got == exp).all(), (bins, v, got)
