"""GPU parity of the batched path: every stream of a mixed batch equals the CPU
oracle on the same host bytes (tolerance 0), for every launch configuration,
with and without graph replay, and equals the one-launch-per-stream form."""
import os

import numpy as np
import pytest
import torch

from paper_1911_02696_amd import batch as B
from paper_1911_02696_amd import inputs as I

from gpu_util import oracle_counts, say

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 3


class Batch:
    """Streams laid out in one device arena, counts in one (m, 32) int64 table."""

    def __init__(self, streams: I.StreamSet, seed: int, max_offset=16, threads=None):
        self.streams = streams
        nb = streams.nbytes.astype(np.int64)
        self.starts, size = I.batch_layout(nb, seed, max_offset=max_offset)
        self.host = np.zeros(size + 64, np.uint8)
        I.fill_streams(self.host, streams, self.starts, seed, threads=threads)
        self.dev = torch.from_numpy(self.host).cuda()
        m = len(nb)
        self.m = m
        self.counts = torch.zeros((m, 32), dtype=torch.int64, device="cuda")
        base = self.dev.data_ptr()
        self.desc_host = B.descriptors(base + self.starts, streams.lengths, streams.ks,
                                       self.counts.data_ptr() + 256 * np.arange(m))
        self.descs = B.to_device(self.desc_host)

    def expected(self, i):
        k = int(self.streams.ks[i])
        n = int(self.streams.lengths[i])
        s = int(self.starts[i])
        return oracle_counts(self.host[s:s + n * k // 8], n, k)

    def check(self, factor=1, which=None):
        got = self.counts.cpu().numpy()
        for i in (range(self.m) if which is None else which):
            k = int(self.streams.ks[i])
            exp = self.expected(i) * factor
            assert (got[i, :k] == exp).all(), f"stream {i}: n={self.streams.lengths[i]} k={k}"
            assert (got[i, k:] == 0).all(), f"stream {i} wrote past its k counters"


def mixed(m, max_log2, seed, min_len=0):
    s = I.loguniform_streams(m, max_log2, seed, min_len=min_len)
    return s


@pytest.fixture(scope="module")
def small_batch():
    s = mixed(600, 17, SEED)
    # force some empty, one-word and edge-only streams
    s.lengths[:5] = 0
    s.lengths[5:10] = 1
    s.lengths[10:20] = np.arange(2, 12)
    return Batch(s, SEED)


def test_batch_matches_oracle(small_batch):
    b = small_batch
    b.counts.zero_()
    plan = B.Plan(b.m)
    say("batch: default config")
    plan.run(b.descs)
    torch.cuda.synchronize()
    b.check()
    assert plan.rejected() == 0
    plan.run(b.descs)  # accumulate
    torch.cuda.synchronize()
    b.check(factor=2)


@pytest.mark.parametrize("cfg", [
    dict(depth=4, block_threads=64, blocks_per_cu=16, stream_weight=2048),
    dict(depth=4, block_threads=256, blocks_per_cu=2, stream_weight=3),
    dict(depth=8, block_threads=64, blocks_per_cu=6, stream_weight=4096),
    dict(depth=8, block_threads=128, blocks_per_cu=1, stream_weight=1),
    dict(depth=16, block_threads=64, blocks_per_cu=1, stream_weight=1),
    dict(depth=16, block_threads=256, blocks_per_cu=16, stream_weight=65536),
    dict(depth=32, block_threads=128, blocks_per_cu=3, stream_weight=17),
    dict(depth=32, block_threads=256, blocks_per_cu=1, stream_weight=1024),
    dict(depth=32, block_threads=64, blocks_per_cu=8, stream_weight=256),
], ids=lambda c: "d{depth}-t{block_threads}-b{blocks_per_cu}-w{stream_weight}".format(**c))
def test_batch_configs_agree(small_batch, cfg):
    b = small_batch
    b.counts.zero_()
    plan = B.Plan(b.m)
    plan.config = cfg
    assert plan.config == cfg
    say(f"batch config {cfg}")
    plan.run(b.descs)
    torch.cuda.synchronize()
    b.check()


@pytest.mark.parametrize("depth", [4, 8, 16, 32])
def test_long_stream_pieces_drain_the_vertical_counter(depth):
    """A wave's piece of a long stream is walked in chunks of 254 tiles, the carry
    counter drained after each: three streams of 64-384 MiB over one-wave blocks,
    one per CU, give each wave 2.5 MiB, more than 254 tiles at every depth (a tile
    is 64 lanes x depth dwords, 8 KiB at depth 32), next to short streams."""
    lengths = np.array([(384 << 20) + 5, 3, (192 << 20) // 2 + 1, 17, (64 << 20) // 4 - 3],
                       dtype=np.uint64)
    ks = np.array([8, 16, 16, 32, 32], dtype=np.int32)
    s = I.StreamSet(lengths, ks, np.array([0.5, 0.5, 0.1, 0.9, 0.7]))
    b = Batch(s, SEED + 60 + depth, threads=I.default_threads())
    plan = B.Plan(b.m)
    plan.config = dict(depth=depth, block_threads=64, blocks_per_cu=1, stream_weight=1)
    say(f"batch long pieces depth {depth}")
    plan.run(b.descs)
    torch.cuda.synchronize()
    b.check()


def test_graph_replay_reads_current_descriptors(small_batch):
    b = small_batch
    plan = B.Plan(b.m, graph=True)
    b.counts.zero_()
    for _ in range(3):
        plan.run(b.descs)
    torch.cuda.synchronize()
    b.check(factor=3)
    # same descriptor buffer, new contents: stream i now counts into row i - 1
    shifted = b.desc_host.copy()
    shifted[:, 3] = np.roll(b.desc_host[:, 3], 1)
    b.descs.copy_(B.to_device(shifted))
    b.counts.zero_()
    plan.run(b.descs)
    torch.cuda.synchronize()
    got = b.counts.cpu().numpy()
    for i in range(b.m):
        k = int(b.streams.ks[i])
        assert (got[(i - 1) % b.m, :k] == b.expected(i)).all(), f"stream {i}"
    b.descs.copy_(B.to_device(b.desc_host))
    torch.cuda.synchronize()


def test_each_matches_batch(small_batch):
    b = small_batch
    b.counts.zero_()
    B.pospopcnt_each(b.desc_host)
    torch.cuda.synchronize()
    b.check()


def test_shared_counts_and_rejected_descriptors():
    s = mixed(64, 14, SEED + 1, min_len=1)
    bt = Batch(s, SEED + 1)
    d = bt.desc_host.copy()
    ks = s.ks.copy()
    total = torch.zeros(32, dtype=torch.int64, device="cuda")
    shared = np.nonzero(ks == 16)[0]
    d[shared, 3] = total.data_ptr()  # every k = 16 stream adds into one vector
    others = [int(i) for i in np.nonzero(ks != 16)[0]]
    bad = others[:5]
    d[bad[0], 2] = 12                                   # width not 8/16/32
    d[bad[1], 2] = int(d[bad[1], 2]) | (1 << 32)        # reserved != 0
    d[bad[2], 3] = int(d[bad[2], 3]) + 4                # misaligned counts
    d[bad[3], 0] = 0                                    # NULL input
    d[bad[4], 3] = d[bad[4], 0]                         # counts inside the input
    plan = B.Plan(64)
    plan.run(B.to_device(d))
    torch.cuda.synchronize()
    assert plan.rejected() == 5
    got = bt.counts.cpu().numpy()
    for i in others:
        k = int(ks[i])
        if i in bad:
            assert (got[i] == 0).all(), f"rejected stream {i} was counted"
        else:
            assert (got[i, :k] == bt.expected(i)).all(), f"stream {i}"
    exp_total = sum(bt.expected(int(i)) for i in shared)
    assert (total.cpu().numpy()[:16] == exp_total).all()
    assert (total.cpu().numpy()[16:] == 0).all()


def test_one_huge_stream_over_all_blocks():
    n = (1 << 27) + 3
    s = I.StreamSet(np.array([n], np.uint64), np.array([16], np.int32), np.array([0.5]))
    bt = Batch(s, SEED + 2)
    for cfg in (dict(blocks_per_cu=1), dict(blocks_per_cu=16, block_threads=64)):
        bt.counts.zero_()
        plan = B.Plan(1)
        plan.config = cfg
        plan.run(bt.descs)
        torch.cuda.synchronize()
        bt.check()


@pytest.mark.timeout(600)
def test_stream_over_4_gib_in_a_batch():
    """A stream of 2^32 + 7 uint8 words (its word count and its bytes both past 32
    bits) at an odd address, between small streams of the other widths: at the
    default shape and at one block per compute unit, where a block's share of the
    long stream is largest; every stream against the oracle in full."""
    lengths = np.array([1000, (1 << 32) + 7, 77, 5], np.uint64)
    ks = np.array([16, 8, 32, 8], np.int32)
    s = I.StreamSet(lengths, ks, np.array([0.5, 0.5, 0.02, 0.9]))
    bt = Batch(s, SEED + 70, threads=I.default_threads())
    assert int(bt.starts[1]) % 16 == 7  # the seed places the long stream at an odd address
    for cfg in (None, dict(blocks_per_cu=1, block_threads=64)):
        bt.counts.zero_()
        plan = B.Plan(len(lengths))
        if cfg:
            plan.config = cfg
        say(f"stream over 4 GiB in a batch, cfg={cfg}")
        plan.run(bt.descs)
        torch.cuda.synchronize()
        plan.close()
        bt.check()


def test_autotune_leaves_counts_and_picks_valid_config(small_batch, tmp_path):
    b = small_batch
    b.counts.zero_()
    plan = B.Plan(b.m)
    ms = plan.autotune(b.descs)
    assert ms > 0
    assert (b.counts.cpu().numpy() == 0).all(), "autotune must not touch the counters"
    cfg = plan.config
    plan.run(b.descs)
    torch.cuda.synchronize()
    b.check()
    path = str(tmp_path / "plan.json")
    plan.save(path)
    other = B.Plan(b.m)
    other.load(path)
    assert other.config == cfg


@pytest.mark.timeout(900)
def test_c4_full_mix():
    """20,000 streams, lengths log-uniform in [1, 2^22] words, k uniform in {8,16,32},
    Bernoulli(p) bits with p ~ U(0,1): batched (graph + autotuned) equals the oracle
    and the one-launch-per-stream form."""
    s = I.loguniform_streams(20_000, 22, SEED)
    say(f"C4: generating {s.nbytes.sum() / 1e9:.2f} GB")
    bt = Batch(s, SEED, threads=I.default_threads())
    plan = B.Plan(bt.m, graph=True)
    plan.autotune(bt.descs)
    say(f"C4: batched run, config {plan.config}")
    plan.run(bt.descs)
    torch.cuda.synchronize()
    got = bt.counts.cpu().numpy().copy()
    bt.counts.zero_()
    B.pospopcnt_each(bt.desc_host)
    torch.cuda.synchronize()
    each = bt.counts.cpu().numpy()
    assert (got == each).all()
    say("C4: oracle")
    bt.counts.copy_(torch.from_numpy(got))
    bt.check()


@pytest.mark.parametrize("weight", [1, 3, 4096])
def test_tiny_totals_smaller_than_the_grid(weight):
    """A few edge-only streams: the weighted axis is shorter than the grid, so most
    blocks have empty shares."""
    s = I.StreamSet(np.array([1, 3, 0, 7, 2], np.uint64), np.array([8, 16, 32, 8, 32], np.int32),
                    np.array([0.5] * 5))
    bt = Batch(s, SEED + 5)
    for cfg in (dict(blocks_per_cu=16, block_threads=64), dict(blocks_per_cu=1, block_threads=256)):
        bt.counts.zero_()
        plan = B.Plan(5)
        plan.config = dict(cfg, stream_weight=weight)
        plan.run(bt.descs)
        torch.cuda.synchronize()
        bt.check()


@pytest.mark.parametrize("m", [4096, 4097, 6143, 6144, 6145, 10_241])
def test_many_streams_split_preparation(m):
    """Batches above 4096 streams are prepared by one block per 2048 positions: sizes
    at and around those boundaries, with empty and rejected descriptors among them
    (the rejected count sums over the chunks), with and without graph replay."""
    s = mixed(m, 9, SEED + 40 + m)
    s.lengths[::97] = 0
    bt = Batch(s, SEED + 40 + m)
    d = bt.desc_host.copy()
    bad = list(range(3, m, 1001))
    d[bad, 2] = 24  # width not 8/16/32
    for graph in (False, True):
        say(f"split preparation m={m} graph={graph}")
        bt.counts.zero_()
        plan = B.Plan(m, graph=graph)
        plan.run(B.to_device(d))
        torch.cuda.synchronize()
        assert plan.rejected() == len(bad)
        got = bt.counts.cpu().numpy()
        for i in range(m):
            k = int(s.ks[i])
            exp = 0 if i in bad else bt.expected(i)
            assert (got[i, :k] == exp).all(), f"stream {i}"


def test_many_streams_short_axis_and_one_long_stream():
    """5000 descriptors: mostly empty with a few one-word streams (an axis shorter
    than the grid), then one long stream among the empty ones."""
    m = 5000
    lengths = np.zeros(m, np.uint64)
    lengths[[17, 2500, 4999]] = 1
    s = I.StreamSet(lengths, np.full(m, 16, np.int32), np.full(m, 0.5))
    bt = Batch(s, SEED + 50)
    for cfg in (dict(blocks_per_cu=16, block_threads=64), dict(stream_weight=1)):
        bt.counts.zero_()
        plan = B.Plan(m)
        plan.config = cfg
        say(f"short axis m={m} cfg={cfg}")
        plan.run(bt.descs)
        torch.cuda.synchronize()
        bt.check(which=[17, 2500, 4999, 0, 1, 4998])
    lengths[2500] = (1 << 24) + 5
    s = I.StreamSet(lengths, np.full(m, 16, np.int32), np.full(m, 0.5))
    bt = Batch(s, SEED + 51)
    plan = B.Plan(m)
    say(f"one long stream among {m}")
    plan.run(bt.descs)
    torch.cuda.synchronize()
    bt.check(which=[17, 2500, 4999, 0, 4998])


def test_plan_cache_round_trip(tmp_path, small_batch):
    """Tuned configurations stored per workload key (streams and bytes, log2 buckets) and
    taken back by a new plan; a key with no entry leaves the plan as it was."""
    b = small_batch
    path = str(tmp_path / "plans.jsonl")
    total = int(b.streams.nbytes.sum())
    plan = B.Plan(b.m)
    assert not plan.cache_get(path, b.m, total)  # no file yet: an empty cache
    plan.config = dict(depth=8, block_threads=128, blocks_per_cu=5, stream_weight=777)
    plan.cache_put(path, b.m, total)
    plan.config = dict(depth=32, block_threads=64, blocks_per_cu=2, stream_weight=9)
    plan.cache_put(path, 20_000, 13 << 30)  # another key in the same file
    plan.config = dict(depth=4, block_threads=256, blocks_per_cu=3, stream_weight=5)
    plan.cache_put(path, b.m + 1, total + 1)  # same buckets: replaces the first entry
    assert len(open(path).read().splitlines()) == 2
    fresh = B.Plan(b.m)
    before = fresh.config
    assert not fresh.cache_get(path, b.m, total * 4)  # another bytes bucket
    assert fresh.config == before
    assert fresh.cache_get(path, b.m, total)
    assert fresh.config == dict(depth=4, block_threads=256, blocks_per_cu=3, stream_weight=5)
    assert fresh.cache_get(path, 20_000, 13 << 30)
    assert fresh.config["stream_weight"] == 9
    b.counts.zero_()
    say("batch with a cached configuration")
    fresh.run(b.descs)
    torch.cuda.synchronize()
    b.check()
    with open(path, "a") as f:
        f.write("not json\n")
    with pytest.raises(Exception):
        fresh.cache_get(path, b.m, total)
