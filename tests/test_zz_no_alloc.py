"""The allocation-free batched count (pospopcnt_batch_static, scratch in the
library's file-scope device array) against the plan-based pospopcnt_batch on the
same streams: bit for bit, on calls in a row whose inputs shrink, so that every
call reuses what the previous one left in the array.  Both go through the C ABI."""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import _lib as L
from paper_1911_02696_amd import api
from paper_1911_02696_amd import batch as B
from paper_1911_02696_amd import inputs as I

from gpu_util import oracle_counts, say

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 60


def _workload(m, max_log2, seed):
    """m streams of mixed k and length at seeded start offsets in one device arena,
    some empty and a few invalid (width 24), with two zeroed count tables."""
    s = I.loguniform_streams(m, max_log2, seed)
    s.lengths[::53] = 0
    nb = s.nbytes.astype(np.int64)
    starts, size = I.batch_layout(nb, seed)
    host = np.zeros(size + 64, np.uint8)
    I.fill_streams(host, s, starts, seed)
    dev = torch.from_numpy(host).cuda()
    tables = []
    for _ in range(2):
        counts = torch.zeros((m, 32), dtype=torch.int64, device="cuda")
        d = B.descriptors(dev.data_ptr() + starts, s.lengths, s.ks,
                          counts.data_ptr() + 256 * np.arange(m))
        d[5::701, 2] = 24
        tables.append((counts, B.to_device(d)))
    return s, starts, host, dev, tables


CALLS = [  # (streams, largest length 2^x, configuration): each call smaller than the last
    (5000, 16, None),                       # split preparation (more than 4096 streams)
    (300, 12, None),                        # single-block preparation
    (40, 10, dict(depth=32, block_threads=256, blocks_per_cu=2, stream_weight=1024)),
]


def test_static_equals_plan_on_calls_in_a_row():
    for j, (m, max_log2, cfg) in enumerate(CALLS):
        s, starts, host, dev, ((c_static, d_static), (c_plan, d_plan)) = \
            _workload(m, max_log2, SEED + j)
        say(f"no-alloc batch: call {j}, m={m}, config={cfg}")
        B.batch_static(d_static, config=cfg)
        plan = B.Plan(m)
        if cfg:
            plan.config = cfg
        plan.run(d_plan)
        torch.cuda.synchronize()
        plan.close()
        got, ref = c_static.cpu().numpy(), c_plan.cpu().numpy()
        assert (got == ref).all(), f"call {j}: the static form differs from the plan's"
        # and a sample against the oracle, the invalid descriptors left at zero
        bad = set(range(5, m, 701))
        for i in sorted(set(range(0, m, max(1, m // 60))) | bad):
            k, n, st = int(s.ks[i]), int(s.lengths[i]), int(starts[i])
            exp = 0 if i in bad else oracle_counts(host[st:st + n * k // 8], n, k)
            assert (got[i, :k] == exp).all(), f"call {j} stream {i}"
            assert (got[i, k:] == 0).all()


def test_static_at_its_capacity():
    """PPC_STATIC_MAX_STREAMS streams (the largest table the array holds) on the
    largest grid it allows, 16 one-wave blocks per compute unit (4096 blocks on 256
    units), against the plan-based call and a sample of the oracle."""
    m = L.STATIC_MAX_STREAMS
    bpc = max(1, min(16, 4096 // api.device_info()["compute_units"]))
    cfg = dict(depth=16, block_threads=64, blocks_per_cu=bpc, stream_weight=256)
    s, starts, host, dev, ((c_static, d_static), (c_plan, d_plan)) = \
        _workload(m, 9, SEED + 7)
    say(f"no-alloc batch at capacity: m={m}, config={cfg}")
    B.batch_static(d_static, config=cfg)
    plan = B.Plan(m)
    plan.config = cfg
    plan.run(d_plan)
    torch.cuda.synchronize()
    plan.close()
    got, ref = c_static.cpu().numpy(), c_plan.cpu().numpy()
    assert (got == ref).all(), "the static form differs from the plan's at capacity"
    bad = set(range(5, m, 701))
    for i in sorted(set(range(0, m, 97)) | {m - 1} | bad):
        k, n, st = int(s.ks[i]), int(s.lengths[i]), int(starts[i])
        exp = 0 if i in bad else oracle_counts(host[st:st + n * k // 8], n, k)
        assert (got[i, :k] == exp).all(), f"stream {i}"
        assert (got[i, k:] == 0).all()


def test_static_capacity_is_reported_before_launch():
    m = L.STATIC_MAX_STREAMS + 1
    descs = torch.zeros((m, 4), dtype=torch.int64, device="cuda")
    lib = L.lib()
    assert lib.pospopcnt_batch_static(descs.data_ptr(), m, None, None) == 10
    assert lib.pospopcnt_batch_static(descs.data_ptr(), m - 1, None, None) == 0
    torch.cuda.synchronize()
