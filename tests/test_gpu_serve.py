"""GPU serving: requests replayed through the continuous-batching server give, for
every request, the oracle's counts and the counts of the same input counted
alone (tolerance 0), under memory-budget pressure and with launches
overlapping on several streams."""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import api
from paper_1911_02696_amd import inputs as I
from paper_1911_02696_amd import serve as S

from gpu_util import oracle_counts, say

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 4
POOL = 64 << 20


@pytest.fixture(scope="module")
def workload():
    trace = I.serving_trace(200_000, 0.015, SEED, min_log2=4, max_log2=22, pool_bytes=POOL)
    pools = S.Pools(trace, POOL, SEED)
    return trace, pools, pools.requests(trace)


def expected(trace, pools, i):
    n, k = int(trace.lengths[i]), int(trace.ks[i])
    return oracle_counts(pools.host_bytes(trace, i), n, k)


def alone(req):
    out = torch.zeros(32, dtype=torch.int64, device="cuda")
    api.pospopcnt_ptr(int(req["src"]), int(req["n"]), int(req["k"]), out.data_ptr())
    return out.cpu().numpy()


@pytest.mark.parametrize("in_place", [False, True], ids=["copy", "in_place"])
def test_served_counts_equal_oracle_and_alone(workload, in_place):
    trace, pools, reqs = workload
    m = len(reqs)
    say(f"serve: {m} requests, {trace.nbytes.sum() / 1e9:.2f} GB, in_place={in_place}")
    arena = 96 << 20  # far below the total: requests wait for memory
    srv = S.Server(arena, max_requests=512, max_batch=128, streams=4, in_place=in_place)
    comps = srv.run_trace(reqs)
    st = srv.stats()
    srv.close()
    assert (comps["status"] == 0).all(), np.unique(comps["status"])
    assert (comps["tag"] == np.arange(m)).all()
    assert st["arena_peak"] <= arena and st["max_queued"] > 0 and st["launches"] > 1
    assert st["bytes_counted"] == int(trace.nbytes.sum())
    rng = np.random.Generator(np.random.PCG64(SEED))
    sample = set(rng.choice(m, size=min(m, 400), replace=False).tolist())
    sample |= set(np.argsort(trace.nbytes)[-20:].tolist())
    for i in range(m):
        k = int(trace.ks[i])
        exp = expected(trace, pools, i)
        assert (comps["counts"][i][:k].astype(np.int64) == exp).all(), f"request {i}"
        if i in sample:
            assert (alone(reqs[i])[:k] == exp).all(), f"request {i} alone"
    lat = S.latency_summary(comps)
    assert lat["ok"] == m
    say(f"serve latency {lat}")


def test_request_larger_than_budget_is_rejected(workload):
    trace, pools, reqs = workload
    big = int(np.argmax(trace.nbytes))
    srv = S.Server(int(trace.nbytes[big]) - 1024, max_requests=8, max_batch=8, streams=1)
    comps = srv.run_trace(reqs[[big]])
    srv.close()
    assert comps["status"][0] == 6


def test_many_small_requests_one_stream(workload):
    trace, pools, reqs = workload
    small = np.nonzero(trace.nbytes < 4096)[0][:500]
    r = reqs[small].copy()
    r["arrival"] = 0.0
    srv = S.Server(1 << 24, max_requests=64, max_batch=16, streams=1)
    comps = srv.run_trace(r)
    srv.close()
    for j, i in enumerate(small):
        k = int(trace.ks[i])
        assert (comps["counts"][j][:k].astype(np.int64) == expected(trace, pools, i)).all()
    assert comps["batch"].max() <= 16


def test_unaligned_sources_are_copied_exactly(workload):
    """Request inputs starting at every misalignment 0..15: each copy starts at its source's
    address modulo 16 inside its slab, counted while it is copied."""
    trace, pools, reqs = workload
    pick = np.nonzero(trace.nbytes < (1 << 20))[0][:64]
    r = reqs[pick].copy()
    shift = (np.arange(len(pick)) % 16).astype(np.uint64)
    # keep each window inside its pool: move it left when the shift would run past the end
    room = POOL - (trace.offset[pick] + trace.nbytes[pick])
    shift = np.where(room >= shift, shift, 0)
    r["src"] = r["src"] + shift
    r["arrival"] = 0.0
    srv = S.Server(1 << 28, max_requests=64, max_batch=32, streams=2)
    comps = srv.run_trace(r)
    srv.close()
    for j, i in enumerate(pick):
        k, n = int(trace.ks[i]), int(trace.lengths[i])
        p, o = int(trace.pool[i]), int(trace.offset[i]) + int(shift[j])
        exp = oracle_counts(pools.host[p][o:o + n * k // 8], n, k)
        assert comps["status"][j] == 0
        assert (comps["counts"][j][:k].astype(np.int64) == exp).all(), f"request {i} shift {shift[j]}"


@pytest.mark.parametrize("in_place", [False, True], ids=["copy", "in_place"])
def test_large_and_small_batches_share_slots(workload, in_place):
    """Launches of more than 1024 requests (prepared in a kernel of their own) and of
    fewer (one kernel that prepares its own shares) on the same two slots: every
    launch must start from cleared counters, which the previous launch of the slot
    cleared after its results were read back."""
    trace, pools, reqs = workload
    pick = np.nonzero(trace.nbytes < (1 << 18))[0][:2500]
    r = reqs[pick].copy()
    r["arrival"] = 0.0
    say(f"serve: {len(pick)} requests at once, max_batch 1030, in_place={in_place}")
    srv = S.Server(1 << 30, max_requests=4096, max_batch=1030, streams=1, in_place=in_place)
    comps = srv.run_trace(r)
    srv.close()
    assert (comps["status"] == 0).all()
    # 2120 requests in launches of at most 1030: two large ones fill both slots, the
    # rest (fewer than 1024) reuses a slot after its counters were cleared
    batches = np.unique(comps["batch"])
    assert batches.max() > 1024 and batches.min() <= 1024 and len(pick) > 2 * 1030, batches
    for j, i in enumerate(pick):
        k = int(trace.ks[i])
        assert (comps["counts"][j][:k].astype(np.int64) == expected(trace, pools, i)).all(), j


@pytest.mark.parametrize("in_place", [False, True], ids=["copy", "in_place"])
def test_benchmark_configuration_sampled(in_place):
    """One second of the benchmark's C5 trace in its configuration (512 MiB pools, a
    64 GiB arena, 4096 requests in flight, batches of up to 1024, 4 streams): every
    request succeeds, and 150 of them (the 30 largest among them) equal the oracle."""
    seed = I.BASE_SEED + 4
    pool = 1 << 29
    trace = I.serving_trace(50_000, 1.0, seed, pool_bytes=pool)
    pools = S.Pools(trace, pool, seed)
    reqs = pools.requests(trace)
    say(f"serve C5 config: {len(reqs)} requests, {trace.nbytes.sum() / 1e9:.1f} GB, "
        f"in_place={in_place}")
    srv = S.Server(64 << 30, max_requests=4096, max_batch=1024, streams=4, in_place=in_place)
    comps = srv.run_trace(reqs)
    srv.close()
    assert (comps["status"] == 0).all()
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    sample = np.unique(np.concatenate([rng.choice(len(reqs), 120, replace=False),
                                       np.argsort(trace.nbytes)[-30:]]))
    for i in sample:
        k = int(trace.ks[i])
        assert (comps["counts"][i][:k].astype(np.int64) == expected(trace, pools, i)).all(), i
    del pools
    torch.cuda.empty_cache()
