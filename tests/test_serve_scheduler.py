"""The serving scheduler on the CPU: the same C++ request loop the GPU server runs,
driven through executor callbacks with the oracle behind them.  Checks
admission under a memory budget and a slot limit, FIFO order (and its bypass),
continuous batching, failure handling, and that every completion carries its own
request's counts (verified against a numpy brute force)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1911_02696_amd import inputs as I
from paper_1911_02696_amd import serve as S
from paper_1911_02696_amd._lib import PpcError

GRANULE = 256


def brute(raw: np.ndarray, n: int, k: int) -> np.ndarray:
    bits = np.unpackbits(raw[:n * k // 8], bitorder="little").reshape(n, k)
    return bits.sum(axis=0, dtype=np.uint64)


def granules(b):
    return ((max(b, 1) + GRANULE - 1) // GRANULE) * GRANULE


class FakeExecutor:
    """Counts each launch with the oracle on host memory; a launch is reported done
    after `delay` polls.  Records launches and checks the arena slabs of live
    requests never overlap and stay inside the arena."""

    def __init__(self, arena_bytes, delay=2, fail_launches=()):
        self.arena = arena_bytes
        self.delay = delay
        self.fail = set(fail_launches)
        self.live = {}
        self.log = []
        self.errors = []
        self.max_live_requests = 0
        self.next = 1
        self.ops = S.ExecutorOps(S.LAUNCH_FN(self._launch), S.POLL_FN(self._poll),
                                 S.RESULTS_FN(self._results), S.RELEASE_FN(self._release))

    def _launch(self, user, items_ptr, n, handle_ptr):
        try:
            raw = (ctypes.c_char * (n * S.EXEC_ITEM_DTYPE.itemsize)).from_address(items_ptr)
            items = np.frombuffer(raw, dtype=S.EXEC_ITEM_DTYPE).copy()
            idx = len(self.log)
            self.log.append(items["tag"].tolist())
            if idx in self.fail:
                return 5
            spans = [(int(it["arena_offset"]), granules(int(it["n"]) * int(it["k"]) // 8))
                     for it in items]
            for v in self.live.values():
                for it in v[0]:
                    spans.append((int(it["arena_offset"]),
                                  granules(int(it["n"]) * int(it["k"]) // 8)))
            spans.sort()
            for (a, la), (b, _) in zip(spans, spans[1:]):
                if a + la > b:
                    self.errors.append(f"slabs overlap: {a}+{la} > {b}")
            if spans and spans[-1][0] + spans[-1][1] > self.arena:
                self.errors.append("slab outside the arena")
            counts = np.zeros((n, 32), np.uint64)
            for i, it in enumerate(items):
                k, w = int(it["k"]), int(it["n"])
                view = np.ctypeslib.as_array(
                    (ctypes.c_uint8 * (w * k // 8)).from_address(int(it["src"])))
                counts[i, :k] = oracle.count(view, w, k)
            h = self.next
            self.next += 1
            self.live[h] = [items, counts, 0]
            self.max_live_requests = max(self.max_live_requests,
                                         sum(len(v[0]) for v in self.live.values()))
            handle_ptr[0] = h
            return 0
        except Exception as e:  # never let an exception cross the C boundary
            self.errors.append(repr(e))
            return 7

    def _poll(self, user, h, done_ptr):
        v = self.live[h]
        v[2] += 1
        done_ptr[0] = 1 if v[2] >= self.delay else 0
        return 0

    def _results(self, user, h, counts_ptr):
        c = self.live[h][1]
        ctypes.memmove(counts_ptr, c.ctypes.data, c.nbytes)
        return 0

    def _release(self, user, h):
        self.live.pop(h, None)
        return 0


class Workload:
    def __init__(self, m, seed, max_bytes=4096):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.k = rng.choice([8, 16, 32], size=m)
        wb = self.k // 8
        self.n = np.maximum(1, rng.integers(1, max_bytes, size=m) // wb)
        self.bytes = self.n * wb
        self.starts = np.concatenate([[0], np.cumsum(self.bytes)[:-1]])
        self.host = I.generate(int(self.bytes.sum()) + 64, I.Dist.bernoulli(0.4), seed)
        base = self.host.ctypes.data
        self.reqs = S.requests(base + self.starts, self.n, self.k)

    def expected(self, tag):
        s, n, k = int(self.starts[tag]), int(self.n[tag]), int(self.k[tag])
        return brute(self.host[s:], n, k)


def drive(server, reqs=None, max_steps=100000):
    if reqs is not None:
        server.submit(reqs)
    done = []
    for _ in range(max_steps):
        server.progress()
        done.extend(server.take_completions())
        st = server.stats()
        if st["completed"] == st["submitted"]:
            break
    return np.array(done, dtype=S.COMPLETION_DTYPE)


def check_counts(w, comps):
    assert len(comps) == len(w.reqs)
    assert sorted(comps["tag"].tolist()) == list(range(len(w.reqs)))
    for c in comps:
        t = int(c["tag"])
        assert c["status"] == 0, (t, c["status"])
        k = int(w.k[t])
        assert (c["counts"][:k] == w.expected(t)).all(), f"request {t}"
        assert (c["counts"][k:] == 0).all()


def test_all_requests_complete_with_their_own_counts():
    w = Workload(300, 1)
    ex = FakeExecutor(1 << 20)
    srv = S.Server(1 << 20, max_requests=64, max_batch=16, streams=2, executor=ex.ops)
    comps = drive(srv, w.reqs)
    assert not ex.errors, ex.errors
    check_counts(w, comps)
    st = srv.stats()
    assert st["launches"] >= 300 // 16
    assert st["bytes_counted"] == int(w.bytes.sum())
    assert (comps["completed"] >= comps["launched"]).all()
    assert (comps["launched"] >= comps["admitted"]).all()


def test_memory_budget_and_rejection():
    w = Workload(120, 2, max_bytes=30_000)
    arena = 64 << 10
    big = S.requests([w.host.ctypes.data], [100_000], [8], tags=[999])
    ex = FakeExecutor(arena, delay=3)
    srv = S.Server(arena, max_requests=1000, max_batch=8, streams=2, executor=ex.ops)
    srv.submit(big)
    first = srv.take_completions()
    assert len(first) == 1 and first[0]["status"] == 6 and first[0]["tag"] == 999  # BUDGET
    comps = drive(srv, w.reqs)
    assert not ex.errors, ex.errors
    check_counts(w, comps)
    st = srv.stats()
    assert st["rejected"] == 1
    assert 0 < st["arena_peak"] <= arena
    assert st["arena_used_now"] == 0
    assert st["max_queued"] > 0  # the budget made requests wait


def test_slot_limit():
    w = Workload(100, 3)
    ex = FakeExecutor(1 << 30, delay=4)
    srv = S.Server(1 << 30, max_requests=3, max_batch=64, streams=4, executor=ex.ops)
    comps = drive(srv, w.reqs)
    check_counts(w, comps)
    assert ex.max_live_requests <= 3
    assert srv.stats()["max_inflight"] <= 3


def test_fifo_admission_order():
    w = Workload(200, 4, max_bytes=20_000)
    ex = FakeExecutor(48 << 10, delay=2)
    srv = S.Server(48 << 10, max_requests=100, max_batch=5, streams=2, executor=ex.ops)
    comps = drive(srv, w.reqs)
    check_counts(w, comps)
    order = [t for launch in ex.log for t in launch]
    assert order == list(range(200)), "strict FIFO admits and launches in arrival order"


def test_fifo_bypass_lets_small_requests_pass():
    arena = 16 << 10
    host = I.generate(64 << 10, I.Dist.uniform(), 5)
    base = host.ctypes.data
    # a 12 KiB request holds memory; a 10 KiB one then cannot fit; 1 KiB ones can
    reqs = S.requests([base, base + 20000] + [base + 40000 + 2000 * i for i in range(4)],
                      [12 << 10, 10 << 10] + [1024] * 4, [8] * 6)
    for bypass, passes in ((False, False), (True, True)):
        ex = FakeExecutor(arena, delay=5)
        srv = S.Server(arena, max_requests=100, max_batch=100, streams=1,
                       fifo_bypass=bypass, executor=ex.ops)
        srv.submit(reqs[:1])
        srv.progress()   # request 0 launched
        srv.submit(reqs[1:])
        srv.progress()
        second = ex.log[1] if len(ex.log) > 1 else []
        assert (second == [2, 3, 4, 5]) == passes, (bypass, ex.log)
        comps = drive(srv)
        assert (comps["status"] == 0).all()


def test_continuous_batching_overlaps_launches():
    w = Workload(400, 6)
    ex = FakeExecutor(1 << 30, delay=6)
    srv = S.Server(1 << 30, max_requests=1000, max_batch=1000, streams=2, executor=ex.ops)
    comps = []
    for i in range(0, 400, 10):  # requests keep arriving while launches are in flight
        srv.submit(w.reqs[i:i + 10])
        srv.progress()
        comps.extend(srv.take_completions())
    comps = np.concatenate([np.array(comps, S.COMPLETION_DTYPE), drive(srv)])
    check_counts(w, comps)
    sizes = [len(x) for x in ex.log]
    assert len(sizes) > 4 and max(sizes) > 10, sizes  # later launches gather newer arrivals
    assert max(c for c in [len(ex.live)]) <= 4


def test_failed_launch_fails_only_its_requests():
    w = Workload(60, 7)
    ex = FakeExecutor(1 << 30, delay=1, fail_launches={1})
    srv = S.Server(1 << 30, max_requests=10, max_batch=10, streams=1, executor=ex.ops)
    comps = drive(srv, w.reqs)
    failed = set(ex.log[1])
    for c in comps:
        t = int(c["tag"])
        if t in failed:
            assert c["status"] == 5
        else:
            assert c["status"] == 0 and (c["counts"][:w.k[t]] == w.expected(t)).all()
    assert srv.stats()["arena_used_now"] == 0


def test_invalid_requests_complete_at_once():
    host = np.zeros(64, np.uint8)
    r = S.requests([host.ctypes.data, host.ctypes.data, 0, host.ctypes.data],
                   [4, 4, 4, 0], [12, 16, 16, 16])
    r["reserved"][1] = 1
    ex = FakeExecutor(1 << 20)
    srv = S.Server(1 << 20, executor=ex.ops)
    srv.submit(r)
    c = srv.take_completions()
    assert c["status"].tolist() == [3, 7, 1, 0]
    assert (c["counts"][3] == 0).all()
    assert ex.log == []


def test_run_trace_respects_arrivals():
    w = Workload(150, 8)
    w.reqs["arrival"] = np.sort(np.random.Generator(np.random.PCG64(8)).random(150) * 0.05)
    ex = FakeExecutor(1 << 30, delay=2)
    srv = S.Server(1 << 30, max_requests=64, max_batch=32, streams=2, executor=ex.ops)
    t0 = srv.now()
    comps = srv.run_trace(w.reqs)
    assert (comps["tag"] == np.arange(150)).all()
    check_counts(w, comps)
    assert (comps["admitted"] >= comps["arrival"] - 1e-9).all()
    assert (comps["arrival"] - t0 >= w.reqs["arrival"] - 1e-3).all()
    lat = S.latency_summary(comps)
    assert lat["ok"] == 150 and lat["p99_ms"] >= lat["p50_ms"] > 0


def test_run_trace_needs_an_idle_server():
    """A replay indexes its output by request position, so it refuses a server that
    still holds requests submitted directly (their tags are the caller's own)."""
    w = Workload(20, 9)
    ex = FakeExecutor(1 << 20, delay=3)
    srv = S.Server(1 << 20, max_requests=8, max_batch=4, streams=1, executor=ex.ops)
    early = w.reqs[:4].copy()
    early["tag"] = [10 ** 9, 10 ** 9 + 1, 10 ** 9 + 2, 10 ** 9 + 3]
    srv.submit(early)
    srv.progress()
    for held in ("queued or in flight", "completions not taken"):
        with pytest.raises(PpcError) as err:
            srv.run_trace(w.reqs[4:])
        assert err.value.status == 9  # PPC_ERR_STATE
        assert srv.stats()["submitted"] == 4, held
        for _ in range(100):
            srv.progress()
            if srv.stats()["completed"] == 4:
                break
        assert srv.stats()["completed"] == 4
    comps = srv.take_completions()
    assert sorted(comps["tag"].tolist()) == early["tag"].tolist()
    comps = srv.run_trace(w.reqs[4:])
    assert (comps["tag"] == np.arange(4, 20)).all()
    check_counts_subset(w, comps)


def check_counts_subset(w, comps):
    for c in comps:
        t = int(c["tag"])
        assert c["status"] == 0, (t, c["status"])
        k = int(w.k[t])
        assert (c["counts"][:k] == w.expected(t)).all(), f"request {t}"


def test_server_argument_checks():
    from paper_1911_02696_amd import _lib as L
    lib = L.lib()
    h = ctypes.c_void_p()
    for cfg in (S.ServerConfig(1 << 20, 0, 1, 1, 0), S.ServerConfig(1 << 20, 1, 0, 1, 0),
                S.ServerConfig(1 << 20, 1, 1, 9, 0), S.ServerConfig(1 << 20, 1, 1, 1, 64)):
        assert lib.ppc_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 7
    assert lib.ppc_server_create(None, ctypes.byref(h)) == 1
    assert lib.ppc_server_destroy(None) == 0
    assert lib.ppc_server_submit(None, None, 0) == 1
    assert lib.ppc_server_progress(None, None, None) == 1
    ops = S.ExecutorOps()
    assert lib.ppc_server_create_with_executor(ctypes.byref(S.ServerConfig(1, 1, 1, 1, 0)),
                                               ctypes.byref(ops), None, ctypes.byref(h)) == 1


def test_timeout_expires_only_waiting_requests():
    """A request still waiting for memory when its timeout passes completes with
    PPC_ERR_TIMEOUT and is never launched; one without a timeout waits on."""
    import time
    arena = 16 << 10
    host = I.generate(64 << 10, I.Dist.uniform(), 11)
    base = host.ctypes.data
    reqs = S.requests([base, base + 20000, base + 40000], [12 << 10, 10 << 10, 10 << 10],
                      [8, 8, 8], tags=[0, 1, 2], timeouts=[0.0, 0.05, 0.0])
    ex = FakeExecutor(arena, delay=10 ** 9)  # request 0 holds the arena until released
    srv = S.Server(arena, max_requests=10, max_batch=10, streams=1, executor=ex.ops)
    reqs["arrival"] = srv.now()
    srv.submit(reqs)
    srv.progress()
    time.sleep(0.08)
    srv.progress()
    first = srv.take_completions()
    assert first["tag"].tolist() == [1] and first["status"].tolist() == [11]  # TIMEOUT
    ex.delay = 1
    comps = drive(srv)
    assert sorted(comps["tag"].tolist()) == [0, 2] and (comps["status"] == 0).all()
    assert [t for launch in ex.log for t in launch] == [0, 2]
    st = srv.stats()
    assert st["expired"] == 1 and st["completed"] == 3 and st["arena_used_now"] == 0


def test_cancel_waiting_and_admitted_requests():
    """Cancelling drops a waiting request and an admitted one that is not launched yet
    (its slab is given back); a launched request runs to completion."""
    w = Workload(6, 12, max_bytes=2000)
    ex = FakeExecutor(1 << 20, delay=10 ** 9)
    # one launch slot pair (streams=1) and one request per launch: after two steps,
    # requests 0 and 1 are launched and 2..5 admitted but not launched
    srv = S.Server(1 << 20, max_requests=5, max_batch=1, streams=1, executor=ex.ops)
    srv.submit(w.reqs)
    srv.progress()
    srv.progress()
    assert [t for launch in ex.log for t in launch] == [0, 1]
    used = srv.stats()["arena_used_now"]
    assert srv.cancel(3) == 1       # admitted, not launched
    assert srv.stats()["arena_used_now"] < used
    assert srv.cancel(5) == 1       # waiting (slot limit)
    assert srv.cancel(0) == 0       # launched: not cancelled
    assert srv.cancel(77) == 0      # unknown tag
    c = srv.take_completions()
    assert sorted(c["tag"].tolist()) == [3, 5] and (c["status"] == 12).all()  # CANCELLED
    ex.delay = 1
    comps = drive(srv)
    assert sorted(comps["tag"].tolist()) == [0, 1, 2, 4] and (comps["status"] == 0).all()
    for x in comps:
        t = int(x["tag"])
        assert (x["counts"][:w.k[t]] == w.expected(t)).all()
    st = srv.stats()
    assert st["cancelled"] == 2 and st["arena_used_now"] == 0 and st["completed"] == 6


def test_timeout_argument_checks():
    host = np.zeros(64, np.uint8)
    r = S.requests([host.ctypes.data] * 3, [4, 4, 4], [8, 8, 8], timeouts=[-1.0, np.nan, 0.5])
    ex = FakeExecutor(1 << 20)
    srv = S.Server(1 << 20, executor=ex.ops)
    srv.submit(r)
    c = srv.take_completions()
    assert c["status"].tolist() == [7, 7]  # negative and NaN timeouts: PPC_ERR_ARG
    comps = drive(srv)
    assert comps["status"].tolist() == [0]


@pytest.mark.parametrize("in_place", [False, True])
def test_copy_slab_holds_the_source_shift(in_place):
    """In copy mode a request's copy starts at its source address modulo 16 inside its
    slab, which is sized for that; in place the slab is the input size."""
    host = I.generate(4096, I.Dist.uniform(), 13)
    base = (host.ctypes.data + 15) & ~15
    r = S.requests([base + 1, base + 512 + 15], [256, 240], [8, 8], tags=[0, 1])
    ex = FakeExecutor(1 << 20, delay=10 ** 9)
    srv = S.Server(1 << 20, max_requests=10, max_batch=10, streams=1, in_place=in_place,
                   executor=ex.ops)
    srv.submit(r)
    srv.progress()
    # 256 + 1 bytes need two granules in copy mode; 240 + 15 fit one
    assert srv.stats()["arena_used_now"] == (768 if not in_place else 512)
    ex.delay = 1
    comps = drive(srv)
    comps = comps[np.argsort(comps["tag"])]
    items = ex.log
    assert (comps["status"] == 0).all() and items == [[0, 1]]
    shift = np.array([1, 15]) if not in_place else np.array([0, 0])
    assert ((comps["arena_offset"] - shift) % 256 == 0).all()


@pytest.mark.parametrize("seed", range(6))
def test_randomized_schedules_keep_the_invariants(seed):
    """Random arrivals, sizes, slot and memory limits, launch delays, failed launches,
    timeouts and cancellations: every request completes exactly once, with its own counts
    or the status of what happened to it; slabs stay inside the arena and never overlap;
    without bypass, launches follow arrival order; the arena drains."""
    import time
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    m = 120
    w = Workload(m, 200 + seed, max_bytes=int(rng.integers(500, 20_000)))
    arena = int(rng.integers(24 << 10, 256 << 10))
    fail = set(rng.choice(40, size=int(rng.integers(0, 4)), replace=False).tolist())
    ex = FakeExecutor(arena, delay=int(rng.integers(1, 6)), fail_launches=fail)
    bypass = bool(rng.integers(0, 2))
    srv = S.Server(arena, max_requests=int(rng.integers(2, 40)), max_batch=int(rng.integers(1, 12)),
                   streams=int(rng.integers(1, 4)), fifo_bypass=bypass, executor=ex.ops)
    reqs = w.reqs.copy()
    timed = rng.random(m) < 0.2
    reqs["timeout"] = np.where(timed, 1e-4, 0.0)
    cancel_at = {int(i): int(rng.integers(0, 30)) for i in rng.choice(m, size=10, replace=False)}
    done = []
    step, nxt = 0, 0
    reqs["arrival"] = 0.0
    while len(done) < m and step < 20_000:
        burst = int(rng.integers(0, 6))
        if nxt < m and burst:
            batch = reqs[nxt:nxt + burst].copy()
            batch["arrival"] = srv.now()
            srv.submit(batch)
            nxt += len(batch)
        for tag, when in list(cancel_at.items()):
            if when == step:
                srv.cancel(tag)
                del cancel_at[tag]
        if rng.random() < 0.05:
            time.sleep(2e-4)  # lets the short timeouts pass now and then
        srv.progress()
        done.extend(srv.take_completions())
        step += 1
    comps = np.array(done, dtype=S.COMPLETION_DTYPE)
    assert not ex.errors, ex.errors
    assert sorted(comps["tag"].tolist()) == list(range(m)), "each request completes once"
    failed_tags = {t for i, launch in enumerate(ex.log) if i in fail for t in launch}
    for c in comps:
        t = int(c["tag"])
        st = int(c["status"])
        if st == 0:
            k = int(w.k[t])
            assert (c["counts"][:k] == w.expected(t)).all(), f"request {t}"
        elif st == 5:
            assert t in failed_tags
        elif st == 11:
            assert timed[t]
        else:
            assert st == 12, (t, st)  # cancelled
    launched = [t for launch in ex.log for t in launch]
    assert len(launched) == len(set(launched))
    if not bypass:
        assert launched == sorted(launched), "FIFO admission keeps arrival order"
    st = srv.stats()
    assert st["arena_used_now"] == 0 and st["inflight_now"] == 0 and st["queued_now"] == 0
    assert st["arena_peak"] <= arena
    assert st["completed"] == m and st["submitted"] == m
