"""GPU serving in copy mode: the count itself stores every input byte it reads
into the request's slab of the server's arena.  Checked byte for byte: the arena
starts filled with a sentinel byte, and after a run every arena byte must equal
the byte of the last launched request whose copy covered it, or still the
sentinel where no copy reached (so a store before or past a slab, or a missing
one, fails).  Sources start at all 16 addresses modulo 16, the arena is far
smaller than the traffic (slabs are reused), and launches hold fewer and more
than 1024 requests (the two preparation paths).  Counts equal the oracle."""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import inputs as I
from paper_1911_02696_amd import serve as S

from gpu_util import device_fill, device_read, oracle_counts, say

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 44
SENTINEL = 0x5A
POOL = 16 << 20


class Case:
    """m requests over one device pool of mixed bytes: sizes log-uniform in
    [1, max_bytes] bytes (so tiny requests that are all head or tail bytes, requests
    inside one tile and requests over many blocks), k uniform over {8, 16, 32},
    source address = pool + 16 * j + (i mod 16)."""

    def __init__(self, m, max_bytes, seed):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.host = np.concatenate([I.generate(POOL // 2, I.Dist.uniform(), seed),
                                    I.generate(POOL // 2, I.Dist.onehot(16, 1.1), seed + 1)])
        self.dev = torch.from_numpy(self.host).cuda()
        self.k = rng.choice(np.array([8, 16, 32]), size=m)
        wb = self.k // 8
        nb = np.rint(np.exp(rng.random(m) * np.log(max_bytes))).astype(np.int64)
        self.n = np.maximum(nb // wb, 1)
        self.nbytes = self.n * wb
        shift = np.arange(m) % 16
        room = (POOL - self.nbytes - 16) // 16
        self.off = (rng.integers(0, 1 << 62, size=m) % room) * 16 + shift
        self.reqs = S.requests(self.dev.data_ptr() + self.off, self.n, self.k)

    def src(self, i):
        return self.host[self.off[i]:self.off[i] + self.nbytes[i]]


def drive(srv, reqs):
    srv.submit(reqs)
    got = []
    while sum(len(c) for c in got) < len(reqs):
        srv.progress()
        got.append(srv.take_completions())
    return np.concatenate(got)


def check_run(case, comps, arena_ptr, arena_bytes):
    m = len(case.reqs)
    assert len(comps) == m and (comps["status"] == 0).all(), np.unique(comps["status"])
    comps = comps[np.argsort(comps["tag"])]
    for i in range(m):
        k = int(case.k[i])
        exp = oracle_counts(case.src(i), int(case.n[i]), k)
        assert (comps["counts"][i][:k].astype(np.int64) == exp).all(), f"request {i}"
    # copies start at the source's address modulo 16
    assert ((comps["arena_offset"] - case.off) % 16 == 0).all()
    # the arena after the run: each byte from the last launched copy over it
    model = np.full(arena_bytes, SENTINEL, np.uint8)
    for i in np.lexsort((comps["tag"], comps["launched"])):
        o = int(comps["arena_offset"][i])
        assert o + int(case.nbytes[i]) <= arena_bytes
        model[o:o + int(case.nbytes[i])] = case.src(i)
    got = device_read(arena_ptr, arena_bytes)
    bad = np.nonzero(got != model)[0]
    assert bad.size == 0, f"{bad.size} arena bytes differ, first at {bad[:8]}"


@pytest.mark.parametrize("max_batch,m,max_bytes,arena", [
    (64, 3000, 1 << 18, 4 << 20),      # launches of up to 64 requests, direct and copied tables
    (4096, 6000, 4096, 1 << 20),       # launches of more than 1024 requests
    (8, 400, 6 << 20, 12 << 20),       # requests split over many blocks
])
def test_copies_and_counts_are_exact(max_batch, m, max_bytes, arena):
    case = Case(m, max_bytes, SEED + m)
    say(f"serve copy: {m} requests up to {max_bytes} B, max_batch {max_batch}, arena {arena}")
    srv = S.Server(arena, max_requests=max(max_batch, 256), max_batch=max_batch, streams=2)
    ptr, size = srv.arena()
    assert ptr and size == arena
    device_fill(ptr, SENTINEL, arena)
    comps = drive(srv, case.reqs)
    st = srv.stats()
    assert st["launches"] > 1 and st["max_queued"] > 0 and st["arena_used_now"] == 0
    assert int(case.nbytes.sum()) > arena  # slabs were reused
    if max_batch > 1024:
        assert comps["batch"].max() > 1024, np.unique(comps["batch"])
    check_run(case, comps, ptr, arena)
    srv.close()


@pytest.mark.parametrize("in_place,big", [(False, False), (True, False), (False, True)],
                         ids=["copy", "in_place", "copy_large_launches"])
def test_failed_launch_is_reported_and_serving_goes_on(monkeypatch, in_place, big):
    """The executor's third launch fails after its count was enqueued (fault hook):
    its requests complete with PPC_ERR_HIP, its slabs and slots drain, and every
    later request -- including those of later launches on the same counters, which
    the failure path must have cleared -- equals the oracle.  With large launches
    (more than 1024 requests) the count runs as a preparation and a main kernel."""
    case = Case(5000, 512, SEED + 8) if big else Case(300, 1 << 16, SEED + 7)
    monkeypatch.setenv("PPC_FAULT_LAUNCH", "3")
    srv = S.Server(1 << 22 if big else 1 << 20, max_requests=2048 if big else 64,
                   max_batch=1100 if big else 8, streams=1, in_place=in_place)
    monkeypatch.delenv("PPC_FAULT_LAUNCH")
    say(f"serve fault hook: launch 3 of {len(case.reqs)} requests fails, in_place={in_place}")
    comps = drive(srv, case.reqs)
    st = srv.stats()
    srv.close()
    failed = comps[comps["status"] != 0]
    assert len(failed) > 0 and (failed["status"] == 5).all(), np.unique(comps["status"])
    assert len(np.unique(failed["launched"])) == 1 and len(failed) == int(failed["batch"][0])
    assert st["arena_used_now"] == 0 and st["inflight_now"] == 0 and st["queued_now"] == 0
    assert st["launches"] > (3 if big else 6)
    if big:
        assert failed["batch"][0] > 1024
    later = comps[(comps["status"] == 0) & (comps["launched"] > failed["launched"][0])]
    assert len(later) > 0
    for c in comps[comps["status"] == 0]:
        i, k = int(c["tag"]), int(case.k[c["tag"]])
        exp = oracle_counts(case.src(i), int(case.n[i]), k)
        assert (c["counts"][:k].astype(np.int64) == exp).all(), f"request {i}"


def test_source_inside_the_arena_is_refused():
    """A request whose input lies in the server's own arena (where other requests' copies
    are written) completes at once with PPC_ERR_OVERLAP; the others are served."""
    case = Case(20, 4096, SEED + 9)
    srv = S.Server(1 << 20, max_requests=64, max_batch=64, streams=1)
    ptr, size = srv.arena()
    bad = S.requests([ptr + 100, ptr + size - 8, ptr - 8], [64, 64, 16], [8, 8, 8],
                     tags=[1000, 1001, 1002])
    srv.submit(bad)
    first = srv.take_completions()
    assert sorted(first["tag"].tolist()) == [1000, 1001, 1002]
    assert (first["status"] == 8).all(), first["status"]
    comps = drive(srv, case.reqs)
    srv.close()
    assert (comps["status"] == 0).all()
