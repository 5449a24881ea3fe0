"""The single-stream, wide-word and histogram entry points, and the allocation-free
batched count, allocate nothing and enqueue only kernels on the caller's stream, so
they can be captured into a HIP graph: a captured sequence, replayed several times
with eager work and synchronisations in between, adds exactly one eager pass per
replay each time."""
import numpy as np
import pytest
import torch

from paper_1911_02696_amd import api
from paper_1911_02696_amd import batch as B
from paper_1911_02696_amd import inputs as I

from gpu_util import counts_np, host_bytes, oracle_counts, say, to_device

pytestmark = pytest.mark.gpu
SEED = I.BASE_SEED + 8


def test_entry_points_replay_from_a_graph():
    n16, n64, nid, nl = 1_000_003, 250_001, 700_001, 100_003
    b16, o16 = to_device(host_bytes(2 * n16, I.Dist.uniform(), SEED), 3)
    h64 = host_bytes(8 * n64, I.Dist.bernoulli(0.3), SEED + 1)
    b64, o64 = to_device(h64, 5)
    ids, oid = to_device(host_bytes(nid, I.Dist.ids(8, 16, 1.1, 0.02), SEED + 2), 1)
    planes = [to_device(host_bytes(2 * nl, I.Dist.uniform(), SEED + 3 + j), j)[0]
              for j in range(3)]
    offs = list(range(3))

    def calls(c16, c64, ch, cp):
        api.pospopcnt(b16, 16, n=n16, byte_offset=o16, out=c16)
        api.pospopcnt(b64, 64, n=n64, byte_offset=o64, out=c64)
        api.histogram(ids, 16, id_bytes=1, n=nid, byte_offset=oid, out=ch)
        api.pospopcnt_planes(planes, n=nl, byte_offsets=offs, out=cp)

    def fresh():
        return (torch.zeros(16, dtype=torch.int64, device="cuda"),
                torch.zeros(64, dtype=torch.int64, device="cuda"),
                torch.zeros(17, dtype=torch.int64, device="cuda"),
                torch.zeros(48, dtype=torch.int64, device="cuda"))

    say("graph: eager reference")
    ref = fresh()
    calls(*ref)
    ref = [counts_np(t) for t in ref]
    assert (ref[1] == oracle_counts(h64, n64, 64)).all()

    # warm-up on a side stream, then capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls(*fresh())
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    outs = fresh()
    g = torch.cuda.CUDAGraph()
    say("graph: capture")
    with torch.cuda.graph(g):
        calls(*outs)
    torch.cuda.synchronize()
    for r in range(1, 4):
        say(f"graph: replay {r}")
        g.replay()
        eager = fresh()
        calls(*eager)  # eager work between replays
        torch.cuda.synchronize()
        for name, got, one, e in zip(("u16", "u64", "histogram", "planes"), outs, ref, eager):
            assert (counts_np(got) == r * one).all(), (name, r)
            assert (counts_np(e) == one).all(), (name, r)


@pytest.mark.parametrize("form", ["static", "plan"])
@pytest.mark.parametrize("m", [700, 5000])  # single-block and split preparation
def test_batch_replays_from_a_graph(m, form):
    """The batched count captured into the caller's graph after a first eager call:
    pospopcnt_batch_static (whose first call looks up its scratch array's address), or
    pospopcnt_batch on a plan made without its own graph.  Replayed three times; between
    replays an eager call on the same stream uses the same scratch for another counts
    table."""
    s = I.loguniform_streams(m, 14, SEED + 10 + m)
    s.lengths[::37] = 0
    nb = s.nbytes.astype(np.int64)
    starts, size = I.batch_layout(nb, SEED + 10 + m)
    host = np.zeros(size + 64, np.uint8)
    I.fill_streams(host, s, starts, SEED + 10 + m)
    dev = torch.from_numpy(host).cuda()
    tables = []
    for _ in range(2):
        counts = torch.zeros((m, 32), dtype=torch.int64, device="cuda")
        d = B.descriptors(dev.data_ptr() + starts, s.lengths, s.ks,
                          counts.data_ptr() + 256 * np.arange(m))
        tables.append((counts, B.to_device(d)))
    (c_graph, d_graph), (c_eager, d_eager) = tables
    if form == "static":
        run = B.batch_static
    else:
        plan = B.Plan(m)
        run = plan.run
    say(f"graph: {form} batch m={m}, eager reference")
    run(d_eager)
    torch.cuda.synchronize()
    one = c_eager.cpu().numpy().copy()
    for i in range(0, m, max(1, m // 40)):
        k, n, st = int(s.ks[i]), int(s.lengths[i]), int(starts[i])
        assert (one[i, :k] == oracle_counts(host[st:st + n * k // 8], n, k)).all(), i
    g = torch.cuda.CUDAGraph()
    say(f"graph: {form} batch m={m}, capture")
    with torch.cuda.graph(g):
        run(d_graph)
    torch.cuda.synchronize()
    assert (c_graph.cpu().numpy() == 0).all()  # capture alone runs nothing
    for r in range(1, 4):
        say(f"graph: {form} batch m={m}, replay {r}")
        g.replay()
        c_eager.zero_()
        run(d_eager)  # the same scratch, between replays
        torch.cuda.synchronize()
        assert (c_graph.cpu().numpy() == r * one).all(), r
        assert (c_eager.cpu().numpy() == one).all(), r
    del g
    if form == "plan":
        plan.close()
