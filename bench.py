#!/usr/bin/env python3
"""Benchmark of the positional population count on one MI355X.

A step is one pass of the whole path over the workload: one pospopcnt16 call
over a single stream of 2^33 uint16 words (16 GiB, each bit Bernoulli(1/2)),
resident in HBM before timing starts, adding into 16 uint64 counters.

Prints one JSON line: input GB/s of the timed steps, the roofline of the
counting kernel (achieved algorithmic bytes / its average launch duration,
measured with HIP events on the stream it runs on, against 8 TB/s HBM), the
read-only ceiling kernel on the same buffer, and the CPU oracle timed on a
bounded sample of the same input.  After timing, the counts are checked:
the total equals (warmup + steps) times one pass, and the GPU counts of the
sample equal the oracle's.

Further legs, reported in the same line: 20,000 uneven streams in one batched
launch against one launch per stream ("batched"), a Poisson request trace
through the serving loop with latency percentiles ("serving"), the histogram of
categorical ids through their one-hot codes ("histogram"), and 64-bit words,
plain and as 16-bit planes ("wide").  --legs selects a subset.  Each leg checks
its results by properties of the GPU results themselves (passes agree, one
route equals another); their parity with the oracle is the test suite's.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1911_02696_amd import inputs as I  # noqa: E402

HBM_PEAK_GBPS = 8000.0
# The headline metric this benchmark reports: single-stream pospopcnt16 GB/s is the
# line's value; the batched rate and the serving latencies are fields beside it.
METRIC = "pospopcnt16 input GB/s & % of HBM peak (single vs batched); p50/p99 request latency"
SEED = I.BASE_SEED

# name -> (k, n words, distribution, description)
WORKLOADS = {
    "u16_2p33": (16, 1 << 33, I.Dist.uniform(),
                 "single pospopcnt16 stream, 2^33 uint16 words (16 GiB), Bernoulli(0.5) bits"),
    "u16_2p30": (16, 1 << 30, I.Dist.uniform(), "pospopcnt16, 2^30 uint16 words (2 GiB)"),
    "u16_2p31": (16, 1 << 31, I.Dist.uniform(), "pospopcnt16, 2^31 uint16 words (4 GiB)"),
    "u16_2p32": (16, 1 << 32, I.Dist.uniform(), "pospopcnt16, 2^32 uint16 words (8 GiB)"),
    "u8_2p28": (8, 1 << 28, I.Dist.uniform(), "pospopcnt8, 2^28 uint8 words (256 MiB)"),
    "u16_2p28": (16, 1 << 28, I.Dist.uniform(), "pospopcnt16, 2^28 uint16 words (512 MiB)"),
    "u32_2p28": (32, 1 << 28, I.Dist.uniform(), "pospopcnt32, 2^28 uint32 words (1 GiB)"),
    "u8_2p34": (8, 1 << 34, I.Dist.uniform(), "pospopcnt8, 2^34 uint8 words (16 GiB)"),
    "u32_2p32": (32, 1 << 32, I.Dist.uniform(), "pospopcnt32, 2^32 uint32 words (16 GiB)"),
    "u16_2p20": (16, 1 << 20, I.Dist.uniform(), "pospopcnt16, 2^20 uint16 words (2 MiB)"),
}
DEFAULT_WORKLOAD = "u16_2p33"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ppc_single.hip", "ppc_device.h"):
        with open(os.path.join(ROOT, "paper_1911_02696_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag: str, workload: str, src_hash: str, per_launch_algo_bytes: int):
    """HBM bytes per launch from the committed PMC summary of this kernel and
    workload, if the summary was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel_tag}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        m = re.match(r"^\s*([a-z_0-9]+)\s*[:=]\s*([0-9a-fx.eE+-]+)\s*$", line.strip())
        if m:
            vals[m.group(1)] = m.group(2)
    if vals.get("kernel_source_sha256") != src_hash:
        return None
    try:
        fetch = float(vals["fetch_kib_per_dispatch"]) * 1024 * float(vals.get("fetch_scale", 1))
        write = float(vals["write_kib_per_dispatch"]) * 1024 * float(vals.get("write_scale", 1))
    except KeyError:
        return None
    return {"hbm_bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "vs_algorithmic": (fetch + write) / per_launch_algo_bytes, "source": os.path.relpath(path, ROOT)}


def upload(dev, nbytes, dist, seed, chunk=1 << 30):
    import torch
    pinned = torch.empty(min(chunk, nbytes), dtype=torch.uint8).pin_memory()
    pn = pinned.numpy()
    for first in range(0, nbytes, chunk):
        m = min(chunk, nbytes - first)
        I.fill(pn[:m], dist, seed, first_byte=first)
        dev[first:first + m].copy_(pinned[:m], non_blocking=False)


def cpu_baseline(k, dist, seed, target_s: float, max_bytes: int):
    """The oracle on the first S bytes of the same input, S sized for ~target_s of
    wall time on all host threads (the median of 3 runs when each takes under 5 s),
    plus one single-thread run on the first 256 MiB; returns (report, counts of the
    sample, S)."""
    import oracle
    threads = I.default_threads()
    probe = 64 << 20
    host = I.generate(probe, dist, seed)
    t0 = time.perf_counter()
    oracle.count(host, probe // (k // 8), k, threads=threads)
    rate = probe / max(time.perf_counter() - t0, 1e-6)
    s = int(min(max_bytes, max(probe, rate * target_s)))
    s -= s % (1 << 20)
    host = I.generate(s, dist, seed)
    times = []
    while True:
        t0 = time.perf_counter()
        counts = oracle.count(host, s // (k // 8), k, threads=threads)
        times.append(time.perf_counter() - t0)
        if len(times) == 3 or times[0] > 5.0:
            break
    used = oracle.get().threads_used
    dt = float(np.median(times))
    one = min(s, 256 << 20)
    t0 = time.perf_counter()
    oracle.count(host[:one], one // (k // 8), k, threads=1)
    dt1 = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    rep = {"value": round(s / dt / 1e9, 4), "unit": "GB/s", "cores": used, "kind": "oracle",
           "sample": f"first {s} bytes ({s // (k // 8)} words) of the same input, "
                     f"{used} threads, median of {len(times)} runs, {dt:.2f} s",
           "words_per_s": round(s // (k // 8) / dt, 1), "cpu": model,
           "single_thread": {"value": round(one / dt1 / 1e9, 4), "unit": "GB/s",
                             "sample": f"first {one} bytes, 1 thread, {dt1:.2f} s"}}
    return rep, counts, s


def batched_leg(args, torch, api):
    """The 20,000-stream uneven mix: one prefix + one persistent kernel per step
    (autotuned, replayed from a HIP graph) against one launch per stream, plain and
    graph-captured.  Returns the report and whether the checks passed: the counts of
    every pass agree, and equal the per-stream launches of the single-stream kernel."""
    from paper_1911_02696_amd import batch as B
    seed = SEED + 3
    streams = I.loguniform_streams(20_000, 22, seed)
    nb = streams.nbytes.astype(np.int64)
    starts, size = I.batch_layout(nb, seed)
    total = int(nb.sum())
    print(f"[bench] batched: {len(nb)} streams, {total / 1e9:.2f} GB", file=sys.stderr, flush=True)
    host = np.zeros(size + 64, np.uint8)
    I.fill_streams(host, streams, starts, seed, threads=I.default_threads())
    dev = torch.from_numpy(host).cuda()
    m = len(nb)
    counts = torch.zeros((m, 32), dtype=torch.int64, device="cuda")
    desc_host = B.descriptors(dev.data_ptr() + starts, streams.lengths, streams.ks,
                              counts.data_ptr() + 256 * np.arange(m))
    descs = B.to_device(desc_host)
    stream = torch.cuda.current_stream()
    profile = args.batched_profile
    plan = B.Plan(m, graph=not profile)
    if profile:
        # for counter profiling: the tuner's usual choice, set directly, and no graph
        plan.config = {"depth": 16, "block_threads": 64, "blocks_per_cu": 4,
                       "stream_weight": 2048}
        tuned_ms = float("nan")
    else:
        tuned_ms = plan.autotune(descs)

    def timed(fn, steps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, ev0.elapsed_time(ev1) / 1e3 / steps

    for _ in range(args.warmup):
        plan.run(descs)
    torch.cuda.synchronize()
    counts.zero_()
    wall, ev = timed(lambda: plan.run(descs), args.steps)
    got = counts.cpu().numpy() // args.steps
    ok_rep = bool((counts.cpu().numpy() == got * args.steps).all())

    if profile:
        cfg = plan.config
        del dev
        plan.close()
        return {"bytes": total, "streams": m, "value": round(total / wall / 1e9, 2),
                "unit": "GB/s", "event_ms_per_step": round(ev * 1e3, 4), "config": cfg,
                "graph": False, "check": {"steps_consistent": ok_rep}}, ok_rep

    counts.zero_()
    each_steps = 3
    B.pospopcnt_each(desc_host)  # warm
    torch.cuda.synchronize()
    counts.zero_()
    each_wall, each_ev = timed(lambda: B.pospopcnt_each(desc_host), each_steps)
    each = counts.cpu().numpy() // each_steps
    ok_each = bool((each == got).all())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.pospopcnt_each(desc_host)
    g.replay()
    torch.cuda.synchronize()
    gwall, gev = timed(lambda: g.replay(), each_steps)

    del dev
    rep = {
        "workload": "20,000 streams, lengths log-uniform in [1, 2^22] words, k uniform in "
                    "{8,16,32}, Bernoulli(p) bits with p ~ U(0,1), start offsets 0..15",
        "bytes": total, "streams": m,
        "value": round(total / wall / 1e9, 2), "unit": "GB/s",
        "frac_of_hbm_peak": round(total / wall / 1e9 / HBM_PEAK_GBPS, 4),
        "ms_per_step": round(wall * 1e3, 4), "event_ms_per_step": round(ev * 1e3, 4),
        "config": plan.config, "autotune_best_ms": round(tuned_ms, 4), "graph": True,
        "per_stream_launches": {"value": round(total / each_wall / 1e9, 2),
                                "ms_per_step": round(each_wall * 1e3, 3),
                                "event_ms_per_step": round(each_ev * 1e3, 3)},
        "per_stream_launches_graph": {"value": round(total / gwall / 1e9, 2),
                                      "ms_per_step": round(gwall * 1e3, 3)},
        "speedup_vs_per_stream": round(each_wall / wall, 2),
        "speedup_vs_per_stream_graph": round(gwall / wall, 2),
        "check": {"steps_consistent": ok_rep, "equals_per_stream": ok_each},
    }
    plan.close()
    return rep, ok_rep and ok_each


def serving_leg(args, torch, api):
    """Poisson arrivals at 50,000 requests/s for args.serve_seconds through the
    continuous-batching server (64 GiB arena, inputs copied into it from
    device-resident pools), then a shorter run counting in place.  Checks: every
    request succeeds, and a sample equals the same input counted alone."""
    from paper_1911_02696_amd import serve as S
    seed = SEED + 4
    pool_bytes = 1 << 29
    trace = I.serving_trace(args.serve_rate, args.serve_seconds, seed, pool_bytes=pool_bytes)
    print(f"[bench] serving: {len(trace.arrival)} requests over {args.serve_seconds} s, "
          f"{trace.nbytes.sum() / 1e12:.2f} TB", file=sys.stderr, flush=True)
    pools = S.Pools(trace, pool_bytes, seed)
    reqs = pools.requests(trace)
    report = {"workload": f"Poisson arrivals {args.serve_rate:,.0f} req/s, lengths log-uniform in "
                          "[2^10, 2^26] words, k uniform in {8,16,32}, one-hot Zipf(1.1) or "
                          "Bernoulli(0.5) inputs from device-resident pools", "arena_bytes": 64 << 30,
              "max_requests": 4096, "max_batch": 1024, "streams": 4}
    ok = True
    for mode, seconds in (("copy", args.serve_seconds), ("in_place", min(3.0, args.serve_seconds))):
        r = reqs[trace.arrival < seconds]
        srv = S.Server(64 << 30, max_requests=4096, max_batch=1024, streams=4,
                       in_place=(mode == "in_place"))
        warm = r[:2000].copy()
        warm["arrival"] = np.linspace(0, 0.02, len(warm))
        srv.run_trace(warm)
        warm_bytes = srv.stats()["bytes_counted"]
        srv.close()
        srv = S.Server(64 << 30, max_requests=4096, max_batch=1024, streams=4,
                       in_place=(mode == "in_place"))
        comps = srv.run_trace(r)
        st = srv.stats()
        srv.close()
        good = comps["status"] == 0
        span = float(comps["completed"].max() - comps["arrival"].min())
        lat = S.latency_summary(comps)
        # sample check: the same request counted alone
        rng = np.random.Generator(np.random.PCG64(seed))
        sample = np.unique(np.concatenate([rng.choice(len(r), 100, replace=False),
                                           np.argsort(trace.nbytes[:len(r)])[-20:]]))
        ok_alone = True
        out = torch.zeros(32, dtype=torch.int64, device="cuda")
        for i in sample:
            k, n = int(trace.ks[i]), int(trace.lengths[i])
            got = comps["counts"][i][:k]
            out.zero_()
            api.pospopcnt_ptr(int(r[i]["src"]), n, k, out.data_ptr())
            ok_alone &= bool((out.cpu().numpy()[:k] == got.astype(np.int64)).all())
        ok &= bool(good.all()) and ok_alone
        report[mode] = dict(lat, seconds=seconds, gbps=round(st["bytes_counted"] / span / 1e9, 1),
                            requests_per_s=round(len(r) / span, 1),
                            launches=st["launches"], admitted=st["admitted"],
                            bytes_counted=st["bytes_counted"], warmup_bytes_counted=warm_bytes,
                            rejected=st["rejected"], max_queued=st["max_queued"],
                            max_inflight=st["max_inflight"],
                            arena_peak_gib=round(st["arena_peak"] / 2**30, 3),
                            check={"all_ok": bool(good.all()),
                                   f"alone_equals_in_mix_{len(sample)}": ok_alone})
    del pools
    torch.cuda.empty_cache()
    return report, ok


def onehot_leg(args, torch, api):
    """Histogram of 16 GiB of categorical ids (u8: 2^34 ids, u16: 2^33 ids) for 8, 16
    and 32 categories.  Ids follow Zipf(1.1) over the categories, every id a category
    as in the paper's example (Table 1); two more cases put 1% of the ids outside the
    categories, which sends nearly every tile through the masked code path.  The first
    GiB of each id stream is generated and repeated over the 16 GiB on the device (1 GiB
    is far beyond the 256 MB last-level cache, so every pass still reads HBM).  Checks:
    the totals of every pass add up to the id count, and on the first 256 MiB the
    histogram equals pospopcnt over the same ids written out as one-hot words by torch,
    with the ids outside the categories counted by torch."""
    out = {}
    ok = True
    nbytes, gen = 1 << 34, 1 << 30
    dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    cases = [(idb, bins, 0.0) for idb in (1, 2) for bins in (8, 16, 32)]
    cases += [(1, 8, 0.01), (2, 16, 0.01)]
    for id_bytes, bins, p_invalid in cases:
        dist = I.Dist.ids(8 * id_bytes, bins, 1.1, p_invalid)
        upload(dev, gen, dist, SEED + 6)
        for c in range(1, nbytes // gen):
            dev[c * gen:(c + 1) * gen].copy_(dev[:gen])
        n = nbytes // id_bytes
        counts = torch.zeros(bins + 1, dtype=torch.int64, device="cuda")
        for _ in range(args.warmup):
            api.histogram(dev, bins, id_bytes=id_bytes, out=counts)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            api.histogram(dev, bins, id_bytes=id_bytes, out=counts)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / args.steps
        got = counts.cpu().numpy()
        sample = 1 << 28
        g = api.histogram(dev, bins, id_bytes=id_bytes, n=sample // id_bytes).cpu().numpy()
        exp = onehot_reference(torch, api, dev[:sample], id_bytes, bins)
        passes = args.warmup + args.steps
        good = bool((g == exp).all()) and int(got.sum()) == n * passes
        ok &= good
        name = f"u{8 * id_bytes}_bins{bins}" + ("_1pct_invalid" if p_invalid else "")
        out[name] = {
            "ids": n, "gbps": round(nbytes / t / 1e9, 1),
            "frac_of_hbm_peak": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4),
            "ids_per_s": round(n / t, 1), "ms": round(t * 1e3, 4),
            "invalid_ids_per_pass": int(got[bins]) // passes, "check": good}
    del dev
    torch.cuda.empty_cache()
    return out, ok


def onehot_reference(torch, api, raw, id_bytes, bins):
    """The histogram of the ids in ``raw`` by another route: torch writes each id below
    ``bins`` as the word 1 << id of ``bins`` bits (an id outside the categories as 0),
    pospopcnt counts those words, and torch counts the ids outside."""
    ids = raw.to(torch.int64) if id_bytes == 1 else raw.view(torch.int16).to(torch.int64) & 0xFFFF
    valid = ids < bins
    words = torch.where(valid, torch.ones_like(ids) << ids.clamp(max=bins - 1), 0)
    words = words.to(torch.int32).view(torch.uint8).view(-1, 4)[:, :bins // 8].contiguous()
    exp = np.zeros(bins + 1, dtype=np.int64)
    exp[:bins] = api.pospopcnt(words, bins).cpu().numpy()
    exp[bins] = int((~valid).sum())
    return exp


def wide_leg(args, torch, api):
    """Words wider than 32 bits (Sec. 4), 16 GiB per launch: one stream of 2^31 64-bit
    words, and 64-bit words held as 4 planes of 2^31 16-bit limbs (4 GiB each).  Bits
    are Bernoulli(0.5).  Checks, over the whole 16 GiB: the 64 counts folded onto 32
    positions equal pospopcnt32 of the same bytes, each plane's 16 counts equal
    pospopcnt16 of that plane, and every pass adds the same counts."""
    out, ok = {}, True
    nbytes = 1 << 34
    stream = torch.cuda.current_stream()
    dist = I.Dist.uniform()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / args.steps

    passes = args.warmup + args.steps
    dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    upload(dev, nbytes, dist, SEED + 7)
    n = nbytes // 8
    counts = torch.zeros(64, dtype=torch.int64, device="cuda")
    t = timed(lambda: api.pospopcnt_u64(dev, n=n, out=counts))
    one = api.pospopcnt_u64(dev, n=n).cpu().numpy()
    c32 = api.pospopcnt(dev, 32, n=2 * n).cpu().numpy()
    good = bool((one[:32] + one[32:] == c32).all()) \
        and bool((counts.cpu().numpy() == one * passes).all())
    ok &= good
    out["u64_2p31"] = {"bytes": nbytes, "words": n, "gbps": round(nbytes / t / 1e9, 1),
                       "frac_of_hbm_peak": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4),
                       "ms": round(t * 1e3, 4), "check": good}
    m = 4
    per = nbytes // m
    planes = [dev[j * per:(j + 1) * per] for j in range(m)]
    for j in range(m):
        upload(planes[j], per, dist, SEED + 8 + j)
    n = per // 2
    counts = torch.zeros(16 * m, dtype=torch.int64, device="cuda")
    t = timed(lambda: api.pospopcnt_planes(planes, n=n, out=counts))
    one = api.pospopcnt_planes(planes, n=n).cpu().numpy()
    each = np.concatenate([api.pospopcnt(planes[j], 16, n=n).cpu().numpy() for j in range(m)])
    good = bool((one == each).all()) and bool((counts.cpu().numpy() == one * passes).all())
    ok &= good
    out["planes16_4x2p31"] = {"bytes": nbytes, "words": n, "k": 16 * m,
                              "gbps": round(nbytes / t / 1e9, 1),
                              "frac_of_hbm_peak": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4),
                              "ms": round(t * 1e3, 4), "check": good}
    del dev, planes
    torch.cuda.empty_cache()
    return out, ok


def calls_leg(args, torch, api):
    """The fixed cost of one call on a small input (C1: 2^20 uint16 words, 2 MiB,
    resident in the last-level cache): host time per call of 2000 back-to-back
    pospopcnt16 calls through the Python binding, and the same from C through the
    library's C ABI (the C caller in tests/c_abi, when built).  The kernel itself takes
    a few microseconds, so both are bound by the host's launch path."""
    import subprocess
    n, calls = 1 << 20, 2000
    x = torch.full((2 * n,), 0x5A, dtype=torch.uint8, device="cuda")
    out = torch.zeros(16, dtype=torch.int64, device="cuda")
    for _ in range(100):
        api.pospopcnt(x, 16, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        api.pospopcnt(x, 16, out=out)
    torch.cuda.synchronize()
    py_us = (time.perf_counter() - t0) / calls * 1e6
    want = np.array([n * (calls + 100) if (0x5A5A >> q) & 1 else 0 for q in range(16)])
    ok = bool((out.cpu().numpy() == want).all())
    rep = {"workload": "2^20 uint16 words (2 MiB), 2000 back-to-back calls on one stream",
           "python_us_per_call": round(py_us, 3), "python_gbps": round(2 * n / py_us / 1e3, 1)}
    exe = os.path.join(ROOT, "tests", "c_abi", "abi_check")
    if os.path.exists(exe):
        res = subprocess.run([exe, "calls", str(calls)], capture_output=True, text=True)
        c = json.loads(res.stdout.strip().splitlines()[-1]) if res.returncode == 0 else None
        ok &= c is not None and c.get("ok", False)
        if c:
            rep["c_us_per_call"] = c["c_us_per_call"]
            rep["python_over_c"] = round(py_us / c["c_us_per_call"], 2)
    rep["check"] = ok
    del x
    return rep, ok


def variants_leg(args, torch, api):
    """The three counting kernels on the same 16 GiB of Bernoulli(0.5) bytes, read as
    8-, 16- and 32-bit words, each at its default launch shape: the per-lane CSA circuit
    (csa), the wave-wide ballot transposition (ballot) and the CSA circuit with its
    carries counted by ballot (hybrid).  Timed with HIP events over args.steps launches
    after args.warmup.  Check: every variant's counts equal the CSA kernel's."""
    nbytes = 1 << 34
    dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    upload(dev, nbytes, I.Dist.uniform(), SEED + 9)
    stream = torch.cuda.current_stream()
    out, ok = {"bytes": nbytes}, True
    for k in (8, 16, 32):
        n = nbytes // (k // 8)
        ref = api.pospopcnt(dev, k, n=n).cpu().numpy()
        row = {}
        for variant in ("csa", "hybrid", "ballot"):
            counts = torch.zeros(k, dtype=torch.int64, device="cuda")
            for _ in range(args.warmup):
                api.pospopcnt(dev, k, n=n, out=counts, variant=variant)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                api.pospopcnt(dev, k, n=n, out=counts, variant=variant)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / max(args.steps, 1)
            good = bool((counts.cpu().numpy() == ref * (args.warmup + args.steps)).all())
            ok &= good
            row[variant] = {"gbps": round(nbytes / t / 1e9, 1),
                            "frac_of_hbm_peak": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4),
                            "check": good}
        out[f"u{k}"] = row
        print(f"[bench] variants k={k}: {row}", file=sys.stderr, flush=True)
    del dev
    torch.cuda.empty_cache()
    return out, ok


DEPTH_SHAPES = [(64, b) for b in (2, 3, 4, 6, 8, 12, 16)] + [(256, b) for b in (1, 2, 3, 4)]


def depth_leg(args, torch, api):
    """Circuit depth against throughput (Sec. 4.1 compares 256 B, 512 B and 1 kB
    circuits): for 8-, 16- and 32-bit words over the same 16 GiB of Bernoulli(0.5)
    bytes, every circuit depth (4, 8, 16, 32 dwords per lane per step) at every launch
    shape of DEPTH_SHAPES (block size x blocks per CU), each timed with HIP events
    over args.steps launches after args.warmup; reports each depth's best shape and
    its GB/s.  Check: every configuration's counts equal the default one's."""
    nbytes = 1 << 34
    dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    upload(dev, nbytes, I.Dist.uniform(), SEED + 9)
    stream = torch.cuda.current_stream()
    out, ok = {"bytes": nbytes, "shapes": [list(x) for x in DEPTH_SHAPES]}, True
    for k in (8, 16, 32):
        n = nbytes // (k // 8)
        ref = api.pospopcnt(dev, k, n=n).cpu().numpy()
        per_depth = {}
        for depth in (4, 8, 16, 32):
            rows = []
            for threads, bpc in DEPTH_SHAPES:
                cfg = dict(depth=depth, block_threads=threads, blocks_per_cu=bpc)
                counts = torch.zeros(k, dtype=torch.int64, device="cuda")
                for _ in range(args.warmup):
                    api.pospopcnt(dev, k, n=n, out=counts, **cfg)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    api.pospopcnt(dev, k, n=n, out=counts, **cfg)
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) / 1e3 / args.steps
                good = bool((counts.cpu().numpy() == ref * (args.warmup + args.steps)).all())
                ok &= good
                rows.append((round(nbytes / t / 1e9, 1), threads, bpc, good))
            best = max(rows)
            per_depth[str(depth)] = {"best_gbps": best[0], "best_block_threads": best[1],
                                     "best_blocks_per_cu": best[2],
                                     "frac_of_hbm_peak": round(best[0] / HBM_PEAK_GBPS, 4),
                                     "gbps_by_shape": [r[0] for r in rows],
                                     "check": all(r[3] for r in rows)}
            print(f"[bench] depth k={k} d={depth}: best {best[0]} GB/s at {best[1]}x{best[2]}",
                  file=sys.stderr, flush=True)
        out[f"u{k}"] = per_depth
    del dev
    torch.cuda.empty_cache()
    return out, ok


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="csa", choices=["csa", "ballot", "hybrid"])
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 20,000-stream batched leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--batched-profile", action="store_true",
                    help="batched leg for counter profiling: the tuned shape set directly, no "
                         "graph, no autotuning and no per-stream comparison")
    ap.add_argument("--legs", default="single,batched,serving,onehot,wide,calls",
                    help="comma-separated subset of single,batched,serving,onehot,wide,calls,"
                         "depth,variants to run (the full JSON line is printed only when the "
                         "single leg runs; depth, the circuit-depth sweep, and variants, the three "
                         "counting kernels side by side, run only when named)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=50_000.0,
                    help="Poisson arrival rate of the serving leg, requests/s")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-reference", type=int, default=0, metavar="BYTES",
                    help="only run --steps device-to-device copies of BYTES bytes (a plain copy "
                         "kernel of known traffic, to scale profiler byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the count would shard by byte range with one 256-byte sum per GPU; only the "
              "one-GPU path is implemented).", file=sys.stderr)
        sys.exit(2)

    legs = set(args.legs.split(","))
    if not legs <= {"single", "batched", "serving", "onehot", "wide", "calls", "depth", "variants"}:
        ap.error("--legs takes single, batched, serving, onehot, wide, calls, depth and variants")

    import torch
    from paper_1911_02696_amd import api

    if args.copy_reference:
        src = torch.ones(args.copy_reference, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes": args.copy_reference, "copies": args.steps,
                          "read_bytes_per_copy": args.copy_reference,
                          "write_bytes_per_copy": args.copy_reference}))
        return

    args.no_batched |= "batched" not in legs
    args.no_serving |= "serving" not in legs
    if "single" not in legs:
        torch.cuda.set_device(0)
        out = {}
        if "depth" in legs:
            out["depth"] = depth_leg(args, torch, api)[0]
        if "calls" in legs:
            out["calls"] = calls_leg(args, torch, api)[0]
        if "variants" in legs:
            out["variants"] = variants_leg(args, torch, api)[0]
        if "onehot" in legs:
            out["onehot"] = onehot_leg(args, torch, api)[0]
        if "wide" in legs:
            out["wide"] = wide_leg(args, torch, api)[0]
        if not args.no_batched:
            out["batched"] = batched_leg(args, torch, api)[0]
        if not args.no_serving:
            out["serving"] = serving_leg(args, torch, api)[0]
        print(json.dumps(out), flush=True)
        return

    k, n, dist, desc = WORKLOADS[args.workload]
    nbytes = n * (k // 8)
    torch.cuda.set_device(0)
    info = api.device_info()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (256 << 20):
        print(f"workload needs {nbytes / 2**30:.1f} GiB, {free / 2**30:.1f} GiB free",
              file=sys.stderr)
        sys.exit(3)
    print(f"[bench] {desc}: uploading {nbytes / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    # Inputs smaller than 1 GiB would stay in the 256 MB last-level cache between
    # steps; such workloads cycle through identical copies spanning at least 2 GiB.
    copies = 1 if nbytes >= (1 << 30) else min(1024, -(-(2 << 30) // nbytes))
    stride = -(-nbytes // 256) * 256
    dev = torch.empty(stride * copies, dtype=torch.uint8, device="cuda")
    upload(dev, nbytes, dist, SEED + 2)
    for c in range(1, copies):
        dev[c * stride:c * stride + nbytes].copy_(dev[:nbytes])
    views = [dev[c * stride:c * stride + nbytes] for c in range(copies)]
    counts = torch.zeros(k, dtype=torch.int64, device="cuda")
    cfg = dict(variant=args.variant, depth=args.depth, block_threads=args.block_threads,
               blocks_per_cu=args.blocks_per_cu)
    stream = torch.cuda.current_stream()

    one = api.pospopcnt(views[0], k, n=n, **cfg)  # one pass, for the consistency check
    for i in range(args.warmup):
        api.pospopcnt(views[i % copies], k, n=n, out=counts, **cfg)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        api.pospopcnt(views[(args.warmup + i) % copies], k, n=n, out=counts, **cfg)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]) / 1e3
    avg_kernel = float(ev[0].elapsed_time(ev[-1]) / 1e3 / args.steps)
    ms_per_step = wall / args.steps * 1e3

    total = counts.cpu().numpy()
    one_np = one.cpu().numpy()
    ok_total = bool((total == one_np * (args.warmup + args.steps)).all())

    ceiling = None
    if not args.no_ceiling:
        sink = torch.zeros(1, dtype=torch.int64, device="cuda")
        for i in range(args.warmup):
            api.read_ceiling(views[i % copies], sink=sink, depth=args.depth)
        cev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        cev[0].record(stream)
        for i in range(args.steps):
            api.read_ceiling(views[(args.warmup + i) % copies], sink=sink, depth=args.depth)
        cev[1].record(stream)
        torch.cuda.synchronize()
        c_avg = cev[0].elapsed_time(cev[1]) / 1e3 / args.steps
        ceiling = {"kernel": "ceiling_kernel (XOR of the same loads)",
                   "gbps": round(nbytes / c_avg / 1e9, 1),
                   "frac_of_peak": round(nbytes / c_avg / 1e9 / HBM_PEAK_GBPS, 4)}
        # Context from a library kernel: torch's int64 sum over the same bytes, a plain
        # streaming reduction that none of this code touches.
        words = nbytes // 8
        lib_views = [v[:8 * words].view(torch.int64) for v in views]
        for i in range(args.warmup):
            lib_views[i % copies].sum()
        lev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        lev[0].record(stream)
        for i in range(args.steps):
            lib_views[(args.warmup + i) % copies].sum()
        lev[1].record(stream)
        torch.cuda.synchronize()
        l_avg = lev[0].elapsed_time(lev[1]) / 1e3 / args.steps
        ceiling["library_read_reference"] = {
            "kernel": "torch int64 sum of the same bytes",
            "gbps": round(8 * words / l_avg / 1e9, 1),
            "frac_of_peak": round(8 * words / l_avg / 1e9 / HBM_PEAK_GBPS, 4)}

    cpu = None
    ok_sample = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu, sample_counts, s = cpu_baseline(k, dist, SEED + 2, args.cpu_seconds, nbytes)
        g = api.pospopcnt(views[0], k, n=s // (k // 8), **cfg).cpu().numpy()
        ok_sample = bool((g == sample_counts.astype(np.int64)).all())

    # Sec. 5: no branch depends on the data, so all-zero and all-one inputs must run as
    # fast as random ones (timed on the same buffer, refilled, after the checks above).
    data_independence = {"random_gbps": round(nbytes / avg_kernel / 1e9, 1)}
    for name, fill in (("zeros", 0), ("ones", 255)):
        views[0].fill_(fill)
        scratch = torch.zeros(k, dtype=torch.int64, device="cuda")
        for _ in range(2):
            api.pospopcnt(views[0], k, n=n, out=scratch, **cfg)
        dev0, dev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(3, min(args.steps, 10))
        dev0.record(stream)
        for _ in range(reps):
            api.pospopcnt(views[0], k, n=n, out=scratch, **cfg)
        dev1.record(stream)
        torch.cuda.synchronize()
        data_independence[f"{name}_gbps"] = round(nbytes / (dev0.elapsed_time(dev1) / 1e3 / reps) / 1e9, 1)
        expect_each = 0 if fill == 0 else n
        if not bool((scratch.cpu().numpy() == expect_each * (2 + reps)).all()):
            ok_total = False

    del dev, views
    torch.cuda.empty_cache()
    batched, ok_batched = None, True
    if not args.no_batched:
        batched, ok_batched = batched_leg(args, torch, api)
        torch.cuda.empty_cache()
    serving, ok_serving = None, True
    if not args.no_serving:
        serving, ok_serving = serving_leg(args, torch, api)
    onehot, ok_onehot = None, True
    if "onehot" in legs:
        onehot, ok_onehot = onehot_leg(args, torch, api)
    wide, ok_wide = None, True
    if "wide" in legs:
        wide, ok_wide = wide_leg(args, torch, api)
    depth, ok_depth = None, True
    if "depth" in legs:
        depth, ok_depth = depth_leg(args, torch, api)
    calls, ok_calls = None, True
    if "calls" in legs:
        calls, ok_calls = calls_leg(args, torch, api)

    achieved = nbytes / avg_kernel / 1e9
    src_hash = kernel_source_hash()
    kname = {"csa": "csa_kernel", "ballot": "ballot_kernel", "hybrid": "hybrid_kernel"}[args.variant]
    traffic = read_traffic(args.variant, args.workload, src_hash, nbytes)
    value = nbytes / (wall / args.steps) / 1e9
    line = {
        "metric": METRIC if k == 16 else f"pospopcnt{k} input GB/s (single stream)",
        "value_is": f"single-stream pospopcnt{k} input GB/s (wall clock over the timed steps); "
                    "the batched GB/s and % of peak are under 'batched', the serving p50/p99 "
                    "latency under 'serving'",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16" if k == 16 else f"u{k}",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "k": k, "n_words": n,
                   "bytes": nbytes, "offset": 0, "copies_cycled": copies, "variant": args.variant,
                   "depth": args.depth or None, "parallelism": "single GPU"},
        "words_per_s": round(n / (wall / args.steps), 1),
        "frac_of_hbm_peak": round(value / HBM_PEAK_GBPS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic["hbm_bytes"] if traffic else None,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled)",
                     "traffic_detail": traffic, "kernel": kname,
                     "algorithmic_bytes_per_launch": nbytes,
                     "avg_launch_ms": round(avg_kernel * 1e3, 4),
                     "min_launch_ms": round(float(per.min()) * 1e3, 4),
                     "median_launch_ms": round(float(np.median(per)) * 1e3, 4),
                     "p10_launch_ms": round(float(np.percentile(per, 10)) * 1e3, 4),
                     "p90_launch_ms": round(float(np.percentile(per, 90)) * 1e3, 4),
                     "kernel_source_sha256": src_hash},
        "ceiling": ceiling,
        "data_independence": data_independence,
        "batched": batched,
        "serving": serving,
        "histogram": onehot,
        "wide": wide,
        "depth": depth,
        "calls": calls,
        "cpu_baseline": cpu,
        "check": {"total_equals_passes_times_one_pass": ok_total,
                  "sample_equals_oracle": ok_sample},
        "device": {"name": info["name"], "arch": info["arch"], "cus": info["compute_units"],
                   "clock_mhz": info["clock_khz"] / 1000},
    }
    print(json.dumps(line), flush=True)
    if not ok_total or ok_sample is False or not ok_batched or not ok_serving or not ok_onehot \
            or not ok_wide or not ok_depth or not ok_calls:
        sys.exit(1)


if __name__ == "__main__":
    main()
