"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's formula: they check it against the
paper's worked example and printed truth tables (tests/golden/), closed forms,
invariants checked with library popcounts, and a brute force built from
numpy.unpackbits.  The last test plants plausible mistakes in the oracle (on the
CPU, in separate builds) and shows that each one fails at least one pin.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import build as obuild
from paper_1911_02696_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KS = (8, 16, 32)


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def brute(buf: np.ndarray, n: int, k: int, offset: int = 0) -> np.ndarray:
    """Independent definition: unpack every byte little-bit-first, lay the bits out as
    an (n, k) matrix (byte b of a word holds word bits 8b..8b+7) and sum its columns."""
    raw = np.asarray(buf, dtype=np.uint8).reshape(-1)[offset:offset + n * k // 8]
    bits = np.unpackbits(raw, bitorder="little").reshape(n, k)
    return bits.sum(axis=0, dtype=np.uint64)


def rand_bytes(nbytes, seed, p=0.5):
    return I.generate(nbytes, I.Dist.bernoulli(p) if p != 0.5 else I.Dist.uniform(), seed)


# --------------------------------------------------------------------------- pins
# Each pin returns a list of failure strings, so that the same suite can be run on
# a planted variant of the oracle (test_planted_mistakes_are_caught).

def pin_country_example(o):
    rows = _golden("country_example.txt")
    mapping = {r[1]: int(r[2], 2) for r in rows if r[0] == "mapping"}
    stream = next(r[1:] for r in rows if r[0] == "stream")
    hist = {r[1]: int(r[2]) for r in rows if r[0] == "histogram"}
    data = np.array([mapping[c] for c in stream], dtype=np.uint8)
    fails = []
    for k in KS:  # the same values zero-extended to 16 and 32 bits
        words = data.astype({8: np.uint8, 16: np.uint16, 32: np.uint32}[k])
        c = o.count(words.view(np.uint8), len(stream), k)
        for name, expect in hist.items():
            bit = mapping[name].bit_length() - 1
            if int(c[bit]) != expect:
                fails.append(f"k={k}: {name} counted {int(c[bit])}, paper says {expect}")
        if int(c[8:].sum()) != 0:
            fails.append(f"k={k}: counts above bit 7 must be zero")
        if int(c.sum()) != len(stream):
            fails.append(f"k={k}: one-hot counts must sum to n")
    return fails


def pin_csa_truth_tables(o):
    rows = _golden("csa_truth_tables.txt")
    imm = {r[1]: int(r[2]) for r in rows if r[0] == "immediate"}
    fails = []
    for r in rows:
        if r[0] != "row":
            continue
        a, b, c, lsb, msb, index = map(int, r[1:])
        if index != a + 2 * b + 4 * c:
            fails.append(f"golden row index {index}")
        ones = 2**64 - 1
        h, l = o.csa(a * ones, b * ones, c * ones)
        if l != lsb * ones or h != msb * ones:
            fails.append(f"csa({a},{b},{c}) = h{h:#x} l{l:#x}, table says msb {msb} lsb {lsb}")
        if (imm["lsb"] >> index) & 1 != lsb or (imm["msb"] >> index) & 1 != msb:
            fails.append(f"immediates disagree with row {index}")
    return fails


def pin_csa_identity(o):
    rng = np.random.Generator(np.random.PCG64(7))
    fails = []
    for _ in range(200):
        a, b, c = (int(x) for x in rng.integers(0, 2**63, size=3, dtype=np.uint64) * 2
                   + rng.integers(0, 2, size=3, dtype=np.uint64))
        h, l = o.csa(a, b, c)
        for i in range(64):
            s = (a >> i & 1) + (b >> i & 1) + (c >> i & 1)
            if s != 2 * (h >> i & 1) + (l >> i & 1):  # Sec. 2: a + b + c = 2h + l per bit
                fails.append(f"bit {i}: {s} != 2h + l")
                return fails
    return fails


def pin_closed_forms(o):
    fails = []
    allu16 = np.arange(1 << 16, dtype=np.uint16)
    if not (o.count(allu16.view(np.uint8), 1 << 16, 16) == 1 << 15).all():
        fails.append("every uint16 once must give 32768 per position")
    allu8 = np.arange(256, dtype=np.uint8)
    if not (o.count(allu8, 256, 8) == 128).all():
        fails.append("every uint8 once must give 128 per position")
    u32 = np.arange(1 << 20, dtype=np.uint32)
    c = o.count(u32.view(np.uint8), 1 << 20, 32)
    if not ((c[:20] == 1 << 19).all() and (c[20:] == 0).all()):
        fails.append("uint32 0..2^20-1 must give 2^19 below bit 20, 0 above")
    for k, w in ((8, 0xA5), (16, 0x8001), (32, 0xDEADBEEF), (64, 0x0123456789ABCDEF)):
        n = 1234
        words = np.full(n, w, dtype={8: np.uint8, 16: np.uint16, 32: np.uint32,
                                     64: np.uint64}[k])
        expect = np.array([n * ((w >> p) & 1) for p in range(k)], dtype=np.uint64)
        if not (o.count(words.view(np.uint8), n, k) == expect).all():
            fails.append(f"constant word {w:#x} repeated (k={k})")
        if not (o.count(np.zeros(n * k // 8, np.uint8), n, k) == 0).all():
            fails.append(f"all-zero input (k={k})")
        if not (o.count(np.full(n * k // 8, 255, np.uint8), n, k) == n).all():
            fails.append(f"all-ones input (k={k})")
    return fails


def pin_brute_force(o):
    fails = []
    for k in (8, 16, 32, 64):
        for n in (0, 1, 2, 3, 7, 64, 1000):
            for seed in (1, 2):
                buf = rand_bytes(n * k // 8 + 8, seed)
                for off in (0, 1, 3):
                    got = o.count(buf, n, k, offset=off)
                    if not (got == brute(buf, n, k, off)).all():
                        fails.append(f"brute force k={k} n={n} offset={off}")
    return fails


def pin_invariants(o):
    fails = []
    rng = np.random.Generator(np.random.PCG64(11))
    for k in KS:
        wb = k // 8
        n = 5003
        buf = rand_bytes(n * wb, 100 + k, p=0.3)
        c = o.count(buf, n, k)
        # (i) the k sums add up to the total popcount (library popcount)
        if int(c.sum()) != int(np.bitwise_count(buf).sum()):
            fails.append(f"k={k}: sum of counts != total popcount")
        # (iii) additivity at arbitrary split points
        for split in (0, 1, 2500, n - 1, n):
            parts = o.count(buf, split, k) + o.count(buf[split * wb:], n - split, k)
            if not (parts == c).all():
                fails.append(f"k={k}: additivity at {split}")
        # (iv) permutation invariance
        perm = rng.permutation(n)
        shuffled = buf.reshape(n, wb)[perm].reshape(-1).copy()
        if not (o.count(shuffled, n, k) == c).all():
            fails.append(f"k={k}: permutation")
        # (v) complement: counts(~w)[p] = n - counts(w)[p]
        if not (o.count(~buf, n, k) == n - c).all():
            fails.append(f"k={k}: complement")
        # (vi) rotating every word by s bits rotates the counts by s
        words = buf.view({8: np.uint8, 16: np.uint16, 32: np.uint32}[k]).astype(np.uint64)
        for s in (1, 5, k - 1):
            rot = ((words << np.uint64(s)) | (words >> np.uint64(k - s))) & np.uint64(2**k - 1)
            rb = rot.astype({8: np.uint8, 16: np.uint16, 32: np.uint32}[k]).view(np.uint8)
            if not (o.count(rb, n, k) == np.roll(c, s)).all():
                fails.append(f"k={k}: rotation by {s}")
        # (ii) one-hot words sum to n
        oh = I.generate(n * wb, I.Dist.onehot(k, 1.1), 200 + k)
        if int(o.count(oh, n, k).sum()) != n:
            fails.append(f"k={k}: one-hot sum != n")
        # (viii) alignment: any start offset equals an aligned copy of the same bytes
        big = rand_bytes(n * wb + 16, 300 + k)
        for off in range(1, 16):
            if not (o.count(big, n, k, offset=off) ==
                    o.count(big[off:off + n * wb].copy(), n, k)).all():
                fails.append(f"k={k}: offset {off}")
                break
    # (vii) one byte buffer seen as u8, u16 and u32 words
    L = 4 * 4099
    buf = rand_bytes(L, 77)
    c8, c16, c32 = (o.count(buf, L * 8 // k, k) for k in KS)
    if not all(int(c8[b]) == int(c16[b::8].sum()) == int(c32[b::8].sum()) for b in range(8)):
        fails.append("u8/u16/u32 byte-position folding")
    if not (c16 == c32[:16] + c32[16:]).all():
        fails.append("u16 = u32 halves folded")
    return fails


def pin_accumulate(o):
    buf = rand_bytes(4096, 5)
    seeded = np.arange(16, dtype=np.uint64) * 1000
    got = o.count(buf, 2048, 16, counts=seeded.copy())
    if not (got == seeded + brute(buf, 2048, 16)).all():
        return ["counts must be accumulated into, not overwritten"]
    return []


def pin_threads(o):
    fails = []
    buf = rand_bytes(3 * 100003, 9)
    for k in KS:
        n = 3 * 100003 // (k // 8)
        ref = brute(buf, n, k)
        for t in (2, 3, 8, 64):
            if not (o.count(buf, n, k, threads=t) == ref).all():
                fails.append(f"k={k} threads={t}")
        tiny = o.count(buf, 3, k, threads=8)
        if not (tiny == brute(buf, 3, k)).all():
            fails.append(f"k={k}: fewer words than threads")
    return fails


def pin_harley_seal_model(o):
    fails = []
    for N, calls in ((2, 3), (3, 7), (4, 15)):  # Sec. 4.1: 3, 7, 15 CSA calls per block
        n = (1 << N) * 32
        buf = rand_bytes(2 * n, 40 + N)
        c, got_calls = o.hs16(buf, n, N)
        if got_calls != calls:
            fails.append(f"N={N}: {got_calls} CSA calls, paper says {calls}")
        if not (c == brute(buf, n, 16)).all():
            fails.append(f"N={N}: one block")
    for N in range(1, 7):  # 2^N - 1 CSAs per 2^N registers (Sec. 2), any size
        block_words = (1 << N) * 32
        for blocks, resid in ((0, 5), (3, 0), (5, 77 % block_words)):
            n = blocks * block_words + resid
            buf = rand_bytes(2 * n + 2, 50 + N + blocks)
            c, got_calls = o.hs16(buf, n, N)
            if got_calls != blocks * ((1 << N) - 1):
                fails.append(f"N={N}: CSA count")
            if not (c == brute(buf, n, 16)).all():
                fails.append(f"N={N} blocks={blocks} residual={resid}")
    ones = np.full(2 * 16 * 32 * 3, 255, np.uint8)  # every carry register all ones
    c, _ = o.hs16(ones, 16 * 32 * 3, 4)
    if not (c == 16 * 32 * 3).all():
        fails.append("all-ones through the 1 kB circuit")
    return fails


PINS = [pin_country_example, pin_csa_truth_tables, pin_csa_identity, pin_closed_forms,
        pin_brute_force, pin_invariants, pin_accumulate, pin_threads, pin_harley_seal_model]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(orc, pin):
    fails = pin(orc)
    assert not fails, fails


def test_country_reading_is_msb_first(orc):
    """The bit-level vector under the adopted reading of Table 1 (leftmost = bit 7)."""
    stream = np.array([0x10, 0x10, 0x04, 0x10, 0x01, 0x04, 0x01, 0x01, 0x01, 0x20], np.uint8)
    assert orc.count(stream, 10, 8).tolist() == [4, 0, 2, 0, 3, 1, 0, 0]


def test_bad_width_rejected(orc):
    with pytest.raises(ValueError):
        orc.count(np.zeros(8, np.uint8), 1, 12)


def test_statistics_of_inputs(orc):
    """Not parity: the generators produce the densities they are asked for (5 sigma)."""
    n = 1 << 20
    for p in (0.02, 0.5, 0.9):
        c = orc.count(I.generate(n * 2, I.Dist.bernoulli(p), 3), n, 16)
        sigma = np.sqrt(n * p * (1 - p))
        assert (np.abs(c.astype(np.float64) - n * p) < 5 * sigma).all()
    cdf = I.zipf_cdf(16, 1.1).astype(np.float64)
    probs = np.diff(cdf) / 2**32
    c = orc.count(I.generate(n * 2, I.Dist.onehot(16, 1.1), 4), n, 16)
    assert (np.abs(c - n * probs) < 5 * np.sqrt(n * probs * (1 - probs))).all()


PLANTS = {
    1: "words assembled big-endian",
    2: "last word dropped",
    3: "bit index off by one",
    4: "counters overwritten instead of accumulated",
    5: "a word lost at each thread split",
    6: "CSA carry term dropped",
    7: "carry weight 2^(N-1) instead of 2^N",
}


@pytest.mark.parametrize("plant", sorted(PLANTS), ids=lambda p: PLANTS[p].replace(" ", "_"))
def test_planted_mistakes_are_caught(tmp_path, plant):
    lib = obuild.build(plant=plant, out=str(tmp_path / f"libplant{plant}.so"))
    o = oracle.Oracle(lib)
    caught = [p.__name__ for p in PINS if p(o)]
    assert caught, f"planted mistake '{PLANTS[plant]}' passed every pin"


# ------------------------------------------------------- histogram of categorical ids

def pin_histogram(o):
    """The id histogram equals encode-then-count (one-hot words through the plain
    definition), numpy's bincount, and the Table 1 example as category ids."""
    fails = []
    rng = np.random.Generator(np.random.PCG64(21))
    for id_bytes in (1, 2):
        for bins in (1, 5, 8, 16, 32, 64):
            n = 3001
            ids = rng.integers(0, min(256 ** id_bytes, bins + 9), size=n).astype(
                np.uint8 if id_bytes == 1 else np.uint16)
            h = o.histogram(ids.view(np.uint8), n, id_bytes, bins)
            ref = np.bincount(ids.astype(np.int64), minlength=bins + 9)
            if not ((h[:bins] == ref[:bins]).all() and h[bins] == ref[bins:].sum()):
                fails.append(f"bincount id_bytes={id_bytes} bins={bins}")
            k = 8 if bins <= 8 else 16 if bins <= 16 else 32 if bins <= 32 else 64
            wt = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}[k]
            valid = ids.astype(np.int64) < bins
            words = np.where(valid, np.left_shift(np.uint64(1), ids.astype(np.uint64)
                                                   % np.uint64(64)), np.uint64(0)).astype(wt)
            enc = o.count(words.view(np.uint8), n, k)
            if not ((h[:bins] == enc[:bins]).all() and h[bins] == n - int(valid.sum())):
                fails.append(f"encode-then-count id_bytes={id_bytes} bins={bins}")
    rows = _golden("country_example.txt")
    mapping = {r[1]: int(r[2], 2).bit_length() - 1 for r in rows if r[0] == "mapping"}
    stream = next(r[1:] for r in rows if r[0] == "stream")
    hist = {r[1]: int(r[2]) for r in rows if r[0] == "histogram"}
    ids = np.array([mapping[c] for c in stream], np.uint8)
    h = o.histogram(ids, len(ids), 1, 8)
    for name, expect in hist.items():
        if int(h[mapping[name]]) != expect:
            fails.append(f"country {name}")
    edge = np.array([7, 8, 9, 0], np.uint8)  # bins = 8: ids 8 and 9 have no code
    if o.histogram(edge, 4, 1, 8).tolist() != [1, 0, 0, 0, 0, 0, 0, 1, 2]:
        fails.append("ids at and past the bin count")
    return fails


def test_histogram_pin(orc):
    fails = pin_histogram(orc)
    assert not fails, fails


def test_planted_histogram_boundary_is_caught(tmp_path):
    o = oracle.Oracle(obuild.build(plant=8, out=str(tmp_path / "libplant8.so")))
    assert pin_histogram(o)


# ------------------------------------------ wider words as 16-bit planes (Sec. 4)

def pin_planes(o):
    """Words of 16*m bits held as m planes of 16-bit limbs count like the words
    themselves: against the plain definition for k = 16, 32, 64 (the interleaved
    words through count), and brute force on the assembled bits for m = 3, 5 and 64."""
    fails = []
    rng = np.random.Generator(np.random.PCG64(31))
    for m in (1, 2, 4):
        k = 16 * m
        for n in (0, 1, 5, 1000):
            words = rng.integers(0, 256, size=n * 2 * m, dtype=np.uint8)
            limbs = words.view(np.uint16).reshape(n, m)
            planes = [np.ascontiguousarray(limbs[:, j]) for j in range(m)]
            if not (o.count_planes(planes, n) == o.count(words, n, k)).all():
                fails.append(f"planes m={m} n={n} vs k={k} words")
    for m, n in ((3, 777), (5, 300), (64, 20)):
        limbs = rng.integers(0, 1 << 16, size=(n, m), dtype=np.uint16)
        # planes at odd byte offsets inside larger buffers
        bufs, offs = [], []
        for j in range(m):
            b = np.zeros(2 * n + 3, np.uint8)
            b[1:1 + 2 * n] = np.ascontiguousarray(limbs[:, j]).view(np.uint8)
            bufs.append(b)
            offs.append(1)
        bits = np.unpackbits(np.ascontiguousarray(limbs).view(np.uint8).reshape(n, 2 * m),
                             axis=1, bitorder="little")
        if not (o.count_planes(bufs, n, offsets=offs) == bits.sum(axis=0)).all():
            fails.append(f"planes m={m} brute force")
    return fails


def test_planes_pin(orc):
    fails = pin_planes(orc)
    assert not fails, fails


def test_planted_plane_order_is_caught(tmp_path):
    o = oracle.Oracle(obuild.build(plant=9, out=str(tmp_path / "libplant9.so")))
    assert pin_planes(o)
